"""Contraction-order refinement (host only): annealed rotations of the greedy
tree keep every intermediate's variable set consistent (the library recounts
them and fails otherwise), and on square lattices the chosen order is far
cheaper than the greedy one ("Tropical Tensor Networks": time and space
complexity of a contraction order; Eq. 4 for the overflow measure)."""
import numpy as np
import pytest

import instances as I


@pytest.fixture(scope="module")
def B():
    import paper_2602_05470_amd as B
    B.load()
    return B


def _sg(L, seed=0):
    g = I.spin_glass_square(L, seed)
    return g["n"], np.asarray(g["edges"]), np.asarray(g["J"])


@pytest.mark.parametrize("L", [4, 8])
@pytest.mark.parametrize("refine", [0, 8])
def test_complexity_invariants(B, L, refine):
    """Time of a pairwise tree is at least its largest intermediate; the
    overflow measure is zero exactly when T_target covers the largest
    intermediate, and at least the largest overflow otherwise."""
    n, edges, J = _sg(L)
    t = L // 2 + 1
    tc, sc, rho = B.order_complexity(0, n, edges, J, order_refine=refine, log2_target=t)
    assert tc >= sc - 1e-9
    assert sc >= 2                      # an edge tensor joins two spins
    assert rho >= max(0, sc - t)
    assert (rho == 0) == (sc <= t)


@pytest.mark.parametrize("L,t", [(16, 10), (24, 16)])
def test_refined_order_is_cheaper_than_greedy(B, L, t):
    n, edges, J = _sg(L)
    tc0, sc0, _ = B.order_complexity(0, n, edges, J, order_refine=0, log2_target=t)
    tc1, sc1, _ = B.order_complexity(0, n, edges, J, order_refine=4, log2_target=t)
    assert sc1 <= sc0
    assert tc1 <= tc0 - 1.0, (tc0, tc1)


def test_refined_order_other_topologies(B):
    """The variable recount inside the refinement runs on every topology the
    builders make: random 3-regular graphs, cubic lattices and weighted King's
    subgraphs (MWIS, vertex tensors)."""
    g = I.spin_glass_random_regular(40, 3)
    B.order_complexity(0, g["n"], np.asarray(g["edges"]), np.asarray(g["J"]),
                       order_refine=3, log2_target=4)
    g = I.spin_glass_cubic(3, 3, 3, 1)
    B.order_complexity(0, g["n"], np.asarray(g["edges"]), np.asarray(g["J"]),
                       order_refine=3, log2_target=4)
    g = I.kings_subgraph(8, 2, weights="1..10")
    B.order_complexity(1, g["n"], np.asarray(g["edges"]).reshape(-1, 2), np.asarray(g["w"]),
                       order_refine=3, log2_target=4)


def test_order_refine_bounds(B):
    n, edges, J = _sg(4)
    with pytest.raises(B.BBTNError):
        B.order_complexity(0, n, edges, J, order_refine=65, log2_target=2)
    with pytest.raises(B.BBTNError):
        B.order_complexity(0, n, edges, J, order_refine=-2, log2_target=2)


def test_minfill_beats_greedy_on_kings_64(B):
    """On the 64 x 64 King's subgraph (seed 0) the greedy pairwise order has
    space complexity 2^98; the min-fill elimination tree stays far below it
    (2^61), which is what makes it a starting order worth refining there."""
    g = I.kings_subgraph(64, 0)
    args = (1, g["n"], np.asarray(g["edges"]).reshape(-1, 2), None)
    tc_g, sc_g, _ = B.order_complexity(*args, order_refine=0, log2_target=64)
    tc_m, sc_m, _ = B.order_complexity(*args, order_refine=-1, log2_target=64)
    assert sc_m < sc_g - 20 and tc_m < tc_g - 20


def test_order_choice_is_deterministic(B):
    """The refined order is chosen by probe searches that run on parallel
    threads in rounds of fixed node budgets: repeated choices for the same
    structure give the same tree (same complexity and the same leaves)."""
    g = I.kings_subgraph(14, 3)
    args = (1, g["n"], np.asarray(g["edges"]).reshape(-1, 2), None)
    runs = [B.order_complexity(*args, order_refine=8, log2_target=8) for _ in range(3)]
    assert runs[0] == runs[1] == runs[2]
    leaves = [B.plan_leaves(*args, log2_target=8, order_refine=8)[0] for _ in range(3)]
    assert all(np.array_equal(leaves[0], x) for x in leaves[1:])
    n, edges, J = _sg(16)
    runs = [B.order_complexity(0, n, edges, J, order_refine=8, log2_target=10) for _ in range(3)]
    assert runs[0] == runs[1] == runs[2]
