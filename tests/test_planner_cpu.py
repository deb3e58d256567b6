"""The planner's leaves against brute force (host only, no device): the
branches are disjoint, and every optimal configuration lies in exactly one
leaf ("Branch-and-Bound Tensor Network": complete and orthogonal branching;
boundary equivalence and pruning drop only strictly worse configurations)."""
import itertools

import numpy as np
import pytest

import instances as I
from oracle import brute


def _all_states(n):
    return np.array(list(itertools.product([0, 1], repeat=n)), dtype=np.int8)[:, ::-1]


def _membership(leaves, states):
    """[configurations, leaves] boolean: configuration agrees with every
    fixed state of the leaf."""
    fixed = leaves >= 0
    agree = (states[:, None, :] == leaves[None, :, :]) | ~fixed[None, :, :]
    return agree.all(axis=2)


def _sg_energy(states, edges, J, h=None):
    s = 2 * states.astype(np.int64) - 1
    e = np.zeros(len(states), np.int64)
    for (a, b), j in zip(edges, J):
        e -= j * s[:, a] * s[:, b]
    if h is not None:
        e -= (s * np.asarray(h, np.int64)).sum(axis=1)
    return e


@pytest.fixture(scope="module")
def B():
    import paper_2602_05470_amd as B
    B.load()
    return B


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("t,rmax", [(1, 3), (2, 4), (3, 8)])
@pytest.mark.parametrize("field", [False, True])
@pytest.mark.parametrize("refine", [-1, 0, 4])
def test_sg_leaves_complete_and_disjoint(B, seed, t, rmax, field, refine):
    """+-J on 4 x 4 (field 0.5 doubled to integers: J = +-2, h = 1), with the
    min-fill tree (refine -1), the greedy order and an annealed refinement of
    it."""
    g = I.spin_glass_square(4, seed)
    n, edges, J = g["n"], np.asarray(g["edges"]), np.asarray(g["J"])
    h = None
    if field:
        J, h = 2 * J, np.ones(n, np.int64)
    leaves, inc = B.plan_leaves(0, n, edges, J, h, log2_target=t, region_max=rmax,
                                order_refine=refine)
    states = _all_states(n)
    mem = _membership(leaves, states)
    assert (mem.sum(axis=1) <= 1).all()          # orthogonal
    e = _sg_energy(states, edges, J, h)
    e0, deg, _ = brute.spin_glass(n, edges, J, h)
    opt = e == e0
    assert opt.sum() == deg
    assert (mem[opt].sum(axis=1) == 1).all()     # every ground state, exactly once
    assert inc is None or inc >= e0


@pytest.mark.parametrize("seed", range(4))
def test_sg_values_only_keeps_an_optimum(B, seed):
    g = I.spin_glass_square(4, seed)
    n, edges, J = g["n"], np.asarray(g["edges"]), np.asarray(g["J"])
    leaves, inc = B.plan_leaves(0, n, edges, J, log2_target=2, region_max=4, values_only=True)
    states = _all_states(n)
    mem = _membership(leaves, states)
    assert (mem.sum(axis=1) <= 1).all()
    e = _sg_energy(states, edges, J)
    e0 = e.min()
    # an optimum survives in some leaf, or the incumbent already is one
    assert mem[e == e0].any() or inc == e0


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("refine", [-1, 0, 4])
def test_mwis_leaves_complete_and_disjoint(B, seed, refine):
    g = I.kings_subgraph(4, seed, weights="1..10")
    n, edges, w = g["n"], np.asarray(g["edges"]).reshape(-1, 2), np.asarray(g["w"])
    leaves, inc = B.plan_leaves(1, n, edges, w, log2_target=1, region_max=4, order_refine=refine)
    states = _all_states(n)
    mem = _membership(leaves, states)
    assert (mem.sum(axis=1) <= 1).all()
    indep = np.ones(len(states), bool)
    for a, b in edges:
        indep &= ~((states[:, a] == 1) & (states[:, b] == 1))
    weight = (states.astype(np.int64) * w).sum(axis=1)
    weight[~indep] = -1
    wmax, cnt = brute.mwis(n, edges, w)[:2]
    opt = weight == wmax
    assert opt.sum() == cnt
    assert (mem[opt].sum(axis=1) == 1).all()
