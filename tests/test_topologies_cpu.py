"""Other spin-glass topologies (random 3-regular graphs, open cubic
lattices): the variable-elimination oracle pinned to brute force on small
instances, and the planner's leaves checked against brute force (disjoint,
every optimal configuration in exactly one leaf).  Host only."""
import itertools

import numpy as np
import pytest

import instances as I
from oracle import brute, ve


def _all_states(n):
    return np.array(list(itertools.product([0, 1], repeat=n)), dtype=np.int8)[:, ::-1]


def _energy(states, edges, J):
    s = 2 * states.astype(np.int64) - 1
    e = np.zeros(len(states), np.int64)
    for (a, b), j in zip(edges, J):
        e -= j * s[:, a] * s[:, b]
    return e


def _instances():
    out = [("rr16", I.spin_glass_random_regular(16, s)) for s in range(3)]
    out += [("rr18", I.spin_glass_random_regular(18, s)) for s in range(2)]
    out += [("cube223", I.spin_glass_cubic(2, 2, 3, s)) for s in range(2)]
    out += [("cube233", I.spin_glass_cubic(2, 3, 3, s)) for s in range(2)]
    return out


def test_generators_are_regular_and_simple():
    for n in (16, 40, 80):
        g = I.spin_glass_random_regular(n, 3)
        e = g["edges"]
        assert len(e) == 3 * n // 2
        assert (e[:, 0] < e[:, 1]).all()
        assert len({tuple(x) for x in e.tolist()}) == len(e)
        assert (np.bincount(e.ravel(), minlength=n) == 3).all()
    g = I.spin_glass_cubic(3, 4, 5, 0)
    assert g["n"] == 60 and len(g["edges"]) == 2 * 4 * 5 + 3 * 3 * 5 + 3 * 4 * 4


@pytest.mark.parametrize("name,g", _instances())
def test_ve_matches_brute_force(name, g):
    e0, deg, _ = brute.spin_glass(g["n"], g["edges"], g["J"])
    assert ve.spin_glass(g["n"], g["edges"], g["J"])[:2] == (e0, deg)


@pytest.fixture(scope="module")
def B():
    import paper_2602_05470_amd as B
    B.load()
    return B


@pytest.mark.parametrize("name,g", _instances())
@pytest.mark.parametrize("t", [1, 3])
def test_leaves_complete_and_disjoint(B, name, g, t):
    n, edges, J = g["n"], np.asarray(g["edges"]), np.asarray(g["J"])
    leaves, _ = B.plan_leaves(0, n, edges, J, None, log2_target=t, region_max=6)
    states = _all_states(n)
    fixed = leaves >= 0
    mem = ((states[:, None, :] == leaves[None, :, :]) | ~fixed[None, :, :]).all(axis=2)
    assert (mem.sum(axis=1) <= 1).all()
    e = _energy(states, edges, J)
    opt = e == e.min()
    assert (mem[opt].sum(axis=1) == 1).all()
