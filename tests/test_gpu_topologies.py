"""GPU path on other spin-glass topologies (random 3-regular graphs, open
cubic lattices) against the variable-elimination oracle: exact ground
energy, exact degeneracy, a configuration reaching it, with branching
forced by a small T_target, one call per instance and all in one batch."""
import numpy as np
import pytest

import instances as I
from oracle import config, ve

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from tests.gpu_util import torch_cuda
    torch_cuda()
    import paper_2602_05470_amd as B
    return B


def _cases():
    out = [I.spin_glass_random_regular(n, s) for n in (40, 60, 80) for s in range(2)]
    out += [I.spin_glass_cubic(3, 3, 4, s) for s in range(2)]
    out += [I.spin_glass_cubic(4, 4, 4, 0)]
    return out


def _check(r, g, want):
    assert (r.value, r.count) == want
    assert r.certified
    assert config.spin_glass_energy(r.config, g["edges"], g["J"]) == r.value


@pytest.mark.parametrize("t", [6, 8])
def test_one_call_each(B, t):
    with B.Context(B.Options(log2_target=t, residues_per_pass=3)) as ctx:
        for g in _cases():
            want = ve.spin_glass(g["n"], g["edges"], g["J"])[:2]
            r = ctx.solve_spinglass(g["n"], g["edges"], g["J"])
            if t == 6:
                assert r.leaves > 1  # every case branches at this T_target
            _check(r, g, want)


def test_one_batch(B):
    gs = _cases()
    want = [ve.spin_glass(g["n"], g["edges"], g["J"])[:2] for g in gs]
    with B.Context(B.Options(log2_target=7, residues_per_pass=3)) as ctx:
        rs, st = ctx.solve_batch(0, [(g["n"], g["edges"], g["J"], None) for g in gs])
    assert st == [0] * len(gs)
    for r, g, w in zip(rs, gs, want):
        _check(r, g, w)
