"""The spin-flip option (one spin of a zero-field spin glass fixed to +1, the
count doubled) against the oracle through the C ABI: the same ground energy
and degeneracy as brute force, the transfer matrix and the solve without the
option, and a configuration that reaches the energy.  The zero-field
degeneracy is even by construction here, so the evenness pin of the other
tests (the spin-flip symmetry itself) is checked with the option off."""
import os

import numpy as np
import pytest

import instances as I
from oracle import brute, config

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    out = {}
    for line in open(os.path.join(GOLDEN, name)):
        if line.startswith("#") or not line.strip():
            continue
        row = [int(x) for x in line.split()]
        out[row[0]] = row[1:]
    return out


@pytest.fixture(scope="module")
def B():
    from tests.gpu_util import torch_cuda
    torch_cuda()
    import paper_2602_05470_amd as B
    return B


def _check(r, edges, J, h, want):
    assert (r.value, r.count) == tuple(want)
    assert r.certified
    assert set(np.unique(r.config)) <= {-1, 1}
    assert config.spin_glass_energy(r.config, edges, J, h) == r.value


@pytest.mark.parametrize("seed", range(6))
def test_sg4_spin_flip_vs_brute_force(B, seed):
    g = I.spin_glass_square(4, seed)
    e0, deg, _ = brute.spin_glass(g["n"], g["edges"], g["J"])
    for branching, t in ((0, 0), (1, 2)):
        with B.Context(B.Options(branching=branching, log2_target=t, region_max=3,
                                 spin_flip=1)) as ctx:
            r = ctx.solve_spinglass(g["n"], g["edges"], g["J"])
        _check(r, g["edges"], g["J"], None, (e0, deg))


@pytest.mark.parametrize("seed", range(4))
def test_sg16_spin_flip_vs_transfer_matrix(B, seed):
    want = _golden("sg16.txt")[seed]
    g = I.spin_glass_square(16, seed)
    with B.Context(B.Options(log2_target=10, residues_per_pass=3, spin_flip=1)) as ctx:
        r = ctx.solve_spinglass(g["n"], g["edges"], g["J"])
    _check(r, g["edges"], g["J"], None, want)


def test_sg20_spin_flip_batch_vs_transfer_matrix(B):
    """Several 20x20 instances in one call (shared launches), T_target 2^12."""
    want = _golden("sg20.txt")
    gs = [I.spin_glass_square(20, s) for s in range(3)]
    with B.Context(B.Options(log2_target=12, residues_per_pass=3, spin_flip=1)) as ctx:
        rs, st = ctx.solve_batch(0, [(g["n"], g["edges"], g["J"], None) for g in gs])
    for s, (g, r) in enumerate(zip(gs, rs)):
        _check(r, g["edges"], g["J"], None, want[s])


def test_spin_flip_on_irregular_graphs(B):
    """Random graphs with duplicate edges (including couplings that cancel
    on the fixed spin's edges), isolated spins, and a field (option
    ignored), against brute force."""
    rng = np.random.default_rng(7)
    for trial in range(12):
        n = int(rng.integers(3, 13))
        m = int(rng.integers(1, 2 * n))
        edges = []
        while len(edges) < m:
            a, b = (int(x) for x in rng.integers(0, n, 2))
            if a != b:
                edges.append((a, b))
        J = [int(x) for x in rng.choice([-2, -1, 1, 2], size=m)]
        if trial % 4 == 0:
            # a coupling and its negative on the same pair: they cancel
            a, b = edges[0]
            edges.append((b, a))
            J.append(-J[0])
        h = [int(x) for x in rng.integers(-1, 2, size=n)] if trial % 3 == 2 else None
        e0, deg, _ = brute.spin_glass(n, edges, J, h)
        with B.Context(B.Options(log2_target=2, region_max=3, spin_flip=1)) as ctx:
            r = ctx.solve_spinglass(n, edges, J, h)
        _check(r, edges, J, h, (e0, deg))


def test_sg32_spin_flip_agrees(B):
    """32x32 seed 0 with the refined order: the same (E0, degeneracy) with and
    without the option, E0 equal to the matching oracle's, half the MACs."""
    g = I.spin_glass_square(32, 0)
    out = []
    for flip in (0, 1):
        with B.Context(B.Options(log2_target=26, order_refine=8, residues_per_pass=3,
                                 spin_flip=flip, time_limit_s=200)) as ctx:
            r = ctx.solve_spinglass(g["n"], g["edges"], g["J"])
        assert r.certified
        assert config.spin_glass_energy(r.config, g["edges"], g["J"], None) == r.value
        out.append((r.value, r.count, r.macs))
    (v0, c0, m0), (v1, c1, m1) = out
    assert (v0, c0) == (v1, c1)
    assert v0 == _golden("sg32_values.txt")[0][0]
    assert c0 % 2 == 0                 # spin-flip symmetry, option off
    assert m1 < 0.75 * m0


def test_values_only_spin_flip(B):
    """Values-only solve (no count) with the option: the ground energy and a
    configuration reaching it."""
    want = _golden("sg16.txt")
    for seed in range(2):
        g = I.spin_glass_square(16, seed)
        with B.Context(B.Options(log2_target=10, residues_per_pass=0, spin_flip=1)) as ctx:
            r = ctx.solve_spinglass(g["n"], g["edges"], g["J"])
        assert r.value == want[seed][0]
        assert config.spin_glass_energy(r.config, g["edges"], g["J"], None) == r.value
