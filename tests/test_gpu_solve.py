"""End-to-end parity of the GPU path against the oracle, through the C ABI:
exact ground value, exact degeneracy, and a configuration that reaches the
value."""
import os

import numpy as np
import pytest

import instances as I
from oracle import brute, config, tm

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = []
    for line in open(os.path.join(GOLDEN, name)):
        if line.startswith("#") or not line.strip():
            continue
        rows.append([int(x) for x in line.split()])
    return rows


@pytest.fixture(scope="module")
def B():
    from tests.gpu_util import torch_cuda
    torch_cuda()
    import paper_2602_05470_amd as B
    return B


def _check_sg(r, g, want):
    assert (r.value, r.count) == tuple(want)
    assert r.certified
    assert set(np.unique(r.config)) <= {-1, 1}
    assert config.spin_glass_energy(r.config, g["edges"], g["J"], g.get("h")) == r.value


@pytest.mark.parametrize("seed", range(20))
def test_sg4_plain_contraction_vs_brute_force(B, seed):
    """4x4 +-J lattice, whole-network contraction, no branching."""
    g = I.spin_glass_square(4, seed)
    e0, deg, _ = brute.spin_glass(g["n"], g["edges"], g["J"])
    with B.Context(B.Options(branching=0, residues_per_pass=3)) as ctx:
        r = ctx.solve_spinglass(g["n"], g["edges"], g["J"])
    _check_sg(r, g, (e0, deg))
    assert deg % 2 == 0


@pytest.mark.parametrize("seed", range(20))
def test_sg16_bbtn_vs_transfer_matrix(B, seed):
    """16x16 +-J lattice, BBTN with T_target = 2^10, 3 residues per pass."""
    want = {s: (e, d) for s, e, d in _golden("sg16.txt")}[seed]
    g = I.spin_glass_square(16, seed)
    with B.Context(B.Options(log2_target=10, residues_per_pass=3)) as ctx:
        r = ctx.solve_spinglass(g["n"], g["edges"], g["J"])
    _check_sg(r, g, want)
    assert r.leaves >= 1


def test_sg16_unbatched_equals_batched(B):
    g = I.spin_glass_square(16, 3)
    want = {s: (e, d) for s, e, d in _golden("sg16.txt")}[3]
    with B.Context(B.Options(log2_target=10, batched=0)) as ctx:
        r = ctx.solve_spinglass(g["n"], g["edges"], g["J"])
    _check_sg(r, g, want)


@pytest.mark.parametrize("t", [6, 8, 12, 18])
def test_plan_independence_over_targets(B, t):
    g = I.spin_glass_square(12, 1)
    want = tm.spin_glass_square(g)
    with B.Context(B.Options(log2_target=t, residues_per_pass=2)) as ctx:
        r = ctx.solve_spinglass(g["n"], g["edges"], g["J"])
    _check_sg(r, g, want)


def test_field_and_rect(B):
    g = I.spin_glass_rect(6, 9, 4)
    h = np.random.default_rng(4).integers(-2, 3, size=g["n"]).astype(np.int32)
    g["h"] = h
    want = tm.spin_glass_lattice(6, 9, g["edges"], g["J"], h)
    with B.Context(B.Options(log2_target=5)) as ctx:
        r = ctx.solve_spinglass(g["n"], g["edges"], g["J"], h)
    _check_sg(r, g, want)


@pytest.mark.parametrize("seed", range(5))
def test_ksg16_vs_transfer_matrix(B, seed):
    s, n, w, c = _golden("ksg16.txt")[seed]
    g = I.kings_subgraph(16, seed)
    assert g["n"] == n
    with B.Context(B.Options(log2_target=10)) as ctx:
        r = ctx.solve_mwis(g["n"], g["edges"], g["w"])
    assert (r.value, r.count) == (w, c) and r.certified
    assert config.independent_set_weight(r.config, g["edges"], g["w"]) == w


def test_weighted_ksg(B):
    g = I.kings_subgraph(7, 2, weights="1..10")
    want = tm.kings_subgraph(g)
    with B.Context(B.Options(log2_target=4)) as ctx:
        r = ctx.solve_mwis(g["n"], g["edges"], g["w"])
    assert (r.value, r.count) == want
    assert config.independent_set_weight(r.config, g["edges"], g["w"]) == want[0]


def test_closed_forms(B):
    with B.Context(B.Options(branching=0)) as ctx:
        g = I.spin_glass_square(4, 0)
        r = ctx.solve_spinglass(g["n"], g["edges"], np.ones(len(g["J"]), np.int32))
        assert (r.value, r.count) == (-24, 2)
        r = ctx.solve_spinglass(4, [(0, 1), (1, 3), (3, 2), (2, 0)], [1, 1, 1, -1])
        assert (r.value, r.count) == (-2, 8)
        r = ctx.solve_mwis(6, np.zeros((0, 2), np.int32))
        assert (r.value, r.count) == (6, 1)
        kn = [(i, j) for i in range(7) for j in range(i + 1, 7)]
        r = ctx.solve_mwis(7, kn)
        assert (r.value, r.count) == (1, 7)
        g = I.full_kings_graph(5)
        r = ctx.solve_mwis(g["n"], g["edges"])
        assert (r.value, r.count) == (9, 1)


def test_invalid_arguments(B):
    with B.Context(B.Options()) as ctx:
        with pytest.raises(B.BBTNError) as e:
            ctx.solve_spinglass(3, [(0, 3)], [1])
        assert e.value.status == -1
        with pytest.raises(B.BBTNError):
            ctx.solve_spinglass(3, [(1, 1)], [1])
        with pytest.raises(B.BBTNError):
            ctx.solve_mwis(3, [(0, 1)], [1, 0, 1])


@pytest.mark.parametrize("seed", [0, 7])
def test_per_branch_graph_replay_equals_eager(B, seed):
    """One branch at a time: with graphs the step program of the group is
    captured once and replayed for every branch (inputs refreshed eagerly,
    stream synchronised between replays); every replay feeds the count."""
    g = I.spin_glass_square(16, seed)
    want = {s: (e, d) for s, e, d in _golden("sg16.txt")}[seed]
    res = {}
    for graphs in (0, 1):
        with B.Context(B.Options(log2_target=10, batched=0, graphs=graphs)) as ctx:
            r = ctx.solve_spinglass(g["n"], g["edges"], g["J"])
        _check_sg(r, g, want)
        res[graphs] = (r.value, r.count, r.leaves, bytes(r.config))
    assert res[0] == res[1]


@pytest.mark.parametrize("seed", range(5))
def test_sg20_bbtn_vs_c_transfer_matrix(B, seed):
    """20x20 +-J (65536 branches at T_target = 2^12), counts past 2^57."""
    want = {s: (e, d) for s, e, d in _golden("sg20.txt")}[seed]
    g = I.spin_glass_square(20, seed)
    with B.Context(B.Options(log2_target=12, residues_per_pass=3)) as ctx:
        r = ctx.solve_spinglass(g["n"], g["edges"], g["J"])
    _check_sg(r, g, want)


@pytest.mark.parametrize("seed", range(5))
def test_ksg20_bbtn_vs_c_transfer_matrix(B, seed):
    s, n, w, c = _golden("ksg20.txt")[seed]
    g = I.kings_subgraph(20, seed)
    assert g["n"] == n
    with B.Context(B.Options(log2_target=12, residues_per_pass=4)) as ctx:
        r = ctx.solve_mwis(g["n"], g["edges"], g["w"])
    assert (r.value, r.count) == (w, c) and r.certified
    assert config.independent_set_weight(r.config, g["edges"], g["w"]) == w


@pytest.mark.parametrize("seed", range(2))
def test_sg24_large_leaves_four_residues(B, seed):
    """24x24 at T_target = 2^16: branch tensors too large for LDS go through
    the step-by-step batched executor; 4 residues per pass."""
    want = {s: (e, d) for s, e, d in _golden("sg24.txt")}[seed]
    g = I.spin_glass_square(24, seed)
    with B.Context(B.Options(log2_target=16, residues_per_pass=4)) as ctx:
        r = ctx.solve_spinglass(g["n"], g["edges"], g["J"])
    _check_sg(r, g, want)


def test_one_context_many_instances(B):
    """One context solving different couplings on repeated topologies (the
    contraction-tree cache) and switching between problem kinds."""
    sg = {s: (e, d) for s, e, d in _golden("sg16.txt")}
    ksg = {s: (w, c) for s, _, w, c in _golden("ksg16.txt")}
    with B.Context(B.Options(log2_target=10)) as ctx:
        for seed in (0, 1, 2):
            g = I.spin_glass_square(16, seed)
            _check_sg(ctx.solve_spinglass(g["n"], g["edges"], g["J"]), g, sg[seed])
            k = I.kings_subgraph(16, seed)
            r = ctx.solve_mwis(k["n"], k["edges"], k["w"])
            assert (r.value, r.count) == ksg[seed] and r.certified
        g = I.spin_glass_square(16, 5)
        _check_sg(ctx.solve_spinglass(g["n"], g["edges"], g["J"]), g, sg[5])


def test_device_mem_cap(B):
    """device_mem_cap: a cap below what a solve needs fails with OOM (no
    allocation past it); a cap that only limits the branch chunks still
    gives the exact result, through more, smaller chunks."""
    sg = {s: (e, d) for s, e, d in _golden("sg24.txt")}
    g = I.spin_glass_square(16, 0)
    with B.Context(B.Options(log2_target=10, device_mem_cap=2 << 20)) as ctx:
        with pytest.raises(B.BBTNError) as ei:
            ctx.solve_spinglass(g["n"], g["edges"], g["J"])
        assert ei.value.status == -2
    g = I.spin_glass_square(24, 1)
    with B.Context(B.Options(log2_target=16, residues_per_pass=4,
                             device_mem_cap=1 << 30)) as ctx:
        r = ctx.solve_spinglass(g["n"], g["edges"], g["J"])
    _check_sg(r, g, sg[1])
