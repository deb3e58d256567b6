"""Parity of the GPU path with a refined contraction order (annealed
rotations of the greedy tree, chosen by a probe search): exact ground value,
exact degeneracy and a configuration reaching it, against the exact transfer
matrix ("Tropical Tensor Networks": any contraction order gives the same
tropical contraction; only its cost changes)."""
import os

import numpy as np
import pytest

import instances as I
from oracle import config

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
    assert config.spin_glass_energy(r.config, g["edges"], g["J"], g.get("h")) == r.value


def test_sg16_refined_order_batch(B):
    """Twenty 16x16 instances in one call with order_refine = 8: the order
    is chosen once for the lattice and every instance is exact."""
    want = {s: (e, d) for s, e, d in _golden("sg16.txt")}
    gs = [I.spin_glass_square(16, s) for s in range(20)]
    with B.Context(B.Options(log2_target=10, order_refine=8)) as ctx:
        rs, st = ctx.solve_batch(0, [(g["n"], g["edges"], g["J"], None) for g in gs])
    assert all(s == 0 for s in st)
    for s, (g, r) in enumerate(zip(gs, rs)):
        _check_sg(r, g, want[s])
        assert r.leaves <= 1024


@pytest.mark.parametrize("seed", range(2))
def test_sg24_refined_order(B, seed):
    """24x24 at T_target = 2^16 with the refined order (about 1,000 leaves
    instead of the greedy order's 2^18)."""
    want = {s: (e, d) for s, e, d in _golden("sg24.txt")}[seed]
    g = I.spin_glass_square(24, seed)
    with B.Context(B.Options(log2_target=16, order_refine=8)) as ctx:
        r = ctx.solve_spinglass(g["n"], g["edges"], g["J"])
    _check_sg(r, g, want)


@pytest.mark.parametrize("seed", range(2))
def test_sg32x24_refined_order(B, seed):
    """32 x 24 lattice at T_target = 2^20: branch tensors of up to 2^20
    entries, contracted step by step in memory-sized chunks of branches."""
    want = {s: (e, d) for s, e, d in _golden("sg32x24.txt")}[seed]
    g = I.spin_glass_rect(32, 24, seed)
    with B.Context(B.Options(log2_target=20, order_refine=8)) as ctx:
        r = ctx.solve_spinglass(g["n"], g["edges"], g["J"])
    _check_sg(r, g, want)


@pytest.mark.parametrize("seed", range(3))
def test_ksg20_refined_order(B, seed):
    """Unweighted MIS on King's subgraphs 20x20 (vertex tensors, a different
    network shape) at T_target = 2^10 with the refined order, 4 residues."""
    s, n, w, c = _golden("ksg20.txt")[seed]
    g = I.kings_subgraph(20, seed)
    assert g["n"] == n
    with B.Context(B.Options(log2_target=10, residues_per_pass=4, order_refine=8)) as ctx:
        r = ctx.solve_mwis(g["n"], g["edges"], g["w"])
    assert (r.value, r.count) == (w, c) and r.certified
    assert config.independent_set_weight(r.config, g["edges"], g["w"]) == w


@pytest.mark.parametrize("seed", range(3))
def test_sg20_refined_order_values_only(B, seed):
    """Values-only mode (no counts) on 20x20 with the refined order: the
    ground energy and a configuration reaching it."""
    s, e0, _ = _golden("sg20.txt")[seed]
    g = I.spin_glass_square(20, seed)
    with B.Context(B.Options(log2_target=12, residues_per_pass=0, order_refine=8)) as ctx:
        r = ctx.solve_spinglass(g["n"], g["edges"], g["J"])
    assert r.value == e0
    assert config.spin_glass_energy(r.config, g["edges"], g["J"], None) == e0


def test_field_and_weights_refined_order(B):
    """A field on a rectangle and integer weights 1..10 on a King's subgraph
    (both break the symmetries of the zero-field unit cases), refined order,
    against the transfer matrix."""
    from oracle import tm
    g = I.spin_glass_rect(10, 12, 7)
    h = np.random.default_rng(7).integers(-2, 3, size=g["n"]).astype(np.int32)
    want = tm.spin_glass_lattice(10, 12, g["edges"], g["J"], h)
    with B.Context(B.Options(log2_target=6, order_refine=8)) as ctx:
        r = ctx.solve_spinglass(g["n"], g["edges"], g["J"], h)
    assert (r.value, r.count) == tuple(want) and r.certified
    assert config.spin_glass_energy(r.config, g["edges"], g["J"], h) == r.value
    k = I.kings_subgraph(10, 3, weights="1..10")
    want = tm.kings_subgraph(k)
    with B.Context(B.Options(log2_target=6, order_refine=8)) as ctx:
        r = ctx.solve_mwis(k["n"], k["edges"], k["w"])
    assert (r.value, r.count) == tuple(want) and r.certified
    assert config.independent_set_weight(r.config, k["edges"], k["w"]) == want[0]


def test_measured_order_candidates(B):
    """bbtn_order_candidates / bbtn_order_use: every ranked candidate order of
    the 24 x 24 lattice, installed for the structure, gives the same exact
    ground energy and degeneracy (both seeds, against the transfer matrix);
    a candidate index out of range, or a structure without candidates, is an
    argument error."""
    want = {s: (e, d) for s, e, d in _golden("sg24.txt")}
    gs = [I.spin_glass_square(24, s) for s in range(2)]
    with B.Context(B.Options(log2_target=16, order_refine=4)) as ctx:
        n = ctx.order_candidates(0, gs[0]["n"], gs[0]["edges"], gs[0]["J"])
        assert 1 <= n <= 2 * 4 + 3
        # the same structure: the list is built once
        assert ctx.order_candidates(0, gs[1]["n"], gs[1]["edges"], gs[1]["J"]) == n
        for i in range(min(n, 3)):
            ctx.order_use(0, gs[0]["n"], gs[0]["edges"], gs[0]["J"], which=i)
            for s, g in enumerate(gs):
                _check_sg(ctx.solve_spinglass(g["n"], g["edges"], g["J"]), g, want[s])
        with pytest.raises(B.BBTNError):
            ctx.order_use(0, gs[0]["n"], gs[0]["edges"], gs[0]["J"], which=n)
        other = I.spin_glass_square(20, 0)
        with pytest.raises(B.BBTNError):
            ctx.order_use(0, other["n"], other["edges"], other["J"], which=0)
