"""bbtn_solve_batch: several instances through shared launches give exactly
the single-instance results (values, counts, certified, configurations that
reach the value), also with mixed sizes, fields, King's subgraphs, the
values-only mode and a failing instance in the batch."""
import os

import numpy as np
import pytest

import instances as I
from oracle import config, tm_c

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    out = {}
    for line in open(os.path.join(GOLDEN, name)):
        if line.startswith("#") or not line.strip():
            continue
        row = [int(x) for x in line.split()]
        out[row[0]] = (row[-2], row[-1])
    return out


@pytest.fixture(scope="module")
def B():
    from tests.gpu_util import torch_cuda
    torch_cuda()
    import paper_2602_05470_amd as B
    return B


def test_sg16_twenty_seeds_in_one_call(B):
    want = _golden("sg16.txt")
    gs = [I.spin_glass_square(16, s) for s in range(20)]
    with B.Context(B.Options(log2_target=10, residues_per_pass=3)) as ctx:
        rs, st = ctx.solve_batch(0, [(g["n"], g["edges"], g["J"], None) for g in gs])
    assert st == [0] * 20
    for s, (g, r) in enumerate(zip(gs, rs)):
        assert (r.value, r.count) == want[s] and r.certified
        assert config.spin_glass_energy(r.config, g["edges"], g["J"]) == r.value


def test_mixed_sizes_and_fields(B):
    cases = [(5, 0), (9, 1), (12, 2), (7, 3)]
    insts, wants = [], []
    for L, s in cases:
        g = I.spin_glass_square(L, s)
        J2 = [2 * j for j in g["J"]]
        h = [1] * g["n"] if s % 2 else None
        insts.append((g["n"], g["edges"], J2, h))
        wants.append(tm_c.spin_glass_lattice(L, L, g["edges"], J2, h))
    with B.Context(B.Options(log2_target=5, residues_per_pass=2)) as ctx:
        rs, st = ctx.solve_batch(0, insts)
    assert st == [0] * len(cases)
    for (n, e, J2, h), r, w in zip(insts, rs, wants):
        assert (r.value, r.count) == w and r.certified
        assert config.spin_glass_energy(r.config, e, J2, h) == r.value


def test_ksg16_batch(B):
    want = _golden("ksg16.txt")
    gs = [I.kings_subgraph(16, s) for s in range(5)]
    with B.Context(B.Options(log2_target=10)) as ctx:
        rs, st = ctx.solve_batch(1, [(g["n"], g["edges"], g["w"], None) for g in gs])
    assert st == [0] * 5
    for s, (g, r) in enumerate(zip(gs, rs)):
        assert (r.value, r.count) == want[s] and r.certified
        assert config.independent_set_weight(r.config, g["edges"], g["w"]) == r.value


def test_batch_equals_single_calls(B):
    gs = [I.spin_glass_square(11, s) for s in range(4)]
    with B.Context(B.Options(log2_target=6)) as ctx:
        rs, _ = ctx.solve_batch(0, [(g["n"], g["edges"], g["J"], None) for g in gs])
        for g, r in zip(gs, rs):
            r1 = ctx.solve_spinglass(g["n"], g["edges"], g["J"])
            assert (r.value, r.count, r.primes, r.residues) == \
                (r1.value, r1.count, r1.primes, r1.residues)
            assert np.array_equal(r.config, r1.config)


def test_values_only_batch(B):
    want = _golden("sg16.txt")
    gs = [I.spin_glass_square(16, s) for s in range(6)]
    with B.Context(B.Options(log2_target=10, residues_per_pass=0)) as ctx:
        rs, st = ctx.solve_batch(0, [(g["n"], g["edges"], g["J"], None) for g in gs])
    assert st == [0] * 6
    for s, (g, r) in enumerate(zip(gs, rs)):
        assert r.value == want[s][0] and r.count == 0
        assert config.spin_glass_energy(r.config, g["edges"], g["J"]) == r.value


def test_failing_instance_reports_its_own_status(B):
    good = I.spin_glass_square(8, 1)
    bad = (10, [(0, 99)], [1], None)   # vertex id out of range
    with B.Context(B.Options(log2_target=4)) as ctx:
        rs, st = ctx.solve_batch(0, [bad, (good["n"], good["edges"], good["J"], None)],
                                 raise_failed=False)
        with pytest.raises(B.BBTNError):
            ctx.solve_batch(0, [bad])
    assert st[0] == -1 and st[1] == 0
    assert (rs[1].value, rs[1].count) == tm_c.spin_glass_lattice(8, 8, good["edges"], good["J"])


@pytest.mark.parametrize("L,t,branching", [(20, 12, 1), (12, 0, 0)])
def test_small_step_forest_matches_plain_launches(B, L, t, branching):
    """Programs too large for the persistent executor run their small
    once-per-pass steps as subtree tasks of one persistent launch
    (batched = 1): the same exact results as every step its own launch
    (batched = 2) and, without branching, as per-branch launches
    (batched = 0), against the C
    transfer matrix; several instances of one structure in one call (same
    program, different base-tensor offsets) and a one-branch program
    (branching off) included."""
    gs = [I.spin_glass_square(L, s) for s in range(3)]
    want = [tm_c.spin_glass_lattice(L, L, g["edges"], g["J"]) for g in gs]
    insts = [(g["n"], g["edges"], g["J"], None) for g in gs]
    for batched in ((1, 2, 0) if branching == 0 else (1, 2)):
        opt = B.Options(log2_target=t, residues_per_pass=3, branching=branching, batched=batched)
        with B.Context(opt) as ctx:
            rs, st = ctx.solve_batch(0, insts)
        assert st == [0] * len(gs)
        for (n, e, J, _), r, w in zip(insts, rs, want):
            assert (r.value, r.count) == w and r.certified, (batched, r.value, r.count, w)
            assert config.spin_glass_energy(r.config, e, J) == r.value
