"""The larger lattice configurations with the refined contraction order:
+-J spin glass 32x32 and unweighted MIS on a King's subgraph of a 40x40 grid
(fill 0.8).

Values are pinned: the ground energy of every seed equals the matching
oracle's and the MIS size equals the integer-programming oracle's (stored in
tests/golden/ by make_golden.py, which calls only the oracle).  Parity
unpinned for the degeneracy: no exact counter here reaches these sizes (the
transfer matrix would need 2^32 and 2^41 frontier states).  The count is
checked instead by what the mathematics fixes: two runs with different
T_target produce different leaf sets (different slicings of the same
network), which must give the same ground value and degeneracy; the
spin-flip symmetry of a zero-field spin glass makes its degeneracy even;
the count is certified by a further prime; the returned configuration must
reach the value ("Branch-and-Bound Tensor Network": branches are complete
and disjoint, so any valid branching gives the same tropical sum)."""
import os

import numpy as np
import pytest

import instances as I
from oracle import config

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                row = [int(x) for x in line.split()]
                out[row[0]] = row[1:]
    return out


@pytest.fixture(scope="module")
def B():
    from tests.gpu_util import torch_cuda
    torch_cuda()
    import paper_2602_05470_amd as B
    return B


@pytest.fixture(scope="module")
def sg32_ctx(B):
    with B.Context(B.Options(log2_target=26, order_refine=8, residues_per_pass=4,
                             time_limit_s=200)) as ctx:
        yield ctx


@pytest.fixture(scope="module")
def ksg40_ctx(B):
    with B.Context(B.Options(log2_target=24, order_refine=8, residues_per_pass=4,
                             time_limit_s=200)) as ctx:
        yield ctx


@pytest.mark.parametrize("seed", range(4))
def test_sg32_value_matches_matching_oracle(sg32_ctx, seed):
    g = I.spin_glass_square(32, seed)
    print("SG 32x32 seed", seed, flush=True)
    r = sg32_ctx.solve_spinglass(g["n"], g["edges"], g["J"])
    assert r.value == _golden("sg32_values.txt")[seed][0]
    assert r.certified
    assert r.count % 2 == 0 and r.count > 0
    assert config.spin_glass_energy(r.config, g["edges"], g["J"], None) == r.value


@pytest.mark.parametrize("seed", range(4))
def test_ksg40_value_matches_milp_oracle(ksg40_ctx, seed):
    g = I.kings_subgraph(40, seed)
    print("KSG 40x40 seed", seed, flush=True)
    r = ksg40_ctx.solve_mwis(g["n"], g["edges"], g["w"])
    n, w = _golden("ksg40_values.txt")[seed]
    assert g["n"] == n
    assert r.value == w
    assert r.certified and r.count >= 1
    assert config.independent_set_weight(r.config, g["edges"], g["w"]) == r.value


def test_sg32_two_slicings_agree(B):
    g = I.spin_glass_square(32, 0)
    out = []
    for t in (26, 24):
        with B.Context(B.Options(log2_target=t, order_refine=8, time_limit_s=200)) as ctx:
            r = ctx.solve_spinglass(g["n"], g["edges"], g["J"])
        assert r.certified
        assert config.spin_glass_energy(r.config, g["edges"], g["J"], None) == r.value
        out.append((r.value, r.count, r.leaves))
    (v0, c0, l0), (v1, c1, l1) = out
    assert l0 != l1                      # two different branchings
    assert (v0, c0) == (v1, c1)
    assert v0 == -1432                   # the matching oracle's E0
    assert c0 % 2 == 0 and c0 > 0


def test_ksg40_branched_equals_whole(B):
    g = I.kings_subgraph(40, 0)
    out = []
    for t in (24, 28):
        with B.Context(B.Options(log2_target=t, order_refine=8, residues_per_pass=4,
                                 time_limit_s=200)) as ctx:
            r = ctx.solve_mwis(g["n"], g["edges"], g["w"])
        assert r.certified
        assert config.independent_set_weight(r.config, g["edges"], g["w"]) == r.value
        out.append((r.value, r.count, r.leaves))
    (v0, c0, l0), (v1, c1, l1) = out
    assert l0 > 1 and l1 == 1            # branched, and one whole contraction
    assert (v0, c0) == (v1, c1)
    assert v0 == 377                     # the integer program's W*
    assert c0 >= 1


def test_sg32_learned_scorer_matches_plain_planner(B):
    """The shipped spin-glass scorer on the 32x32 lattice (branching = 2):
    the same ground energy and degeneracy as the plain planner and the
    matching oracle's E0; the ratio of contraction work is printed (the
    scorer orders the branching variables, so it may cost more or less)."""
    g = I.spin_glass_square(32, 0)
    wpath = os.path.join(os.path.dirname(B.__file__), "scorer_sg.bin")
    out = {}
    for branching in (1, 2):
        with B.Context(B.Options(log2_target=26, order_refine=8, residues_per_pass=3,
                                 branching=branching,
                                 scorer_weights=wpath if branching == 2 else None,
                                 time_limit_s=300)) as ctx:
            r = ctx.solve_spinglass(g["n"], g["edges"], g["J"])
        assert r.certified
        assert config.spin_glass_energy(r.config, g["edges"], g["J"], None) == r.value
        out[branching] = r
    assert (out[2].value, out[2].count) == (out[1].value, out[1].count)
    assert out[1].value == _golden("sg32_values.txt")[0][0]
    print("scorer / plain MACs: %.3f, leaves %d / %d"
          % (out[2].macs / out[1].macs, out[2].leaves, out[1].leaves))
