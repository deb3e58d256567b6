"""The larger lattice configurations with the refined contraction order:
+-J spin glass 32x32 and unweighted MIS on a King's subgraph of a 40x40 grid
(fill 0.8).  Parity unpinned: no oracle here reaches these sizes (the
transfer matrix would need 2^32 and 2^41 frontier states).  Checked instead
by what the mathematics fixes: two runs with different T_target produce
different leaf sets (different slicings of the same network), which must give
the same ground value and degeneracy; the spin-flip symmetry of a zero-field
spin glass makes its degeneracy even; the returned configuration must reach
the value ("Branch-and-Bound Tensor Network": branches are complete and
disjoint, so any valid branching gives the same tropical sum)."""
import numpy as np
import pytest

import instances as I
from oracle import config

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from tests.gpu_util import torch_cuda
    torch_cuda()
    import paper_2602_05470_amd as B
    return B


def test_sg32_two_slicings_agree(B):
    g = I.spin_glass_square(32, 0)
    out = []
    for t in (26, 24):
        with B.Context(B.Options(log2_target=t, order_refine=8, time_limit_s=100)) as ctx:
            r = ctx.solve_spinglass(g["n"], g["edges"], g["J"])
        assert r.certified
        assert config.spin_glass_energy(r.config, g["edges"], g["J"], None) == r.value
        out.append((r.value, r.count, r.leaves))
    (v0, c0, l0), (v1, c1, l1) = out
    assert l0 != l1                      # two different branchings
    assert (v0, c0) == (v1, c1)
    assert c0 % 2 == 0 and c0 > 0


def test_ksg40_branched_equals_whole(B):
    g = I.kings_subgraph(40, 0)
    out = []
    for t in (24, 28):
        with B.Context(B.Options(log2_target=t, order_refine=8, residues_per_pass=4,
                                 time_limit_s=100)) as ctx:
            r = ctx.solve_mwis(g["n"], g["edges"], g["w"])
        assert r.certified
        assert config.independent_set_weight(r.config, g["edges"], g["w"]) == r.value
        out.append((r.value, r.count, r.leaves))
    (v0, c0, l0), (v1, c1, l1) = out
    assert l0 > 1 and l1 == 1            # branched, and one whole contraction
    assert (v0, c0) == (v1, c1)
    assert c0 >= 1
