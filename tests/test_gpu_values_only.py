"""Values-only mode (residues_per_pass = 0): the ground value and one
configuration reaching it, with the search pruning every branch that cannot
beat the local-search incumbent and keeping one optimal interior per
boundary state."""
import os

import numpy as np
import pytest

import instances as I
from oracle import config, tm_c

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    """seed -> (value, count); the King's-subgraph files also list n."""
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


@pytest.mark.parametrize("seed", range(5))
def test_sg16_values_only(B, seed):
    want = _golden("sg16.txt")[seed]
    g = I.spin_glass_square(16, seed)
    with B.Context(B.Options(log2_target=10, residues_per_pass=0)) as ctx:
        r = ctx.solve_spinglass(g["n"], g["edges"], g["J"])
    assert r.value == want[0]
    assert r.count == 0 and not r.certified and r.primes == []
    assert set(np.unique(r.config)) <= {-1, 1}
    assert config.spin_glass_energy(r.config, g["edges"], g["J"]) == r.value


@pytest.mark.parametrize("seed", range(3))
def test_sg_field_values_only(B, seed):
    """Field 0.5 (doubled to integers: J = +-2, h = 1), 12 x 12."""
    g = I.spin_glass_square(12, seed)
    J2 = [2 * j for j in g["J"]]
    h = [1] * g["n"]
    want = tm_c.spin_glass_lattice(12, 12, g["edges"], J2, h)
    with B.Context(B.Options(log2_target=6, residues_per_pass=0)) as ctx:
        r = ctx.solve_spinglass(g["n"], g["edges"], J2, h)
    assert r.value == want[0]
    assert config.spin_glass_energy(r.config, g["edges"], J2, h) == r.value


@pytest.mark.parametrize("seed", range(3))
def test_ksg16_values_only(B, seed):
    want = _golden("ksg16.txt")[seed]
    g = I.kings_subgraph(16, seed)
    with B.Context(B.Options(log2_target=8, residues_per_pass=0)) as ctx:
        r = ctx.solve_mwis(g["n"], g["edges"], g["w"])
    assert r.value == want[0]
    assert config.independent_set_weight(r.config, g["edges"], g["w"]) == r.value


def test_values_only_without_incumbent(B):
    """No local search: nothing to prune against; the best leaf decides."""
    g = I.spin_glass_square(10, 2)
    want = tm_c.spin_glass_lattice(10, 10, g["edges"], g["J"])
    with B.Context(B.Options(log2_target=5, residues_per_pass=0, local_search=0)) as ctx:
        r = ctx.solve_spinglass(g["n"], g["edges"], g["J"])
    assert r.value == want[0]
    assert config.spin_glass_energy(r.config, g["edges"], g["J"]) == r.value
