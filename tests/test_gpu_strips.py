"""+-J strips as long as the 48x48 and 64x64 lattices (48x20 and 64x16,
rows x columns) against the exact transfer matrix: branching and slicing
along the long dimension, counts of 68-97 bits (certified across passes),
with the plain and the five-residue (k = 4 plus a fused check prime)
counting passes and with the spin-flip option."""
import os

import pytest

import instances as I
from oracle import config

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    out = {}
    for line in open(os.path.join(GOLDEN, name)):
        if line.strip() and not line.startswith("#"):
            s, e, d = (int(x) for x in line.split())
            out[s] = (e, d)
    return out


@pytest.fixture(scope="module")
def B():
    from tests.gpu_util import torch_cuda
    torch_cuda()
    import paper_2602_05470_amd as B
    return B


@pytest.mark.parametrize("shape,t", [((48, 20), 18), ((64, 16), 16)])
@pytest.mark.parametrize("seed", [0, 1])
@pytest.mark.parametrize("k,flip", [(3, 0), (4, 1)])
def test_long_strip_vs_transfer_matrix(B, shape, t, seed, k, flip):
    Lr, Lc = shape
    want = _golden("sg%dx%d.txt" % shape)[seed]
    g = I.spin_glass_rect(Lr, Lc, seed)
    print("strip", shape, "seed", seed, "k", k, "flip", flip, flush=True)
    # greedy order: 64 leaves on 48x20 at T_target 2^18, 16 on 64x16 at 2^16
    with B.Context(B.Options(log2_target=t, residues_per_pass=k,
                             spin_flip=flip, time_limit_s=200)) as ctx:
        r = ctx.solve_spinglass(g["n"], g["edges"], g["J"])
    assert (r.value, r.count) == want
    assert r.certified and r.leaves > 1
    assert config.spin_glass_energy(r.config, g["edges"], g["J"], None) == r.value
