"""The tile autotuner: with an autotune cache path set, a product of at
least 2^24 multiply-accumulates is timed over the candidate tile
configurations and split factors on the device; the pick is written to the
cache file, and the products and solves run with the tuned tiles match the
oracle."""
import os

import numpy as np
import pytest

import instances as I
from oracle import device_ops as D
from oracle import config
from tests.gpu_util import torch_cuda, to_dev, from_dev, empty_dev

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def B():
    torch_cuda()
    import paper_2602_05470_amd as B
    return B


def _cache_rows(path):
    rows = []
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            rows.append([int(x) for x in line.split()])
    return rows


def test_autotuned_product_matches_oracle(B, tmp_path):
    torch = torch_cuda()
    cache = str(tmp_path / "tune.txt")
    k = 3
    primes = I.PRIMES_31[:k]
    b, M, N, K = 1, 512, 256, 256          # 2^25 MACs: tuned
    Av, Ar = I.random_entries((b, M, K), k, seed=41, vrange=3)
    Bv, Br = I.random_entries((b, K, N), k, seed=42, vrange=3)
    dA, dB = to_dev(torch, Av, Ar), to_dev(torch, Bv, Br)
    dC = empty_dev(torch, k, b * M * N)
    with B.Context(B.Options(autotune_cache=cache)) as ctx:
        ctx.tgemm(k, primes, b, M, N, K, dA, dB, dC)
        torch.cuda.synchronize()
    rows = _cache_rows(cache)
    # k, log2 batch, log2 M, log2 N, log2 K, tile config, split factor
    assert [r[:5] for r in rows] == [[3, 0, 9, 8, 8]]
    assert 0 <= rows[0][5] < 12 and rows[0][6] >= 1
    gv, gr = from_dev(dC, k, b * M * N)
    wv, wr = D.tgemm(Av, Ar, Bv, Br, primes)
    assert np.array_equal(gv, wv.reshape(-1))
    assert np.array_equal(gr, wr.reshape(k, -1))
    # a second context reads the cache (no new entry for the same bucket)
    dC2 = empty_dev(torch, k, b * M * N)
    with B.Context(B.Options(autotune_cache=cache)) as ctx:
        ctx.tgemm(k, primes, b, M, N, K, dA, dB, dC2)
        torch.cuda.synchronize()
    assert _cache_rows(cache) == rows
    assert torch.equal(dC, dC2)


def test_autotuned_solve_matches_transfer_matrix(B, tmp_path):
    """24x24 +-J lattice (T_target = 2^20, refined order; leaves too large for
    the persistent executor, so every step is a product launch): every
    product of 2^24 MACs or more runs with tuned tiles; exact against the C
    transfer matrix's stored degeneracy."""
    cache = str(tmp_path / "tune.txt")
    want = {}
    for line in open(os.path.join(GOLDEN, "sg24.txt")):
        if line.strip() and not line.startswith("#"):
            s, e, d = (int(x) for x in line.split())
            want[s] = (e, d)
    g = I.spin_glass_square(24, 0)
    with B.Context(B.Options(log2_target=20, order_refine=8, residues_per_pass=3,
                             autotune_cache=cache, time_limit_s=300)) as ctx:
        r = ctx.solve_spinglass(g["n"], g["edges"], g["J"])
    assert (r.value, r.count) == want[0] and r.certified
    assert config.spin_glass_energy(r.config, g["edges"], g["J"], None) == r.value
    assert len(_cache_rows(cache)) >= 1
