"""bbtn_tgemm_noalloc (the counting tropical product for callers that cannot
allocate device memory) against bbtn_tgemm through the C ABI: bit-exact on
two calls in a row, the second with a smaller product, both split along K so
that the static scratch array holds partial results; a third product whose
split-K partials would overflow the scratch runs with fewer splits and still
matches.  The calls allocate no device memory."""
import numpy as np
import pytest

import instances as I
from oracle import device_ops as D
from tests.gpu_util import torch_cuda, to_dev, from_dev, empty_dev

pytestmark = pytest.mark.gpu

SCRATCH_WORDS = 1 << 24


@pytest.fixture(scope="module")
def B():
    torch_cuda()
    import paper_2602_05470_amd as B
    return B


def _operands(torch, shape, k, seed):
    b, M, N, K = shape
    Av, Ar = I.random_entries((b, M, K), k, seed=seed, vrange=3)
    Bv, Br = I.random_entries((b, K, N), k, seed=seed + 1, vrange=3)
    return (Av, Ar, Bv, Br), to_dev(torch, Av, Ar), to_dev(torch, Bv, Br)


def test_noalloc_matches_tgemm_on_two_calls(B):
    torch = torch_cuda()
    k = 3
    primes = I.PRIMES_31[:k]
    # both split along K by the heuristic (few output tiles, K >= 256)
    big, small = (2, 96, 80, 2048), (1, 40, 24, 600)
    host, ops = {}, {}
    for i, shape in enumerate((big, small)):
        host[shape], *ops[shape] = _operands(torch, shape, k, 900 + 10 * i)
    ref = {s: empty_dev(torch, k, s[0] * s[1] * s[2]) for s in (big, small)}
    got = {s: empty_dev(torch, k, s[0] * s[1] * s[2]) for s in (big, small)}
    with B.Context(B.Options()) as c_ref, B.Context(B.Options()) as c_na:
        for s in (big, small):
            c_ref.tgemm(k, primes, *s, ops[s][0], ops[s][1], ref[s])
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        print("noalloc", big, flush=True)
        c_na.tgemm_noalloc(k, primes, *big, ops[big][0], ops[big][1], got[big])
        print("noalloc", small, flush=True)
        c_na.tgemm_noalloc(k, primes, *small, ops[small][0], ops[small][1], got[small])
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
    assert free0 - free1 < (1 << 20), (free0, free1)
    for s in (big, small):
        E = s[0] * s[1] * s[2]
        gv, gr = from_dev(got[s], k, E)
        rv, rr = from_dev(ref[s], k, E)
        assert np.array_equal(gv, rv) and np.array_equal(gr, rr), s
    # the smaller product also against the oracle's definition
    Av, Ar, Bv, Br = host[small]
    wv, wr = D.tgemm(Av, Ar, Bv, Br, primes)
    gv, gr = from_dev(got[small], k, small[0] * small[1] * small[2])
    assert np.array_equal(gv, wv.reshape(-1))
    assert np.array_equal(gr, wr.reshape(k, -1))


def test_noalloc_lowers_split_to_fit_scratch(B):
    """k = 4, (1, 1024, 512, 4096): the heuristic's 8 splits would need
    5 * 8 * 2^19 words, more than the 2^24-word scratch; the call runs with
    fewer splits and matches bbtn_tgemm."""
    torch = torch_cuda()
    k = 4
    primes = I.PRIMES_31[:k]
    shape = (1, 1024, 512, 4096)
    assert (1 + k) * 8 * shape[1] * shape[2] > SCRATCH_WORDS
    _, dA, dB = _operands(torch, shape, k, 77)
    E = shape[1] * shape[2]
    ref, got = empty_dev(torch, k, E), empty_dev(torch, k, E)
    with B.Context(B.Options()) as c:
        c.tgemm(k, primes, *shape, dA, dB, ref)
        print("noalloc", shape, flush=True)
        c.tgemm_noalloc(k, primes, *shape, dA, dB, got)
        torch.cuda.synchronize()
    assert torch.equal(ref, got)


def test_noalloc_rejects_bad_arguments(B):
    torch = torch_cuda()
    dA = torch.zeros(8, dtype=torch.int32, device="cuda")
    with B.Context(B.Options()) as c:
        with pytest.raises(B.BBTNError):
            c.tgemm_noalloc(5, I.PRIMES_31[:4], 1, 1, 1, 1, dA, dA, dA)
        with pytest.raises(B.BBTNError):
            c.tgemm_noalloc(3, I.PRIMES_31[:3], 1, 0, 1, 1, dA, dA, dA)
