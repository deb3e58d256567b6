"""Per-kernel operations in the device encoding of the counting tropical
algebra (max form), written as plain definitions for parity tests.

Encoding: an entry is an int32 value v and k residues c_i in [0, p_i).  The
tropical zero ("minus infinity", the (inf, 0) tuple of the MWIS paragraph read
in max form) is any v <= NEG_CUT = -2^29; it is stored as NEG = -2^30 with all
residues 0.  Max form: the sum keeps the larger value and adds the counts on
ties; the product adds values and multiplies counts (Eq. 2 with the order
reversed, which is how the spin-glass tensors are negated).

A term a (.) b is finite iff both factors are finite and a.v + b.v > NEG_CUT.

Flat index convention: bit j of a tensor's flat index is the state of the
tensor's j-th variable.  numpy arrays here are reshaped with the reversed
axis order (last numpy axis = bit 0) so that the definitions below use array
transposition and indexing instead of bit arithmetic.
"""
from __future__ import annotations

import numpy as np

NEG = -(1 << 30)
NEG_CUT = -(1 << 29)


def is_finite(v):
    return np.asarray(v) > NEG_CUT


def tgemm(Av, Ar, Bv, Br, primes):
    """C[b,m,n] = (+)_k A[b,m,k] (.) B[b,k,n]  (counting tropical GEMM).

    Av int32[b,M,K], Ar uint32[k,b,M,K], Bv int32[b,K,N], Br uint32[k,b,K,N].
    Returns Cv int32[b,M,N], Cr uint32[k,b,M,N].
    """
    Av = np.asarray(Av, np.int64)
    Bv = np.asarray(Bv, np.int64)
    nb, M, K = Av.shape
    N = Bv.shape[2]
    kk = len(primes)
    Cv = np.full((nb, M, N), NEG, dtype=np.int64)
    Cr = np.zeros((kk, nb, M, N), dtype=np.uint64)
    for q in range(K):
        a = Av[:, :, q][:, :, None]
        b = Bv[:, q, :][:, None, :]
        cand = a + b
        fin = is_finite(a) & is_finite(b) & (cand > NEG_CUT)
        gt = fin & (cand > Cv)
        eq = fin & (cand == Cv)
        for i, p in enumerate(primes):
            p = np.uint64(p)
            prod = (np.asarray(Ar[i], np.uint64)[:, :, q][:, :, None] *
                    np.asarray(Br[i], np.uint64)[:, q, :][:, None, :]) % p
            Cr[i] = np.where(gt, prod, np.where(eq, (Cr[i] + prod) % p, Cr[i]))
        Cv = np.where(gt, cand, Cv)
    return Cv.astype(np.int32), Cr.astype(np.uint32)


def _as_axes(flat, r):
    """flat[2^r] -> array of shape [2]*r with axis j holding bit j."""
    a = np.asarray(flat).reshape([2] * r) if r else np.asarray(flat).reshape(())
    return np.transpose(a, list(range(r - 1, -1, -1))) if r else a


def _from_axes(a, r):
    return np.transpose(a, list(range(r - 1, -1, -1))).reshape(-1) if r else a.reshape(1)


def gather(flat, r_in, src_bits, fixed=None):
    """Permute and slice one tensor plane.

    Output variable j is input variable src_bits[j]; `fixed` maps further
    input variables to a fixed state 0/1 (branch-variable fixing).  Every
    input variable must be either mapped or fixed.
    """
    fixed = fixed or {}
    a = _as_axes(flat, r_in)
    idx = [slice(None)] * r_in
    for pos, val in fixed.items():
        idx[pos] = int(val)
    a = a[tuple(idx)]
    remaining = [j for j in range(r_in) if j not in fixed]   # axis order of a
    order = [remaining.index(s) for s in src_bits]
    a = np.transpose(a, order) if order else a
    return _from_axes(np.ascontiguousarray(a), len(src_bits))


def reduce_bits(v, r, primes, sum_bits):
    """Tropical sum over the variables in `sum_bits` of a tensor with r
    variables; kept variables keep their relative order.
    v = (val int32[2^r], res uint32[k, 2^r])."""
    val, res = v
    Va = _as_axes(np.asarray(val, np.int64), r)
    Ra = [_as_axes(np.asarray(res[i], np.uint64), r) for i in range(len(primes))]
    keep = [j for j in range(r) if j not in sum_bits]
    # move summed axes last and flatten them
    perm = keep + list(sum_bits)
    Va = np.transpose(Va, perm).reshape([2] * len(keep) + [-1])
    Ra = [np.transpose(x, perm).reshape([2] * len(keep) + [-1]) for x in Ra]
    fin = Va > NEG_CUT
    best = np.where(fin, Va, np.iinfo(np.int64).min).max(axis=-1)
    anyfin = fin.any(axis=-1)
    tie = fin & (Va == best[..., None])
    out_v = np.where(anyfin, best, NEG)
    out_r = []
    for i, p in enumerate(primes):
        s = np.where(tie, Ra[i], 0).astype(object).sum(axis=-1)
        out_r.append(np.where(anyfin, np.asarray(s % int(p), dtype=np.uint64), 0))
    ov = _from_axes(np.asarray(out_v), len(keep)).astype(np.int32)
    orr = np.stack([_from_axes(np.asarray(x), len(keep)) for x in out_r]).astype(np.uint32)
    return ov, orr


def merge(vals, res, primes):
    """Tropical sum of a list of scalars: vals int32[L], res uint32[k, L]."""
    vals = np.asarray(vals, np.int64)
    fin = vals > NEG_CUT
    if not fin.any():
        return NEG, [0] * len(primes)
    best = int(vals[fin].max())
    tie = fin & (vals == best)
    out = [int(sum(int(x) for x in np.asarray(res[i])[tie]) % int(p))
           for i, p in enumerate(primes)]
    return best, out


def tensor_max(val):
    """Largest finite value of a tensor (its contribution to the branch
    bound), or NEG if it has none."""
    val = np.asarray(val, np.int64)
    fin = val > NEG_CUT
    return int(val[fin].max()) if fin.any() else NEG
