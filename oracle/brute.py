"""Brute-force enumeration of every configuration (plain definition).

Spin glass, Eq. 1:  H(sigma) = sum_E -J_ij s_i s_j + sum_V -h_i s_i,
sigma in {-1,+1}^n.  Result: (E0 = min H, number of sigma with H = E0).
MWIS (MWIS paragraph): max total weight over independent sets and the number
of independent sets of that weight.

Enumerates in chunks with numpy; meant for n <= ~26.
"""
from __future__ import annotations

import numpy as np


def _chunks(n, chunk_bits=20):
    total = 1 << n
    step = 1 << min(n, chunk_bits)
    for start in range(0, total, step):
        idx = np.arange(start, min(total, start + step), dtype=np.int64)
        yield idx


def spin_glass(n, edges, J, h=None):
    """Return (E0, degeneracy, one ground configuration as +-1 int8 array).

    Bit i of the enumeration index is spin i, with bit 1 meaning sigma=+1.
    """
    edges = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    J = np.asarray(J, dtype=np.int64)
    h = np.zeros(n, np.int64) if h is None else np.asarray(h, dtype=np.int64)
    best, count, arg = None, 0, None
    for idx in _chunks(n):
        sig = ((idx[:, None] >> np.arange(n)) & 1) * 2 - 1          # [chunk, n]
        H = np.zeros(len(idx), dtype=np.int64)
        for (i, j), Jij in zip(edges, J):
            H -= Jij * sig[:, i] * sig[:, j]
        H -= sig @ h
        m = int(H.min())
        c = int((H == m).sum())
        if best is None or m < best:
            best, count = m, c
            arg = sig[int(np.argmax(H == m))].astype(np.int8)
        elif m == best:
            count += c
    return best, count, arg


def mwis(n, edges, w=None):
    """Return (W*, number of maximum-weight independent sets, one of them as
    0/1 int8 array)."""
    edges = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    w = np.ones(n, np.int64) if w is None else np.asarray(w, dtype=np.int64)
    best, count, arg = None, 0, None
    for idx in _chunks(n):
        x = (idx[:, None] >> np.arange(n)) & 1
        ok = np.ones(len(idx), dtype=bool)
        for (i, j) in edges:
            ok &= ~((x[:, i] == 1) & (x[:, j] == 1))
        W = x @ w
        W = np.where(ok, W, np.iinfo(np.int64).min)
        m = int(W.max())
        c = int((W == m).sum())
        if best is None or m > best:
            best, count = m, c
            arg = x[int(np.argmax(W == m))].astype(np.int8)
        elif m == best:
            count += c
    return best, count, arg
