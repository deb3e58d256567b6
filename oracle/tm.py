"""Exact transfer-matrix solvers for lattice instances (min form, exact ints).

Sites are added one at a time in row-major order.  The table holds one
(value, count) pair per state of the most recent W sites (the "frontier");
adding a site replaces the oldest frontier site, which is summed out with the
tropical sum.  This evaluates Eq. 2 exactly, in the order of a
row-by-row sweep, with arbitrary-precision counts.

Frontier slot of site q is q mod W, so a new site takes over exactly the slot
of the site it retires.  Sites not yet added sit in state 0 with count 0 for
state 1, so the first row needs no special case.
"""
from __future__ import annotations

import numpy as np


def _count_dtype(n_sites):
    # Partial counts never exceed 2^(sites added) <= 2^n: int64 is exact for
    # n <= 62; otherwise use Python integers.
    return np.int64 if n_sites <= 62 else object


def _oplus_vec(va, ca, vb, cb):
    """Elementwise tropical sum (min form); c == 0 marks the tropical zero."""
    ma = ca != 0
    mb = cb != 0
    both = ma & mb
    v = np.where(both, np.minimum(va, vb), np.where(ma, va, vb))
    tie_c = np.where(va < vb, ca, np.where(vb < va, cb, ca + cb))
    c = np.where(both, tie_c, np.where(ma, ca, cb))
    return v, c


def _finish(v, c):
    """Tropical sum over all states of the final table."""
    mask = c != 0
    if not mask.any():
        return None, 0
    best = int(v[mask].min())
    total = sum(int(x) for x in c[mask & (v == best)])
    return best, total


def spin_glass_lattice(Lr, Lc, edges, J, h=None):
    """(E0, degeneracy) of Eq. 1 on an Lr x Lc lattice whose bonds are the
    given edges (each a nearest-neighbour pair of sites r*Lc + c)."""
    n = Lr * Lc
    h = np.zeros(n, np.int64) if h is None else np.asarray(h, np.int64)
    right = {}
    down = {}
    for (a, b), Jab in zip(np.asarray(edges).reshape(-1, 2), np.asarray(J)):
        a, b = int(min(a, b)), int(max(a, b))
        if b == a + 1 and a // Lc == b // Lc:
            right[a] = right.get(a, 0) + int(Jab)
        elif b == a + Lc:
            down[a] = down.get(a, 0) + int(Jab)
        else:
            raise ValueError("edge (%d,%d) is not a lattice bond" % (a, b))
    W = Lc
    S = 1 << W
    cdt = _count_dtype(n)
    idx = np.arange(S, dtype=np.int64)
    v = np.zeros(S, dtype=np.int64)
    c = np.zeros(S, dtype=cdt)
    c[0] = 1
    for p in range(n):
        r, col = divmod(p, Lc)
        b = p % W
        bit = (idx >> b) & 1
        lo = idx[bit == 0]                  # states with slot b cleared
        hi = lo | (1 << b)
        new_v = np.zeros(S, dtype=np.int64)
        new_c = np.zeros(S, dtype=cdt)
        for t in (0, 1):                    # new spin state, sigma_p = 2t-1
            sp = 2 * t - 1
            base = np.full(lo.shape, -int(h[p]) * sp, dtype=np.int64)
            if col > 0:                     # left bond to p-1 (slot (p-1) mod W)
                sl = ((lo >> ((p - 1) % W)) & 1) * 2 - 1
                base = base - right[p - 1] * sl * sp
            acc_v, acc_c = None, None
            for u, src in ((0, lo), (1, hi)):   # retired site p-W in state u
                cv = v[src] + base
                if r > 0:
                    cv = cv - down[p - W] * (2 * u - 1) * sp
                cc = c[src]
                if acc_v is None:
                    acc_v, acc_c = cv, cc
                else:
                    acc_v, acc_c = _oplus_vec(acc_v, acc_c, cv, cc)
            dst = lo if t == 0 else hi
            new_v[dst] = acc_v
            new_c[dst] = acc_c
        v, c = new_v, new_c
    return _finish(v, c)


def spin_glass_square(inst):
    L = inst["L"]
    return spin_glass_lattice(L, L, inst["edges"], inst["J"], inst.get("h"))


def kings_subgraph(inst):
    """(W*, number of maximum-weight independent sets) of a King's subgraph
    instance from `instances.kings_subgraph` (MWIS paragraph: hard
    constraint on adjacent occupied sites, weight w_i per occupied site).

    Sweep over the full L x L grid; frontier of W = L + 1 sites covers the
    four earlier king neighbours (left, up-left, up, up-right).  Absent sites
    are held in state 0.
    """
    L = inst["L"]
    present = inst["present"]
    w_site = np.zeros(L * L, dtype=np.int64)
    for vtx, (r, c) in enumerate(inst["sites"]):
        w_site[r * L + c] = int(inst["w"][vtx])
    # edges must be exactly the king-move pairs among present sites
    W = L + 1
    S = 1 << W
    n_sites = L * L
    cdt = _count_dtype(int(present.sum()))
    idx = np.arange(S, dtype=np.int64)
    v = np.zeros(S, dtype=np.int64)
    c = np.zeros(S, dtype=cdt)
    c[0] = 1
    for p in range(n_sites):
        r, col = divmod(p, L)
        b = p % W
        bit = (idx >> b) & 1
        lo = idx[bit == 0]
        hi = lo | (1 << b)
        # occupied earlier king neighbours in the frontier
        nbrs = []
        if col > 0 and present[r, col - 1]:
            nbrs.append(p - 1)
        if r > 0:
            for dc in (-1, 0, 1):
                cc = col + dc
                if 0 <= cc < L and present[r - 1, cc]:
                    nbrs.append(p - L + dc)
        new_v = np.zeros(S, dtype=np.int64)
        new_c = np.zeros(S, dtype=cdt)
        for t in (0, 1):
            if t == 1 and not present[r, col]:
                continue                    # absent site: only state 0 exists
            ok = np.ones(lo.shape, dtype=bool)
            if t == 1:
                for q in nbrs:
                    if q == p - W:          # the retiring site: handled per u
                        continue
                    ok &= ((lo >> (q % W)) & 1) == 0
            acc_v, acc_c = None, None
            for u, src in ((0, lo), (1, hi)):
                cv = v[src] - w_site[p] * t
                cc = np.where(ok, c[src], 0).astype(cdt)
                if t == 1 and u == 1 and (p - W) in nbrs:
                    cc = np.zeros_like(cc)
                if acc_v is None:
                    acc_v, acc_c = cv, cc
                else:
                    acc_v, acc_c = _oplus_vec(acc_v, acc_c, cv, cc)
            dst = lo if t == 0 else hi
            new_v[dst] = acc_v
            new_c[dst] = acc_c
        v, c = new_v, new_c
    best, cnt = _finish(v, c)
    return -best, cnt
