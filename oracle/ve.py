"""Exact variable elimination for arbitrary graphs (min form, exact ints).

Factors are (vars, v, c) with numpy arrays of shape [2]*len(vars) (axis i is
variable vars[i]); c == 0 is the tropical zero.  Eliminating a variable takes
the tropical product of every factor holding it and the tropical sum over its
two states (Eq. 2 evaluated bucket by bucket).  Elimination order: repeatedly
the variable with the fewest neighbours in the current interaction graph,
lowest id first on ties.  Counts are Python integers.
"""
from __future__ import annotations

import numpy as np


def _oplus_vec(va, ca, vb, cb):
    ma = ca != 0
    mb = cb != 0
    both = ma & mb
    v = np.where(both, np.minimum(va, vb), np.where(ma, va, vb))
    tie_c = np.where(va < vb, ca, np.where(vb < va, cb, ca + cb))
    c = np.where(both, tie_c, np.where(ma, ca, cb))
    return v, c


def _expand(f, order):
    """View factor f over the variable list `order` (broadcastable shape)."""
    fv, v, c = f
    perm = sorted(range(len(fv)), key=lambda i: order.index(fv[i]))
    v = np.transpose(v, perm)
    c = np.transpose(c, perm)
    shape = [2 if x in fv else 1 for x in order]
    return v.reshape(shape), c.reshape(shape)


def _product(factors):
    order = sorted(set(x for f in factors for x in f[0]))
    full = [2] * len(order)
    v = np.zeros(full, dtype=np.int64)
    c = np.ones(full, dtype=object)
    for f in factors:
        fv, fc = _expand(f, order)
        v = v + fv
        c = c * fc
    return order, v, c


def _sum_out(order, v, c, x):
    ax = order.index(x)
    v0, v1 = np.take(v, 0, axis=ax), np.take(v, 1, axis=ax)
    c0, c1 = np.take(c, 0, axis=ax), np.take(c, 1, axis=ax)
    nv, nc = _oplus_vec(v0, c0, v1, c1)
    return [y for y in order if y != x], nv, nc


def solve_factors(n, factors):
    """Tropical sum over all 2^n configurations of the product of factors.
    Variables that occur in no factor contribute a factor 2 to the count."""
    factors = [(list(fv), np.asarray(v, np.int64), np.asarray(c, dtype=object))
               for fv, v, c in factors]
    used = set(x for f in factors for x in f[0])
    free_mult = 2 ** (n - len(used))
    nbr = {x: set() for x in used}
    for f in factors:
        for a in f[0]:
            nbr[a].update(y for y in f[0] if y != a)
    remaining = set(used)
    while remaining:
        x = min(remaining, key=lambda y: (len(nbr[y]), y))
        bucket = [f for f in factors if x in f[0]]
        rest = [f for f in factors if x not in f[0]]
        order, v, c = _product(bucket)
        order, v, c = _sum_out(order, v, c, x)
        rest.append((order, v, c))
        factors = rest
        for y in nbr[x]:
            nbr[y].discard(x)
            nbr[y].update(z for z in nbr[x] if z != y)
        del nbr[x]
        remaining.discard(x)
    val, cnt = 0, 1
    for fv, v, c in factors:            # all scalars now
        val += int(np.asarray(v).reshape(()))
        cnt *= int(np.asarray(c).reshape(()))
    return val, cnt * free_mult


def spin_glass(n, edges, J, h=None):
    """(E0, degeneracy) of Eq. 1 on any graph; edge tensor B^ij and vertex
    tensor w^i as in the "Tropical Tensor Networks" section, index s = 0 for
    sigma = -1 and s = 1 for sigma = +1."""
    h = np.zeros(n, np.int64) if h is None else np.asarray(h, np.int64)
    fs = []
    for (i, j), Jij in zip(np.asarray(edges).reshape(-1, 2), np.asarray(J)):
        Jij = int(Jij)
        # B^ij = [[-J, J], [J, -J]]: -J when the spins agree, +J otherwise
        B = np.array([[-Jij, Jij], [Jij, -Jij]], dtype=np.int64)
        fs.append(([int(i), int(j)], B, np.ones((2, 2), dtype=object)))
    for i in range(n):
        if h[i] != 0:
            # energy -h*sigma: sigma=-1 -> +h, sigma=+1 -> -h
            fs.append(([i], np.array([int(h[i]), -int(h[i])]), np.ones(2, dtype=object)))
    if any(i == j for i, j in np.asarray(edges).reshape(-1, 2)):
        raise ValueError("self-loop")
    return solve_factors(n, fs)


def mwis(n, edges, w=None):
    """(W*, number of maximum-weight independent sets): constraint tensor
    B = [[0,0],[0,inf]] becomes count 0 on (1,1); vertex tensor (0, -w_i)."""
    w = np.ones(n, np.int64) if w is None else np.asarray(w, np.int64)
    fs = []
    for (i, j) in np.asarray(edges).reshape(-1, 2):
        c = np.array([[1, 1], [1, 0]], dtype=object)
        fs.append(([int(i), int(j)], np.zeros((2, 2), np.int64), c))
    for i in range(n):
        fs.append(([i], np.array([0, -int(w[i])]), np.ones(2, dtype=object)))
    val, cnt = solve_factors(n, fs)
    return -val, cnt
