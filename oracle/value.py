"""Value-only checks through library routines (no counts).

* Planar zero-field +-J lattice: the ground energy is -|E| + 2 * (fewest
  unsatisfied bonds).  A set of unsatisfied bonds is realisable iff it is odd
  exactly around the frustrated faces (faces with an odd number of J = -1
  bonds), counting the outer face so the total is even.  The fewest such bonds
  is a minimum T-join in the dual lattice, computed as a minimum-weight perfect
  matching on the frustrated faces with dual shortest-path distances
  (networkx's blossom algorithm).
* MIS / MWIS on any graph: integer program max w.x, x_i + x_j <= 1 per edge,
  solved by scipy.optimize.milp (HiGHS).
* Spin glass with field on any graph: integer program over s in {0,1}^n and
  y_e = s_i xor s_j (four linear inequalities per edge), minimising Eq. 1 with
  sigma_i sigma_j = 1 - 2 y_e and sigma_i = 2 s_i - 1.
"""
from __future__ import annotations

import numpy as np


def spin_glass_planar_e0(L, edges, J):
    """E0 for an L x L open lattice with unit |J| and zero field."""
    import networkx as nx
    Jmap = {}
    for (a, b), j in zip(np.asarray(edges).reshape(-1, 2), np.asarray(J)):
        a, b = int(min(a, b)), int(max(a, b))
        if abs(int(j)) != 1:
            raise ValueError("matching check assumes |J| = 1")
        Jmap[(a, b)] = int(j)
    m = len(Jmap)
    frustrated = []
    for r in range(L - 1):
        for c in range(L - 1):
            p = r * L + c
            bonds = [(p, p + 1), (p + L, p + L + 1), (p, p + L), (p + 1, p + L + 1)]
            neg = sum(1 for e in bonds if Jmap[e] < 0)
            if neg % 2 == 1:
                frustrated.append((r, c))
    nodes = list(frustrated)
    if len(nodes) % 2 == 1:
        nodes.append("outer")

    def dbdry(P):
        r, c = P
        return 1 + min(r, c, L - 2 - r, L - 2 - c)

    def dist(P, Q):
        if P == "outer":
            return dbdry(Q)
        if Q == "outer":
            return dbdry(P)
        man = abs(P[0] - Q[0]) + abs(P[1] - Q[1])
        return min(man, dbdry(P) + dbdry(Q))

    if not nodes:
        return -m
    G = nx.Graph()
    for i in range(len(nodes)):
        for j in range(i + 1, len(nodes)):
            G.add_edge(i, j, weight=dist(nodes[i], nodes[j]))
    M = nx.min_weight_matching(G)
    tj = sum(G[a][b]["weight"] for a, b in M)
    return -m + 2 * tj


def mwis_milp(n, edges, w=None, time_limit=None):
    """W* by integer programming (HiGHS)."""
    from scipy.optimize import milp, LinearConstraint, Bounds
    from scipy.sparse import coo_matrix
    w = np.ones(n) if w is None else np.asarray(w, float)
    e = np.asarray(edges, np.int64).reshape(-1, 2)
    rows = np.repeat(np.arange(len(e)), 2)
    A = coo_matrix((np.ones(2 * len(e)), (rows, e.reshape(-1))), shape=(len(e), n))
    cons = [LinearConstraint(A, -np.inf, 1)] if len(e) else []
    opts = {} if time_limit is None else {"time_limit": time_limit}
    res = milp(-w, constraints=cons, integrality=np.ones(n), bounds=Bounds(0, 1), options=opts)
    if not res.success:
        raise RuntimeError(res.message)
    return int(round(-res.fun))


def spin_glass_milp(n, edges, J, h=None, time_limit=None):
    """E0 of Eq. 1 by integer programming (HiGHS)."""
    from scipy.optimize import milp, LinearConstraint, Bounds
    from scipy.sparse import lil_matrix
    e = np.asarray(edges, np.int64).reshape(-1, 2)
    J = np.asarray(J, float)
    h = np.zeros(n) if h is None else np.asarray(h, float)
    m = len(e)
    nv = n + m                       # s_0..s_{n-1}, y_0..y_{m-1}
    # H = sum_e -J_e (1 - 2 y_e) + sum_i -h_i (2 s_i - 1)
    cost = np.zeros(nv)
    cost[n:] = 2 * J
    cost[:n] = -2 * h
    const = -J.sum() + h.sum()
    A = lil_matrix((4 * m, nv))
    lo = np.full(4 * m, -np.inf)
    hi = np.zeros(4 * m)
    for k, (i, j) in enumerate(e):
        y = n + k
        A[4 * k, y] = -1; A[4 * k, i] = 1; A[4 * k, j] = -1; hi[4 * k] = 0      # y >= s_i - s_j
        A[4 * k + 1, y] = -1; A[4 * k + 1, i] = -1; A[4 * k + 1, j] = 1; hi[4 * k + 1] = 0
        A[4 * k + 2, y] = 1; A[4 * k + 2, i] = -1; A[4 * k + 2, j] = -1; hi[4 * k + 2] = 0  # y <= s_i + s_j
        A[4 * k + 3, y] = 1; A[4 * k + 3, i] = 1; A[4 * k + 3, j] = 1; hi[4 * k + 3] = 2   # y <= 2 - s_i - s_j
    opts = {} if time_limit is None else {"time_limit": time_limit}
    res = milp(cost, constraints=[LinearConstraint(A.tocsr(), lo, hi)],
               integrality=np.ones(nv), bounds=Bounds(0, 1), options=opts)
    if not res.success:
        raise RuntimeError(res.message)
    return int(round(res.fun + const))
