"""Evaluation of a single configuration (Eq. 1 and the MWIS objective)."""
from __future__ import annotations

import numpy as np


def spin_glass_energy(sigma, edges, J, h=None):
    """H(sigma) of Eq. 1 for sigma in {-1,+1}^n."""
    sigma = np.asarray(sigma, np.int64)
    e = np.asarray(edges, np.int64).reshape(-1, 2)
    H = -int(np.sum(np.asarray(J, np.int64) * sigma[e[:, 0]] * sigma[e[:, 1]]))
    if h is not None:
        H -= int(np.dot(np.asarray(h, np.int64), sigma))
    return H


def independent_set_weight(x, edges, w=None):
    """Total weight of the 0/1 vector x, or None if x is not independent."""
    x = np.asarray(x, np.int64)
    e = np.asarray(edges, np.int64).reshape(-1, 2)
    if len(e) and np.any((x[e[:, 0]] == 1) & (x[e[:, 1]] == 1)):
        return None
    w = np.ones(len(x), np.int64) if w is None else np.asarray(w, np.int64)
    return int(np.dot(w, x))
