"""ctypes wrapper of the C transfer-matrix oracle (oracle/tm.c), exact
multiword counts.  Same results as oracle/tm.py, much faster."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build_c

_lib = None


def _load():
    global _lib
    if _lib is None:
        build_c.build(force=False)
        lib = C.CDLL(build_c.LIB)
        lib.sg_tm.argtypes = [C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                              C.POINTER(C.c_int64), C.c_void_p, C.c_int]
        lib.sg_tm.restype = C.c_int
        lib.ksg_tm.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.POINTER(C.c_int64), C.c_void_p,
                               C.c_int]
        lib.ksg_tm.restype = C.c_int
        lib.tm_threads.argtypes = []
        lib.tm_threads.restype = C.c_int
        _lib = lib
    return _lib


def threads():
    """Threads the C oracle's parallel loops use (OpenMP)."""
    return int(_load().tm_threads())


def _count(words):
    v = 0
    for x in reversed(words.tolist()):
        v = (v << 64) | int(x)
    return v


def spin_glass_lattice(Lr, Lc, edges, J, h=None):
    """(E0, degeneracy) of Eq. 1 on an Lr x Lc lattice (nearest-neighbour
    edges only)."""
    n = Lr * Lc
    right = np.zeros(n, np.int32)
    down = np.zeros(n, np.int32)
    for (a, b), j in zip(np.asarray(edges).reshape(-1, 2), np.asarray(J)):
        a, b = int(min(a, b)), int(max(a, b))
        if b == a + 1 and a // Lc == b // Lc:
            right[a] += int(j)
        elif b == a + Lc:
            down[a] += int(j)
        else:
            raise ValueError("edge (%d,%d) is not a lattice bond" % (a, b))
    hh = None if h is None else np.ascontiguousarray(h, np.int32)
    words = n // 64 + 1
    cnt = np.zeros(words, np.uint64)
    e0 = C.c_int64(0)
    if _load().sg_tm(Lr, Lc, right.ctypes.data, down.ctypes.data,
                     None if hh is None else hh.ctypes.data, C.byref(e0), cnt.ctypes.data,
                     words) != 0:
        raise MemoryError("sg_tm")
    return int(e0.value), _count(cnt)


def kings_subgraph(inst):
    """(W*, number of maximum-weight independent sets) of a King's subgraph
    instance from `instances.kings_subgraph`."""
    L = inst["L"]
    present = np.ascontiguousarray(inst["present"].reshape(-1), np.uint8)
    w = np.zeros(L * L, np.int32)
    for vtx, (r, c) in enumerate(inst["sites"]):
        w[r * L + c] = int(inst["w"][vtx])
    words = int(present.sum()) // 64 + 1
    cnt = np.zeros(words, np.uint64)
    wm = C.c_int64(0)
    if _load().ksg_tm(L, present.ctypes.data, w.ctypes.data, C.byref(wm), cnt.ctypes.data,
                      words) != 0:
        raise MemoryError("ksg_tm")
    return int(wm.value), _count(cnt)
