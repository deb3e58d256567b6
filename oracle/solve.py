"""Exact (value, degeneracy) for an instance, choosing a plain exact method.

Spin glass: E0 = min H (Eq. 1) and the number of minimisers.
MWIS: W* = max weight of an independent set and the number of them.
"""
from __future__ import annotations

from . import brute, tm, ve


def spin_glass(inst, method="auto"):
    n = inst["n"]
    if method == "brute" or (method == "auto" and n <= 20):
        e0, deg, _ = brute.spin_glass(n, inst["edges"], inst["J"], inst.get("h"))
        return e0, deg
    if method == "tm" or (method == "auto" and ("L" in inst or "Lr" in inst)):
        Lr = inst.get("Lr", inst.get("L"))
        Lc = inst.get("Lc", inst.get("L"))
        return tm.spin_glass_lattice(Lr, Lc, inst["edges"], inst["J"], inst.get("h"))
    return ve.spin_glass(n, inst["edges"], inst["J"], inst.get("h"))


def mwis(inst, method="auto"):
    n = inst["n"]
    if method == "brute" or (method == "auto" and n <= 20):
        w, cnt, _ = brute.mwis(n, inst["edges"], inst.get("w"))
        return w, cnt
    if method == "tm" or (method == "auto" and "present" in inst):
        return tm.kings_subgraph(inst)
    return ve.mwis(n, inst["edges"], inst.get("w"))
