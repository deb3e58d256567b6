"""Counting tropical algebra with exact integers (min form, as in the paper).

An element is a pair (v, c): v the best energy, c >= 0 the number of
configurations reaching it.  c == 0 is the tropical zero: "no configuration",
the paper's (inf, 0) tuple of the MWIS paragraph; its v is irrelevant.

  (v1, c1) (+) (v2, c2) = the smaller value, with the counts added on a tie
  (v1, c1) (.) (v2, c2) = (v1 + v2, c1 * c2)

Eq. 2 evaluates (+) over all configurations of the (.) of every tensor entry.
"""
from __future__ import annotations


def oplus(a, b):
    """Tropical sum of two (v, c) pairs (min form)."""
    (v1, c1), (v2, c2) = a, b
    if c1 == 0:
        return (v2, c2)
    if c2 == 0:
        return (v1, c1)
    if v1 < v2:
        return (v1, c1)
    if v2 < v1:
        return (v2, c2)
    return (v1, c1 + c2)


def otimes(a, b):
    """Tropical product of two (v, c) pairs."""
    return (a[0] + b[0], a[1] * b[1])


ZERO = (0, 0)
ONE = (0, 1)


def oplus_all(items):
    acc = ZERO
    for it in items:
        acc = oplus(acc, it)
    return acc
