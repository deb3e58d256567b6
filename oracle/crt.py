"""Chinese remaindering: the unique x in [0, prod p_i) with x = r_i mod p_i.

Plain textbook formula x = sum_i r_i * M_i * (M_i^{-1} mod p_i) mod M with
M = prod p_i and M_i = M / p_i, in Python integers.
"""
from __future__ import annotations


def crt(residues, primes):
    M = 1
    for p in primes:
        M *= int(p)
    x = 0
    for r, p in zip(residues, primes):
        p = int(p)
        Mi = M // p
        x += int(r) * Mi * pow(Mi, -1, p)
    return x % M
