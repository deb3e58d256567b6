"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds input generators only: it computes nothing the method
computes (no energies, no contractions, no counts).  Both the CPU oracle and
the GPU path read their inputs from here, so the two see identical instances.

Workload families (the paper's Applications section):
  * +-J spin glass on an L x L open-boundary square lattice, couplings drawn
    uniformly from {-1, +1}; the external field is an optional extra input.
  * King's subgraph (KSG): an L x L grid whose sites are kept with
    probability `fill` (0.8 in the paper), with edges between kept sites that
    are a king move apart; unit or integer vertex weights.
  * +-J spin glass on a random 3-regular graph and on an open cubic lattice
    (the other topologies of the paper's spin-glass experiments).
  * random tensors in the device encoding of the counting tropical algebra
    (int32 value plane + residues modulo 31-bit primes), with planted ties and
    "minus infinity" entries, for kernel-level parity tests.
"""
from __future__ import annotations

import numpy as np

# Largest primes below 2**31, in descending order.  They are inputs (which
# moduli a caller asks for), not arithmetic of the method.
PRIMES_31 = (2147483647, 2147483629, 2147483587, 2147483579, 2147483563,
             2147483549, 2147483543, 2147483497, 2147483489, 2147483477,
             2147483423, 2147483399, 2147483353, 2147483323, 2147483269,
             2147483249)

# Device encoding of the tropical zero ("minus infinity" in max form): any
# value at or below NEG_CUT is minus infinity; the canonical stored value is NEG.
NEG = -(1 << 30)
NEG_CUT = -(1 << 29)


def spin_glass_square(L: int, seed: int, field: int = 0):
    """+-J spin glass on an L x L open-boundary lattice.

    Draw order: horizontal couplings Jh[L, L-1], then vertical Jv[L-1, L],
    both uniform in {-1, +1} from numpy's default_rng(seed).  Spin p = r*L + c.
    Edges are listed row-major per site: the right bond (r,c)-(r,c+1), then
    the down bond (r,c)-(r+1,c).  `field` is a uniform integer field h_i
    (zero unless asked for).

    Returns dict(n, edges[m,2] int32, J[m] int32, h[n] int32, L).
    """
    rng = np.random.default_rng(seed)
    Jh = rng.choice([-1, 1], size=(L, L - 1)) if L > 1 else np.zeros((L, 0), int)
    Jv = rng.choice([-1, 1], size=(L - 1, L)) if L > 1 else np.zeros((0, L), int)
    edges, J = [], []
    for r in range(L):
        for c in range(L):
            p = r * L + c
            if c + 1 < L:
                edges.append((p, p + 1))
                J.append(int(Jh[r, c]))
            if r + 1 < L:
                edges.append((p, p + L))
                J.append(int(Jv[r, c]))
    n = L * L
    return dict(n=n, L=L,
                edges=np.asarray(edges, dtype=np.int32).reshape(-1, 2),
                J=np.asarray(J, dtype=np.int32),
                h=np.full(n, field, dtype=np.int32))


def spin_glass_random_regular(n: int, seed: int, degree: int = 3):
    """+-J spin glass on a random `degree`-regular simple graph with n sites.

    Pairing model: the n * degree half-edges (site i appears `degree` times)
    are shuffled with numpy's default_rng(seed) and paired in order; a
    pairing with a self-loop or a repeated pair is drawn again from the same
    generator.  Then couplings uniform in {-1, +1}, one per edge in pairing
    order (edge = (smaller id, larger id)).

    Returns dict(n, edges[m,2] int32, J[m] int32, h[n] int32 (zero)).
    """
    assert n * degree % 2 == 0 and degree < n
    rng = np.random.default_rng(seed)
    stubs = np.repeat(np.arange(n), degree)
    while True:
        rng.shuffle(stubs)
        pairs = stubs.reshape(-1, 2)
        a = np.minimum(pairs[:, 0], pairs[:, 1])
        b = np.maximum(pairs[:, 0], pairs[:, 1])
        if np.all(a != b) and len(set(zip(a.tolist(), b.tolist()))) == len(a):
            break
    J = rng.choice([-1, 1], size=len(a))
    return dict(n=n, edges=np.stack([a, b], axis=1).astype(np.int32),
                J=J.astype(np.int32), h=np.zeros(n, dtype=np.int32))


def spin_glass_cubic(Lx: int, Ly: int, Lz: int, seed: int):
    """+-J spin glass on an Lx x Ly x Lz open-boundary cubic lattice.

    Site p = (x * Ly + y) * Lz + z.  Edges per site in order: +z, +y, +x
    neighbour (when inside the box), couplings uniform in {-1, +1} drawn in
    edge order from numpy's default_rng(seed).

    Returns dict(n, edges[m,2] int32, J[m] int32, h[n] int32 (zero)).
    """
    edges = []
    for x in range(Lx):
        for y in range(Ly):
            for z in range(Lz):
                p = (x * Ly + y) * Lz + z
                if z + 1 < Lz:
                    edges.append((p, p + 1))
                if y + 1 < Ly:
                    edges.append((p, p + Lz))
                if x + 1 < Lx:
                    edges.append((p, p + Ly * Lz))
    rng = np.random.default_rng(seed)
    J = rng.choice([-1, 1], size=len(edges))
    n = Lx * Ly * Lz
    return dict(n=n, edges=np.asarray(edges, dtype=np.int32).reshape(-1, 2),
                J=J.astype(np.int32), h=np.zeros(n, dtype=np.int32))


def spin_glass_rect(Lr: int, Lc: int, seed: int):
    """+-J spin glass on an Lr x Lc open lattice (strips); same draw scheme
    as `spin_glass_square` with Jh[Lr, Lc-1] then Jv[Lr-1, Lc]."""
    rng = np.random.default_rng(seed)
    Jh = rng.choice([-1, 1], size=(Lr, Lc - 1))
    Jv = rng.choice([-1, 1], size=(Lr - 1, Lc))
    edges, J = [], []
    for r in range(Lr):
        for c in range(Lc):
            p = r * Lc + c
            if c + 1 < Lc:
                edges.append((p, p + 1))
                J.append(int(Jh[r, c]))
            if r + 1 < Lr:
                edges.append((p, p + Lc))
                J.append(int(Jv[r, c]))
    n = Lr * Lc
    return dict(n=n, Lr=Lr, Lc=Lc,
                edges=np.asarray(edges, dtype=np.int32).reshape(-1, 2),
                J=np.asarray(J, dtype=np.int32),
                h=np.zeros(n, dtype=np.int32))


def kings_subgraph(L: int, seed: int, fill: float = 0.8, weights: str = "unit"):
    """King's subgraph on an L x L grid.

    present = default_rng(seed).random((L, L)) < fill; vertices are the present
    sites in row-major order; edges join present (r,c) to present (r,c+1),
    (r+1,c-1), (r+1,c), (r+1,c+1).  weights="unit" gives w_i = 1;
    weights="1..10" draws integers 1..10 after the mask (the paper's MWIS
    setting).

    Returns dict(n, edges[m,2] int32, w[n] int32, L, sites[n,2], present).
    """
    rng = np.random.default_rng(seed)
    present = rng.random((L, L)) < fill
    vid = -np.ones((L, L), dtype=np.int64)
    sites = []
    for r in range(L):
        for c in range(L):
            if present[r, c]:
                vid[r, c] = len(sites)
                sites.append((r, c))
    edges = []
    for (r, c) in sites:
        a = vid[r, c]
        for dr, dc in ((0, 1), (1, -1), (1, 0), (1, 1)):
            rr, cc = r + dr, c + dc
            if 0 <= rr < L and 0 <= cc < L and present[rr, cc]:
                edges.append((a, vid[rr, cc]))
    n = len(sites)
    if weights == "unit":
        w = np.ones(n, dtype=np.int32)
    elif weights == "1..10":
        w = rng.integers(1, 11, size=n).astype(np.int32)
    else:
        raise ValueError(weights)
    return dict(n=n, L=L, edges=np.asarray(edges, dtype=np.int32).reshape(-1, 2),
                w=w, sites=np.asarray(sites, dtype=np.int32).reshape(-1, 2),
                present=present)


def full_kings_graph(L: int):
    """Complete King's graph on L x L (every site present)."""
    g = kings_subgraph(L, seed=0, fill=2.0)
    return g


def random_entries(shape, k: int, seed: int, vrange: int = 8, neg_frac: float = 0.25,
                   primes=PRIMES_31):
    """Random tensor in the device encoding: int32 values uniform in
    [-vrange, vrange] (dense ties), a fraction `neg_frac` set to NEG with zero
    residues, and k residue planes uniform in [0, p_i).

    Returns (val int32[shape], res uint32[k, *shape]).
    """
    rng = np.random.default_rng(seed)
    val = rng.integers(-vrange, vrange + 1, size=shape).astype(np.int32)
    res = np.empty((k,) + tuple(shape), dtype=np.uint32)
    for i in range(k):
        res[i] = rng.integers(0, primes[i], size=shape, dtype=np.uint64).astype(np.uint32)
    if neg_frac > 0:
        neg = rng.random(shape) < neg_frac
        val[neg] = NEG
        res[:, neg] = 0
    return val, res


def to_bf16_bits(x):
    """float32 -> bfloat16 bit patterns, round to nearest even (inputs to the
    scorer's kernels; finite values only)."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16)


def mlp_params(seed: int, n_in: int = 32, n_h: int = 128, scale: float = 1.0):
    """Random MLP parameters (float32) for scorer kernel tests: weights
    uniform in +-scale/sqrt(fan_in), biases uniform in +-0.1."""
    rng = np.random.default_rng(seed)
    def U(shape, fan):
        return (rng.uniform(-1, 1, size=shape) * scale / np.sqrt(fan)).astype(np.float32)
    return dict(W1=U((n_h, n_in), n_in), b1=rng.uniform(-.1, .1, n_h).astype(np.float32),
                W2=U((n_h, n_h), n_h), b2=rng.uniform(-.1, .1, n_h).astype(np.float32),
                w3=U((n_h,), n_h), b3=np.float32(rng.uniform(-.1, .1)))
