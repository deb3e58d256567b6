"""Train the learned branching scorer on data the search itself generates.

Data: for seeded +-J lattices (16 x 16 at T_target = 2^10 and 24 x 24 at
2^16 by default), the planner records, at each of the first `max_nodes`
search nodes and for several candidate seed variables, 32 features and the
label log2(gamma) of the best branching rule grown from that seed (the
characteristic equation's branching factor, after pruning), taken relative to
the node's best candidate.  Collection is host code
(run in threads; the library releases the GIL).  Training runs on the GPU
with the library's own forward/backward/Adam kernels.

    python -m paper_2602_05470_amd.train_scorer --out paper_2602_05470_amd/scorer_weights.bin
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import instances as I  # noqa: E402
import paper_2602_05470_amd as B  # noqa: E402

DEFAULT_OUT = os.path.join(HERE, "scorer_weights.bin")


def collect(specs, max_nodes, cand, threads):
    """specs: list of (L, seed, log2_target)."""
    def one(spec):
        L, seed, t = spec
        g = I.spin_glass_square(L, seed)
        return B.scorer_collect(0, g["n"], g["edges"], g["J"], log2_target=t,
                                max_nodes=max_nodes, cand_per_node=cand)
    Xs, ys = [], []
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        for X, y in ex.map(one, specs):
            Xs.append(X)
            ys.append(y)
    return np.concatenate(Xs), np.concatenate(ys)


def training_specs(n16=250, n24=250):
    return ([(16, 10000 + i, 10) for i in range(n16)] +
            [(24, 20000 + i, 16) for i in range(n24)])


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--n16", type=int, default=250)
    ap.add_argument("--n24", type=int, default=250)
    ap.add_argument("--max-nodes", type=int, default=48)
    ap.add_argument("--cand", type=int, default=8)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=512)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--threads", type=int, default=min(16, os.cpu_count() or 4))
    ap.add_argument("--data", default=None, help="save/load the collected data (.npz)")
    a = ap.parse_args(argv)
    t0 = time.time()
    if a.data and os.path.exists(a.data):
        d = np.load(a.data)
        X, y = d["X"], d["y"]
    else:
        X, y = collect(training_specs(a.n16, a.n24), a.max_nodes, a.cand, a.threads)
        if a.data:
            np.savez_compressed(a.data, X=X, y=y)
    print("collected %d rows from %d instances in %.1f s" % (len(y), a.n16 + a.n24, time.time() - t0),
          flush=True)
    t1 = time.time()
    with B.Context() as ctx:
        loss = ctx.scorer_train(X, y, epochs=a.epochs, batch=a.batch, lr=a.lr, seed=0,
                                save_path=a.out)
    print("trained %d epochs in %.1f s; standardised MSE first %.4f last %.4f -> %s"
          % (a.epochs, time.time() - t1, loss[0], loss[-1], a.out), flush=True)
    return loss


if __name__ == "__main__":
    main()
