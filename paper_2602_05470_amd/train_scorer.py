"""Train the learned branching scorer on data the search itself generates.

Data: for seeded +-J lattices (16 x 16 at T_target = 2^10 and 24 x 24 at
2^16, the default), or for seeded King's subgraphs with fill 0.8 (16 x 16 at
2^8 and 20 x 20 at 2^10, `--problem ksg`), the planner records, at each of the first `max_nodes`
search nodes and for several candidate seed variables, 32 features and the
label log2(gamma) of the best branching rule grown from that seed (the
characteristic equation's branching factor, after pruning), taken relative to
the node's best candidate.  Collection is host code
(run in threads; the library releases the GIL).  Training runs on the GPU
with the library's own forward/backward/Adam kernels.

    python -m paper_2602_05470_amd.train_scorer --out paper_2602_05470_amd/scorer_sg.bin
    python -m paper_2602_05470_amd.train_scorer --problem ksg --out paper_2602_05470_amd/scorer_ksg.bin
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

DEFAULT_OUT = {"sg": os.path.join(HERE, "scorer_sg.bin"),
               "ksg": os.path.join(HERE, "scorer_ksg.bin")}


def collect(specs, max_nodes, cand, threads, problem="sg"):
    """specs: list of (L, seed, log2_target)."""
    def one(spec):
        L, seed, t = spec
        if problem == "ksg":
            g = I.kings_subgraph(L, seed)
            return B.scorer_collect(1, g["n"], g["edges"], g["w"], log2_target=t,
                                    max_nodes=max_nodes, cand_per_node=cand)
        g = I.spin_glass_square(L, seed)
        return B.scorer_collect(0, g["n"], g["edges"], g["J"], log2_target=t,
                                max_nodes=max_nodes, cand_per_node=cand)
    Xs, ys = [], []
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        for X, y in ex.map(one, specs):
            Xs.append(X)
            ys.append(y)
    return np.concatenate(Xs), np.concatenate(ys)


def training_specs(n_small=250, n_large=250, problem="sg"):
    if problem == "ksg":
        return ([(16, 10000 + i, 8) for i in range(n_small)] +
                [(20, 20000 + i, 10) for i in range(n_large)])
    return ([(16, 10000 + i, 10) for i in range(n_small)] +
            [(24, 20000 + i, 16) for i in range(n_large)])


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--problem", choices=["sg", "ksg"], default="sg")
    ap.add_argument("--out", default=None)
    ap.add_argument("--n-small", type=int, default=250)
    ap.add_argument("--n-large", type=int, default=250)
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
        X, y = collect(training_specs(a.n_small, a.n_large, a.problem), a.max_nodes, a.cand,
                       a.threads, a.problem)
        if a.data:
            np.savez_compressed(a.data, X=X, y=y)
    out = a.out or DEFAULT_OUT[a.problem]
    print("collected %d rows from %d instances in %.1f s" % (len(y), a.n_small + a.n_large,
                                                             time.time() - t0), flush=True)
    t1 = time.time()
    with B.Context() as ctx:
        loss = ctx.scorer_train(X, y, epochs=a.epochs, batch=a.batch, lr=a.lr, seed=0,
                                save_path=out)
    print("trained %d epochs in %.1f s; standardised MSE first %.4f last %.4f -> %s"
          % (a.epochs, time.time() - t1, loss[0], loss[-1], out), flush=True)
    return loss


if __name__ == "__main__":
    main()
