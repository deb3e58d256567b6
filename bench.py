"""Benchmark: exact (E0, degeneracy) instances per hour on one MI355X.

Workload (the configuration the headline metric is quoted on): +-J spin glass
on a 16 x 16 open-boundary lattice, couplings +-1 from numpy seeds 0-319, zero
field; plain BBTN with T_target = 2^10 (greedy contraction order, branching on
separator spins), counts as residues modulo 3 primes per pass, CRT-certified.
One step = one call through the C ABI that fully solves --batch-size
instances (default 160 distinct seeds, bbtn_solve_batch): network build,
search, values-only pass, counting pass, CRT and certification,
configuration recovery; --workers contexts (default 3) run steps
concurrently.  Every result is checked against the oracle's stored exact
values; only exact, certified results are counted.

The JSON line also carries
  roofline:      the dominant kernel's semiring operations per second (events
                 around its executor passes on its own stream, over the timed
                 steps) against the VALU integer peak, and its HBM bytes per
                 pass from the stored counter summary;
  refined_order: the same run with the contraction order refined by
                 annealing (order_refine = 8);
  per_branch:    the same solves with one branch at a time (batched = 0);
  cpu_baseline:  the CPU oracle (exact transfer matrix in C, all host
                 threads) timed on a bounded sample of the same instances on
                 this host;
  tgemm_micro:   the counting tropical product alone at large shapes.

--large N prints instead exact solves of the 32 x 32 spin glass and the
40 x 40 King's subgraph (refined order; plain planner and learned scorer).
"""
import argparse
import json
import os
import subprocess
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 64 int32 lanes x 2.4 GHz (one VALU op per lane per clock)
VALU_PEAK_OPS = 256 * 64 * 2.4e9
HBM_PEAK = 8.0e12


# Per-launch HBM traffic of the persistent executor, measured by rocprofv3
# --pmc FETCH_SIZE and WRITE_SIZE on this workload and recorded, with a hash
# of the kernel sources, in a profiles/ summary; reported only while the
# sources are unchanged.
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "persist_sg16_batch160_hbm_traffic.md")
PERSIST_SOURCES = [os.path.join(ROOT, "paper_2602_05470_amd", "csrc", f)
                   for f in ("k_persist.hip", "persist_dev.h", "persist.cpp")]


def persist_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in PERSIST_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def persist_traffic():
    """HBM bytes per persistent-executor launch, or None when no summary
    matches the current kernel sources."""
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    fields = {}
    for line in open(TRAFFIC_SUMMARY):
        if ":" in line and line.strip().startswith(("kernel-sources-sha256", "hbm-bytes-per-launch")):
            key, val = line.strip().split(":", 1)
            fields[key.strip()] = val.strip().strip("`")
    if fields.get("kernel-sources-sha256") != persist_sources_sha256():
        return None
    return int(fields["hbm-bytes-per-launch"])


N_SEEDS = 320  # 16x16 instances with stored exact values (seeds 0-319)


def golden_sg16():
    out = {}
    for fn in ("sg16.txt", "sg16_more.txt"):
        for line in open(os.path.join(ROOT, "tests", "golden", fn)):
            if line.startswith("#") or not line.strip():
                continue
            s, e, d = (int(x) for x in line.split())
            out[s] = (e, d)
    assert sorted(out) == list(range(N_SEEDS))
    return out


def cpu_baseline(gold, seconds_budget=10.0):
    """Time the oracle's C transfer matrix (exact multiword counts, OpenMP over
    all host threads) on seeds 0-19, repeated until the budget is spent; every
    result is checked against the stored exact values."""
    import instances as I
    from oracle import tm_c
    insts = [I.spin_glass_square(16, s) for s in range(20)]
    def solve(g):
        return tm_c.spin_glass_lattice(16, 16, g["edges"], g["J"])
    solve(insts[0])  # load (and build if needed) outside the clock
    t0 = time.time()
    n = 0
    while n < 20 or time.time() - t0 < seconds_budget:
        s = n % 20
        if solve(insts[s]) != gold[s]:
            raise RuntimeError("oracle disagrees with the stored value for seed %d" % s)
        n += 1
    dt = time.time() - t0
    return {"value": round(3600.0 * n / dt, 1), "unit": "instances/hour",
            "cores": tm_c.threads(), "kind": "oracle",
            "sample": "16x16 +-J seeds 0-19 (%d solves), exact transfer matrix in C with "
                      "OpenMP, %.1f s" % (n, dt)}


def tgemm_micro(B, ctx, torch):
    """Counting tropical product alone (k = 3) at large shapes."""
    import numpy as np
    import instances as I
    res = []
    for (b, M, N, K) in [(1, 4096, 4096, 256), (1, 2048, 2048, 2048)]:
        k = 3
        primes = I.PRIMES_31[:k]
        rng = np.random.default_rng(0)

        def buf(E):
            v = rng.integers(-8, 9, size=E).astype(np.int32)
            neg = rng.random(E) < 0.25
            v[neg] = I.NEG
            r = np.stack([rng.integers(0, p, size=E, dtype=np.uint64).astype(np.uint32)
                          for p in primes])
            r[:, neg] = 0
            return torch.from_numpy(np.concatenate([v, r.view(np.int32).reshape(-1)])).cuda()
        A, Bm = buf(b * M * K), buf(b * K * N)
        Cm = torch.empty((1 + k) * b * M * N, dtype=torch.int32, device="cuda")
        ctx.tgemm(k, primes, b, M, N, K, A, Bm, Cm)
        torch.cuda.synchronize()
        ctx.profile(True)
        for _ in range(3):
            ctx.tgemm(k, primes, b, M, N, K, A, Bm, Cm)
        torch.cuda.synchronize()
        st = ctx.kernel_stats("tgemm")
        ctx.profile(False)
        ops = st["ops"] / max(st["seconds"], 1e-12)
        res.append({"shape_bMNK": [b, M, N, K], "k": k,
                    "ms": round(1e3 * st["seconds"] / max(st["launches"], 1), 3),
                    "Gop_s": round(ops / 1e9, 1), "frac_valu": round(ops / VALU_PEAK_OPS, 4)})
    return res


def large_configs(B, I, torch, n_seeds):
    """Exact solves of the larger lattices, one instance per call, with the
    refined contraction order (chosen on the first seed and cached), by the
    plain planner and by the shipped learned scorer."""
    here = os.path.dirname(os.path.abspath(__file__))
    out = {}
    for name, make, kind, t, k, weights in (
            ("sg32x32", lambda s: I.spin_glass_square(32, s), 0, 26, 3, "scorer_sg.bin"),
            ("ksg40x40", lambda s: I.kings_subgraph(40, s), 1, 24, 4, "scorer_ksg.bin")):
        out[name] = {"T_target_log2": t, "residues_per_pass": k}
        for variant, branching in (("plain", 1), ("scorer", 2)):
            wpath = os.path.join(here, "paper_2602_05470_amd", weights) if branching == 2 else None
            ctx = B.Context(B.Options(log2_target=t, order_refine=8, residues_per_pass=k,
                                      branching=branching, scorer_weights=wpath))
            rows = []
            for s in range(n_seeds):
                g = make(s)
                print("large %s %s seed %d" % (name, variant, s), file=sys.stderr, flush=True)
                if s == 1:
                    ctx.profile(True)   # kernel figures over the seeds after the first
                t0 = time.perf_counter()
                if kind == 0:
                    r = ctx.solve_spinglass(g["n"], g["edges"], g["J"])
                else:
                    r = ctx.solve_mwis(g["n"], g["edges"], g["w"])
                torch.cuda.synchronize()
                rows.append({"seed": s, "value": r.value, "count": str(r.count),
                             "certified": bool(r.certified), "leaves": int(r.leaves),
                             "macs": int(r.macs), "seconds": round(time.perf_counter() - t0, 3)})
                print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
            ks = {}
            for kn in ("tgemm", "persist", "gather"):
                st = ctx.kernel_stats(kn)
                ks[kn] = {"launches": st["launches"], "seconds": round(st["seconds"], 4),
                          "Gop_s": round(st["ops"] / max(st["seconds"], 1e-12) / 1e9, 1),
                          "frac_valu": round(st["ops"] / max(st["seconds"], 1e-12) / VALU_PEAK_OPS, 4),
                          "GB_s": round(st["bytes"] / max(st["seconds"], 1e-12) / 1e9, 1)}
            ctx.profile(False)
            ctx.close()
            later = rows[1:] or rows
            out[name][variant] = {
                "instances": rows,
                "mean_seconds_after_first": round(sum(r["seconds"] for r in later) / len(later), 3),
                "total_macs": sum(r["macs"] for r in rows),
                "kernels": ks}
        same = all((a["value"], a["count"]) == (b["value"], b["count"])
                   for a, b in zip(out[name]["plain"]["instances"], out[name]["scorer"]["instances"]))
        out[name]["scorer_results_identical"] = same
    return {"large_configs": out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=24)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-micro", action="store_true")
    ap.add_argument("--no-per-branch", action="store_true")
    ap.add_argument("--micro-only", action="store_true",
                    help="only the counting-product micro-benchmark and a copy of known size "
                         "(for hardware-counter runs)")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="end with a plain device copy of known size (512 MiB each way), "
                         "the reference that scales hardware byte counters")
    ap.add_argument("--batched", type=int, default=1)
    ap.add_argument("--workers", type=int, default=3,
                    help="concurrent solver contexts (threads, one stream each): one "
                         "call's host planning overlaps another's contraction")
    ap.add_argument("--host-threads", type=int, default=0,
                    help="planning threads per call; 0: all host threads with one context, "
                         "half of them with several")
    ap.add_argument("--order-refine", type=int, default=0,
                    help="contraction order of the main run: 0 = greedy (the workload's "
                         "plain BBTN); n > 0 = best of greedy and n annealed refinements")
    ap.add_argument("--no-refined-order", action="store_true",
                    help="skip the second run of the same workload with a refined order")
    ap.add_argument("--large", type=int, default=0,
                    help="instead of the throughput run: solve this many seeds each of the "
                         "+-J 32x32 lattice (T_target=2^26) and the King's subgraph 40x40 MIS "
                         "(T_target=2^24) with the refined order, by the plain planner and by "
                         "the learned scorer, and print their times and kernel figures")
    ap.add_argument("--batch-size", type=int, default=160,
                    help="instances per call (bbtn_solve_batch when > 1): their branch "
                         "sub-networks share every device launch")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the solver path is single-GPU "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    import paper_2602_05470_amd as B
    import instances as I
    if args.micro_only:
        ctx = B.Context(B.Options())
        res = tgemm_micro(B, ctx, torch)
        # a plain device copy of known size (512 MiB read + 512 MiB written):
        # the reference that scales the hardware byte counters
        x = torch.ones(128 << 20, dtype=torch.int32, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        ctx.close()
        print(json.dumps({"tgemm_micro": res, "copy_bytes_each_way": 512 << 20}), flush=True)
        return
    if args.large > 0:
        print(json.dumps(large_configs(B, I, torch, args.large)), flush=True)
        return
    want = golden_sg16()
    insts = [I.spin_glass_square(16, s) for s in range(N_SEEDS)]
    # the contexts share the host: each plans its instances on half the
    # host threads when several run at once (unless --host-threads is given)
    ncpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    host_threads = args.host_threads if args.host_threads > 0 else (
        ncpu if args.workers <= 1 else max(1, ncpu // 2))
    opts = B.Options(log2_target=10, residues_per_pass=3, branching=1, batched=args.batched,
                     host_threads=host_threads, order_refine=args.order_refine)
    T = max(1, args.workers)
    Bsz = max(1, args.batch_size)
    ctxs = [B.Context(opts) for _ in range(T)]

    def solve_step(c, i):
        """Step i: instances i*Bsz .. i*Bsz+Bsz-1 (seeds mod 320), one call."""
        seeds = [(i * Bsz + j) % N_SEEDS for j in range(Bsz)]
        if Bsz == 1:
            g = insts[seeds[0]]
            return seeds, [c.solve_spinglass(g["n"], g["edges"], g["J"])]
        rs, _ = c.solve_batch(0, [(insts[s]["n"], insts[s]["edges"], insts[s]["J"], None)
                                  for s in seeds])
        return seeds, rs

    def timed(cs, profile):
        """Warm-up steps on every context (workspace growth, code loading, the
        order cache), then `steps` calls shared by the contexts' threads."""
        for c in cs:
            for i in range(args.warmup):
                solve_step(c, i)
            if profile:
                c.profile(True)
        torch.cuda.synchronize()
        lock = threading.Lock()
        nxt = [0]
        res = [None] * args.steps
        lat = [0.0] * args.steps

        def worker(c):
            while True:
                with lock:
                    i = nxt[0]
                    nxt[0] += 1
                if i >= args.steps:
                    return
                ts = time.perf_counter()
                res[i] = solve_step(c, i)
                lat[i] = time.perf_counter() - ts

        r0 = os.times()
        ta = time.perf_counter()
        if len(cs) == 1:
            worker(cs[0])
        else:
            th = [threading.Thread(target=worker, args=(c,)) for c in cs]
            for t in th:
                t.start()
            for t in th:
                t.join()
        torch.cuda.synchronize()
        tb = time.perf_counter()
        r1 = os.times()
        return res, lat, tb - ta, (r1.user - r0.user) + (r1.system - r0.system)

    results, call_s, dt, host_cpu_s = timed(ctxs, True)
    exact = 0
    leaves = 0
    n_inst = 0
    phases = [0.0] * 8
    for i, (seeds, rs) in enumerate(results):
        for s, r in zip(seeds, rs):
            n_inst += 1
            leaves += r.leaves
            phases = [a + b for a, b in zip(phases, r.seconds)]
            ok = (r.value, r.count) == want[s] and r.certified
            exact += ok
            print("step %d seed %d E0=%d deg=%d leaves=%d %s" % (i, s, r.value, r.count, r.leaves,
                  "exact" if ok else "MISMATCH"), file=sys.stderr, flush=True)
    stats = {}
    for name in ("tgemm", "persist", "gather"):
        agg = {"launches": 0, "seconds": 0.0, "ops": 0.0, "bytes": 0.0}
        for c in ctxs:
            ks = c.kernel_stats(name)
            for key in agg:
                agg[key] += ks[key]
        stats[name] = agg
    for c in ctxs:
        c.profile(False)
    ctx = ctxs[0]
    dom = max(stats, key=lambda n: stats[n]["seconds"])
    st = stats[dom]
    achieved = st["ops"] / max(st["seconds"], 1e-12)
    line = {
        "metric": "exact (E0,degeneracy) instances/hour",
        "value": round(3600.0 * exact / dt, 1),
        "unit": "instances/hour",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * dt / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "+-J spin glass 16x16 open lattice, seeds 0-319, zero field, "
                               "plain BBTN T_target=2^10, 3 primes per pass; one step = one "
                               "call solving %d instance(s), %d concurrent contexts" % (Bsz, T),
                   "instances": n_inst, "exact": exact,
                   "leaves_per_instance": round(leaves / max(n_inst, 1), 1),
                   "batched": args.batched, "batch_size": Bsz, "workers": T,
                   "host_threads_per_context": host_threads,
                   "contraction_order": "greedy" if args.order_refine == 0 else
                                        "refined (%d candidates)" % args.order_refine},
        "roofline": {"bound": "alu", "kernel": dom,
                     "achieved": round(achieved / 1e12, 4), "peak": round(VALU_PEAK_OPS / 1e12, 2),
                     "unit": "TOP/s", "frac": round(achieved / VALU_PEAK_OPS, 5),
                     "traffic": persist_traffic() if dom == "persist" else None,
                     "launches": st["launches"],
                     "launch_unit": "one executor pass (its shared-subtree and branch dispatches)"
                                    if dom == "persist" else "one kernel dispatch",
                     "avg_launch_ms": round(1e3 * st["seconds"] / max(st["launches"], 1), 4),
                     "kernel_busy_share": round(st["seconds"] / dt, 4)},
        "kernels": {n: {"launches": s["launches"], "seconds": round(s["seconds"], 5),
                        "Gop_s": round(s["ops"] / max(s["seconds"], 1e-12) / 1e9, 2),
                        "GB_s": round(s["bytes"] / max(s["seconds"], 1e-12) / 1e9, 2)}
                    for n, s in stats.items()},
    }
    # host CPU time of the process over the timed region, as a share of
    # the wall time of all the host threads it may run on
    ncpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    line["host_cpu"] = {"seconds": round(host_cpu_s, 3), "cpus": ncpu,
                        "utilisation": round(host_cpu_s / max(dt * ncpu, 1e-9), 3)}
    names = ["total", "build+plan", "search", "contraction", "crt+certification", "configuration"]
    # latency of one call (all its instances), over the timed steps; an
    # instance counts as unsolved when its result is not exact and certified
    cs = sorted(call_s)
    line["latency_ms"] = {"per_call_p50": round(1e3 * cs[len(cs) // 2], 3),
                          "per_call_max": round(1e3 * cs[-1], 3),
                          "unsolved": n_inst - exact}
    line["phases_ms"] = {nm: round(1e3 * phases[i] / max(n_inst, 1), 3)
                         for i, nm in enumerate(names)}
    if not args.no_refined_order and args.order_refine == 0:
        # the same workload and settings with the contraction order refined
        # by annealing (8 candidates, chosen once for the lattice during the
        # warm-up): fewer and cheaper leaves
        ro = B.Options(log2_target=10, residues_per_pass=3, branching=1, batched=args.batched,
                       host_threads=host_threads, order_refine=8)
        rctx = [B.Context(ro) for _ in range(T)]
        rres, rlat, rdt, rcpu = timed(rctx, False)
        for c in rctx:
            c.close()
        r_ok = r_n = r_leaves = 0
        for seeds, rs in rres:
            for s_, r in zip(seeds, rs):
                r_n += 1
                r_leaves += r.leaves
                r_ok += (r.value, r.count) == want[s_] and r.certified
        line["refined_order"] = {
            "value": round(3600.0 * r_ok / rdt, 1), "unit": "instances/hour",
            "instances": r_n, "exact": r_ok,
            "leaves_per_instance": round(r_leaves / max(r_n, 1), 1),
            "ms_per_step": round(1e3 * rdt / args.steps, 3),
            "host_cpu_utilisation": round(rcpu / max(rdt * ncpu, 1e-9), 3),
            "note": "order_refine=8: best of the greedy tree and 8 annealed refinements, "
                    "scored by a probe search"}
    if not args.no_per_branch:
        # the same path without batching: one branch at a time (step programs
        # replayed from a hipGraph), on the first instances
        pb = B.Context(B.Options(log2_target=10, residues_per_pass=3, branching=1, batched=0))
        g = insts[0]
        pb.solve_spinglass(g["n"], g["edges"], g["J"])
        n_pb = 3
        t2 = time.perf_counter()
        ok = 0
        for i in range(n_pb):
            g = insts[i]
            r = pb.solve_spinglass(g["n"], g["edges"], g["J"])
            ok += (r.value, r.count) == want[i] and r.certified
        t3 = time.perf_counter()
        pb.close()
        line["per_branch"] = {"value": round(3600.0 * ok / (t3 - t2), 1), "unit": "instances/hour",
                              "instances": n_pb, "exact": ok,
                              "note": "batched=0: branches contracted one at a time"}
    if not args.no_micro:
        line["tgemm_micro"] = tgemm_micro(B, ctx, torch)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(want)
    for c in ctxs:
        c.close()
    if args.calibration_copy:
        x = torch.ones(128 << 20, dtype=torch.int32, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        line["calibration_copy_bytes_each_way"] = 512 << 20
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
