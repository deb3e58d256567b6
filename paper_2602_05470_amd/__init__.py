"""Python binding of libbbtn (include/bbtn.h): argument marshalling only.

Every step of the branch-and-bound tensor network path runs in the HIP
library; this module converts arguments (numpy arrays, torch device tensors,
streams) into the plain pointers and sizes of the C ABI.  Importing it does
not load the library; the first call does, and fails loudly if the built
library is missing.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbbtn.so")

NEG = -(1 << 30)
NEG_CUT = -(1 << 29)
MAX_PRIMES = 32

STATUS = {0: "OK", -1: "INVALID_ARG", -2: "OOM", -3: "DEVICE", -4: "COUNT_UNCERTIFIED",
          -5: "TIMEOUT", -6: "BUFFER_TOO_SMALL", -7: "INTERNAL"}


class BBTNError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(status, "?"), status, msg))
        self.status = status


class _Options(C.Structure):
    _fields_ = [("device", C.c_int32), ("residues_per_pass", C.c_int32),
                ("max_primes", C.c_int32), ("log2_target", C.c_int32),
                ("branching", C.c_int32), ("batched", C.c_int32),
                ("region_max", C.c_int32), ("local_search", C.c_int32),
                ("graphs", C.c_int32),
                ("scorer_weights", C.c_char_p), ("autotune_cache", C.c_char_p),
                ("time_limit_s", C.c_double), ("stream", C.c_void_p),
                ("host_threads", C.c_int32), ("order_refine", C.c_int32),
                ("device_mem_cap", C.c_uint64), ("spin_flip", C.c_int32)]


class _Result(C.Structure):
    _fields_ = [("value", C.c_int64), ("n_primes", C.c_int32),
                ("primes", C.c_uint32 * MAX_PRIMES), ("residues", C.c_uint32 * MAX_PRIMES),
                ("certified", C.c_int32), ("count_words", C.c_int32),
                ("count", C.POINTER(C.c_uint32)), ("count_capacity", C.c_int32),
                ("config", C.POINTER(C.c_int8)), ("leaves", C.c_uint64),
                ("pruned", C.c_uint64), ("nodes", C.c_uint64), ("macs", C.c_uint64),
                ("seconds", C.c_double * 8)]


# numpy view of a _Result array (pointer fields read as addresses)
_RESULT_DTYPE = np.dtype({
    "names": ["value", "n_primes", "primes", "residues", "certified", "count_words", "leaves",
              "pruned", "nodes", "macs", "seconds"],
    "formats": [np.int64, np.int32, (np.uint32, MAX_PRIMES), (np.uint32, MAX_PRIMES), np.int32,
                np.int32, np.uint64, np.uint64, np.uint64, np.uint64, (np.float64, 8)],
    "offsets": [getattr(_Result, f).offset for f in
                ("value", "n_primes", "primes", "residues", "certified", "count_words", "leaves",
                 "pruned", "nodes", "macs", "seconds")],
    "itemsize": C.sizeof(_Result)})

_lib = None

EXPORTS = ["bbtn_default_options", "bbtn_create", "bbtn_destroy", "bbtn_last_error",
           "bbtn_solve_spinglass", "bbtn_solve_mwis", "bbtn_tgemm", "bbtn_tgemm_values", "bbtn_tgemm_noalloc", "bbtn_gather",
           "bbtn_reduce", "bbtn_bound", "bbtn_last_macs", "bbtn_profile",
           "bbtn_get_kernel_stats", "bbtn_profile_mask", "bbtn_mlp_forward", "bbtn_mlp_backward", "bbtn_mlp_adam",
           "bbtn_scorer_load", "bbtn_scorer_collect", "bbtn_scorer_train", "bbtn_plan_leaves",
           "bbtn_order_complexity", "bbtn_order_candidates", "bbtn_order_use",
           "bbtn_solve_batch"]

# scorer parameter layout (see include/bbtn.h)
MLP_IN, MLP_H = 32, 128
MLP_NW = MLP_H * MLP_IN + MLP_H * MLP_H + MLP_H
MLP_NB = 2 * MLP_H + 1
MLP_NPARAM = MLP_NW + MLP_NB


class _KStats(C.Structure):
    _fields_ = [("launches", C.c_uint64), ("seconds", C.c_double), ("ops", C.c_double),
                ("bytes", C.c_double)]


KERNELS = {"tgemm": 0, "persist": 1, "gather": 2, "reduce": 3, "thin": 4}


def load(path: str = LIB_PATH):
    """Load the built library (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libbbtn.so is not built (%s); run paper_2602_05470_amd.build.build()" % path)
    lib = C.CDLL(path)
    P, I32, I64, U64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64
    lib.bbtn_default_options.argtypes = [C.POINTER(_Options)]
    lib.bbtn_default_options.restype = None
    lib.bbtn_create.argtypes = [C.POINTER(_Options), C.POINTER(P)]
    lib.bbtn_create.restype = I32
    lib.bbtn_destroy.argtypes = [P]
    lib.bbtn_destroy.restype = None
    lib.bbtn_last_error.argtypes = [P]
    lib.bbtn_last_error.restype = C.c_char_p
    lib.bbtn_last_macs.argtypes = [P]
    lib.bbtn_last_macs.restype = U64
    lib.bbtn_solve_spinglass.argtypes = [P, I32, I32, P, P, P, C.POINTER(_Result)]
    lib.bbtn_solve_spinglass.restype = I32
    lib.bbtn_solve_mwis.argtypes = [P, I32, I32, P, P, C.POINTER(_Result)]
    lib.bbtn_solve_mwis.restype = I32
    lib.bbtn_solve_batch.argtypes = [P, I32, I32, P, P, P, P, P, P, P]
    lib.bbtn_solve_batch.restype = I32
    lib.bbtn_tgemm.argtypes = [P, I32, P, I64, I64, I64, I64, P, P, P, P]
    lib.bbtn_tgemm.restype = I32
    lib.bbtn_tgemm_values.argtypes = [P, I64, I64, I64, I64, P, P, P, I32, P]
    lib.bbtn_tgemm_values.restype = I32
    lib.bbtn_tgemm_noalloc.argtypes = [P, I32, P, I64, I64, I64, I64, P, P, P, P]
    lib.bbtn_tgemm_noalloc.restype = I32
    lib.bbtn_gather.argtypes = [P, I32, I32, I32, P, I64, I64, P, P, I64, P, P]
    lib.bbtn_gather.restype = I32
    lib.bbtn_reduce.argtypes = [P, I32, P, I64, I64, I64, I64, P, I64, P, P]
    lib.bbtn_reduce.restype = I32
    lib.bbtn_bound.argtypes = [P, I64, I32, P, P, P, P, I64, P, P, P, P]
    lib.bbtn_bound.restype = I32
    lib.bbtn_profile.argtypes = [P, I32]
    lib.bbtn_profile.restype = I32
    lib.bbtn_profile_mask.argtypes = [P, C.c_uint32]
    lib.bbtn_profile_mask.restype = I32
    lib.bbtn_get_kernel_stats.argtypes = [P, I32, C.POINTER(_KStats)]
    lib.bbtn_get_kernel_stats.restype = I32
    F = C.c_float
    lib.bbtn_mlp_forward.argtypes = [P, I64, P, P, P, P, P, P, P]
    lib.bbtn_mlp_forward.restype = I32
    lib.bbtn_mlp_backward.argtypes = [P, I64, P, P, P, P, P, P, P, P]
    lib.bbtn_mlp_backward.restype = I32
    lib.bbtn_mlp_adam.argtypes = [P, P, P, P, P, P, P, F, F, F, F, I32, P]
    lib.bbtn_mlp_adam.restype = I32
    lib.bbtn_scorer_load.argtypes = [P, C.c_char_p]
    lib.bbtn_scorer_load.restype = I32
    lib.bbtn_plan_leaves.argtypes = [P, I32, I32, I32, P, P, P, I32, I32, I32, I32, I32, P, I64,
                                     C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    lib.bbtn_plan_leaves.restype = I32
    lib.bbtn_order_complexity.argtypes = [I32, I32, I32, P, P, P, I32, I32, I32,
                                          C.POINTER(C.c_double), C.POINTER(C.c_int32),
                                          C.POINTER(C.c_int64)]
    lib.bbtn_order_complexity.restype = I32
    lib.bbtn_order_candidates.argtypes = [P, I32, I32, I32, P, P, P, C.POINTER(C.c_int32)]
    lib.bbtn_order_candidates.restype = I32
    lib.bbtn_order_use.argtypes = [P, I32, I32, I32, P, P, P, I32]
    lib.bbtn_order_use.restype = I32
    lib.bbtn_scorer_collect.argtypes = [P, I32, I32, I32, P, P, P, I32, I32, I32, P, P, I64,
                                        C.POINTER(C.c_int64)]
    lib.bbtn_scorer_collect.restype = I32
    lib.bbtn_scorer_train.argtypes = [P, P, P, I64, I32, I32, F, U64, P, C.c_char_p]
    lib.bbtn_scorer_train.restype = I32
    _lib = lib
    return lib


@dataclass
class Options:
    """Mirror of bbtn_options (see include/bbtn.h)."""
    device: int = 0
    residues_per_pass: int = 3
    max_primes: int = 16
    log2_target: int = 0
    branching: int = 1
    batched: int = 1
    region_max: int = 8
    local_search: int = 100
    graphs: int = 1
    scorer_weights: str | None = None
    autotune_cache: str | None = None
    time_limit_s: float = 0.0
    stream: int | None = None
    host_threads: int = 0
    order_refine: int = 0
    device_mem_cap: int = 0
    spin_flip: int = 0

    def _c(self):
        o = _Options()
        load().bbtn_default_options(C.byref(o))
        for f in ("device", "residues_per_pass", "max_primes", "log2_target", "branching",
                  "batched", "region_max", "local_search", "graphs", "time_limit_s",
                  "host_threads", "order_refine", "device_mem_cap", "spin_flip"):
            setattr(o, f, getattr(self, f))
        o.scorer_weights = self.scorer_weights.encode() if self.scorer_weights else None
        o.autotune_cache = self.autotune_cache.encode() if self.autotune_cache else None
        o.stream = self.stream
        return o


@dataclass
class Result:
    value: int
    count: int
    certified: bool
    primes: list
    residues: list
    config: np.ndarray
    leaves: int
    pruned: int
    nodes: int
    macs: int
    seconds: list = field(default_factory=list)


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _stream(s):
    """hipStream_t for a kernel-level call: the given stream (torch stream or
    int handle), else torch's current stream when torch is in use (its
    default stream is handle 0, the null stream)."""
    if s is None:
        import sys
        torch = sys.modules.get("torch")
        if torch is not None and torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
        return None
    if isinstance(s, int):
        return C.c_void_p(s)
    return C.c_void_p(s.cuda_stream)


def _dptr(t):
    """Device pointer of a torch tensor (or an int address)."""
    if t is None:
        return None
    if isinstance(t, int):
        return C.c_void_p(t)
    return C.c_void_p(t.data_ptr())


class Context:
    """bbtn_ctx: a device context with its workspace and stream."""

    def __init__(self, options: Options | None = None):
        self.lib = load()
        self.options = options or Options()
        self._o = self.options._c()
        h = C.c_void_p()
        s = self.lib.bbtn_create(C.byref(self._o), C.byref(h))
        if s != 0:
            raise BBTNError(s, "bbtn_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.bbtn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, s):
        if s != 0:
            raise BBTNError(s, self.lib.bbtn_last_error(self.h).decode())

    def last_macs(self):
        return int(self.lib.bbtn_last_macs(self.h))

    def profile(self, enable=True, kernels=None):
        """bbtn_profile: start (and clear) or stop per-kernel event timing;
        with `kernels` (names), bbtn_profile_mask: only those kernels."""
        if kernels is None or not enable:
            self._check(self.lib.bbtn_profile(self.h, 1 if enable else 0))
        else:
            mask = 0
            for k in kernels:
                mask |= 1 << KERNELS[k]
            self._check(self.lib.bbtn_profile_mask(self.h, mask))

    def kernel_stats(self, kernel):
        """bbtn_get_kernel_stats: dict(launches, seconds, ops, bytes)."""
        st = _KStats()
        self._check(self.lib.bbtn_get_kernel_stats(self.h, KERNELS.get(kernel, kernel), C.byref(st)))
        return dict(launches=int(st.launches), seconds=st.seconds, ops=st.ops, bytes=st.bytes)

    # -------------------------------------------------------------- solves
    def _solve(self, fn, n, edges, *arrays, raise_uncertified=True):
        edges = _i32(edges).reshape(-1, 2)
        r = _Result()
        cap = (n + 64) // 32 + 2
        cnt = (C.c_uint32 * cap)()
        cfg = np.zeros(n, dtype=np.int8)
        r.count = C.cast(cnt, C.POINTER(C.c_uint32))
        r.count_capacity = cap
        r.config = cfg.ctypes.data_as(C.POINTER(C.c_int8))
        arrs = [None if a is None else _i32(a) for a in arrays]
        s = fn(self.h, n, len(edges), _ptr(edges), *[_ptr(a) for a in arrs], C.byref(r))
        if s != 0 and not (s == -4 and not raise_uncertified):
            self._check(s)
        count = 0
        for i in reversed(range(r.count_words)):
            count = (count << 32) | int(cnt[i])
        return Result(value=int(r.value), count=count, certified=bool(r.certified),
                      primes=[int(r.primes[i]) for i in range(r.n_primes)],
                      residues=[int(r.residues[i]) for i in range(r.n_primes)],
                      config=cfg, leaves=int(r.leaves), pruned=int(r.pruned),
                      nodes=int(r.nodes), macs=int(r.macs), seconds=list(r.seconds))

    def solve_batch(self, kind, instances, raise_failed=True):
        """bbtn_solve_batch: instances is a list of (n, edges, weights, h)
        (kind 0: spin glass, weights = J; kind 1: MWIS, weights = w or None,
        h ignored).  Returns (results, statuses)."""
        N = len(instances)
        M = max(N, 1)
        ns = np.zeros(M, np.int32)
        ms = np.zeros(M, np.int32)
        ptrs = np.zeros((3, M), np.uint64)  # edge, weight and field pointers
        keep = []
        for i, (n, edges, w, h) in enumerate(instances):
            e = _i32(edges)
            ns[i], ms[i] = n, e.size // 2
            ptrs[0, i] = e.ctypes.data
            keep.append(e)
            if w is not None:
                ww = _i32(w)
                ptrs[1, i] = ww.ctypes.data
                keep.append(ww)
            if h is not None and kind == 0:
                hh = _i32(h)
                ptrs[2, i] = hh.ctypes.data
                keep.append(hh)
        # one buffer for every count and one for every configuration
        cap = int(ns.max() + 64) // 32 + 2 if N else 1
        counts = np.zeros((M, cap), np.uint32)
        nmax = int(ns.max()) if N else 1
        cfgs = np.zeros((M, max(nmax, 1)), np.int8)
        res = (_Result * M)()
        cbase, fbase = counts.ctypes.data, cfgs.ctypes.data
        u32p, i8p = C.POINTER(C.c_uint32), C.POINTER(C.c_int8)
        for i in range(N):
            r = res[i]
            r.count = C.cast(cbase + 4 * cap * i, u32p)
            r.count_capacity = cap
            r.config = C.cast(fbase + cfgs.shape[1] * i, i8p)
        st = np.zeros(M, np.int32)
        s = self.lib.bbtn_solve_batch(self.h, kind, N, ns.ctypes.data, ms.ctypes.data,
                                      ptrs[0].ctypes.data, ptrs[1].ctypes.data,
                                      ptrs[2].ctypes.data, res, st.ctypes.data)
        statuses = st[:N].tolist()
        if s != 0 and raise_failed:
            self._check(s)
        # read the results through one structured view of the array
        ra = np.frombuffer(res, dtype=_RESULT_DTYPE)
        vals, cws, certs, nps = (ra["value"].tolist(), ra["count_words"].tolist(),
                                 ra["certified"].tolist(), ra["n_primes"].tolist())
        primes, resid, secs = ra["primes"].tolist(), ra["residues"].tolist(), ra["seconds"].tolist()
        lv, pr, nd, mc = (ra["leaves"].tolist(), ra["pruned"].tolist(), ra["nodes"].tolist(),
                          ra["macs"].tolist())
        out = []
        for i in range(N):
            cw = cws[i]
            count = int.from_bytes(counts[i, :cw].tobytes(), "little") if cw > 0 else 0
            out.append(Result(value=vals[i], count=count, certified=bool(certs[i]),
                              primes=primes[i][:nps[i]], residues=resid[i][:nps[i]],
                              config=cfgs[i, :int(ns[i])], leaves=lv[i], pruned=pr[i],
                              nodes=nd[i], macs=mc[i], seconds=secs[i]))
        return out, statuses

    def solve_spinglass(self, n, edges, J, h=None, **kw) -> Result:
        """bbtn_solve_spinglass: E0 = min H (Eq. 1), exact degeneracy, one
        ground configuration (sigma in {-1,+1})."""
        return self._solve(self.lib.bbtn_solve_spinglass, n, edges, J, h, **kw)

    def solve_mwis(self, n, edges, w=None, **kw) -> Result:
        """bbtn_solve_mwis: W*, number of maximum-weight independent sets,
        one of them (x in {0,1})."""
        return self._solve(self.lib.bbtn_solve_mwis, n, edges, w, **kw)

    def order_candidates(self, kind, n, edges, weights=None, h=None) -> int:
        """bbtn_order_candidates: build and rank the candidate contraction
        orders of the instance's structure on this context; their number."""
        e = _i32(edges).reshape(-1, 2)
        w = None if weights is None else _i32(weights)
        hh = None if h is None else _i32(h)
        cnt = C.c_int32(0)
        self._check(self.lib.bbtn_order_candidates(self.h, kind, n, len(e), _ptr(e), _ptr(w),
                                                   _ptr(hh), C.byref(cnt)))
        return cnt.value

    def order_use(self, kind, n, edges, weights=None, h=None, which=0):
        """bbtn_order_use: make candidate `which` the structure's order."""
        e = _i32(edges).reshape(-1, 2)
        w = None if weights is None else _i32(weights)
        hh = None if h is None else _i32(h)
        self._check(self.lib.bbtn_order_use(self.h, kind, n, len(e), _ptr(e), _ptr(w), _ptr(hh),
                                            int(which)))

    # ------------------------------------------------------- kernel entries
    def tgemm(self, k, primes, batch, M, N, K, A, B, Cout, stream=None):
        """bbtn_tgemm on device tensor buffers (torch tensors, int32 words)."""
        pr = (C.c_uint32 * k)(*[int(p) for p in primes[:k]])
        self._check(self.lib.bbtn_tgemm(self.h, k, pr, batch, M, N, K, _dptr(A), _dptr(B),
                                        _dptr(Cout), _stream(stream)))

    def tgemm_values(self, batch, M, N, K, A, B, Cout, max_abs, stream=None):
        """bbtn_tgemm_values: max-plus product of int32 value planes; max_abs
        bounds |v| of the finite values (below 2^12: packed 16-bit path)."""
        self._check(self.lib.bbtn_tgemm_values(self.h, batch, M, N, K, _dptr(A), _dptr(B),
                                               _dptr(Cout), int(max_abs), _stream(stream)))

    def tgemm_noalloc(self, k, primes, batch, M, N, K, A, B, Cout, stream=None):
        """bbtn_tgemm_noalloc: bbtn_tgemm with no device allocation (split-K
        partials in the library's static device scratch)."""
        pr = (C.c_uint32 * k)(*[int(p) for p in primes[:k]])
        self._check(self.lib.bbtn_tgemm_noalloc(self.h, k, pr, batch, M, N, K, _dptr(A),
                                                _dptr(B), _dptr(Cout), _stream(stream)))

    def gather(self, k, r_in, r_out, src_bits, L, in_stride, fixed_bits, inp, in_entries, out,
               stream=None):
        """bbtn_gather (permutation + branch-variable fixing)."""
        sb = (C.c_int32 * max(1, r_out))(*[int(b) for b in src_bits])
        self._check(self.lib.bbtn_gather(self.h, k, r_in, r_out, sb, L, in_stride,
                                         _dptr(fixed_bits), _dptr(inp), in_entries, _dptr(out),
                                         _stream(stream)))

    def reduce(self, k, primes, outer, S, seg_stride, elem_stride, inp, in_entries, out,
               stream=None):
        """bbtn_reduce (segmented tropical sum)."""
        pr = (C.c_uint32 * k)(*[int(p) for p in primes[:k]])
        self._check(self.lib.bbtn_reduce(self.h, k, pr, outer, S, seg_stride, elem_stride,
                                         _dptr(inp), in_entries, _dptr(out), _stream(stream)))

    def bound(self, n_branch, T, values, tensor_off, tensor_len, offset, incumbent, bound,
              keep_idx, n_keep, stream=None):
        """bbtn_bound (branch bounds + compaction of kept branches)."""
        self._check(self.lib.bbtn_bound(self.h, n_branch, T, _dptr(values), _dptr(tensor_off),
                                        _dptr(tensor_len), _dptr(offset), int(incumbent),
                                        _dptr(bound), _dptr(keep_idx), _dptr(n_keep),
                                        _stream(stream)))

    # ------------------------------------------------------------- scorer
    def mlp_forward(self, rows, X, W, bias, y, h1=None, h2=None, stream=None):
        """bbtn_mlp_forward on device tensors (X, W: int16/bfloat16 bits)."""
        self._check(self.lib.bbtn_mlp_forward(self.h, rows, _dptr(X), _dptr(W), _dptr(bias),
                                              _dptr(y), _dptr(h1), _dptr(h2), _stream(stream)))

    def mlp_backward(self, rows, X, W, y, t, h1, h2, grad, stream=None):
        """bbtn_mlp_backward: grad receives [dW | db | sum of squared errors]."""
        self._check(self.lib.bbtn_mlp_backward(self.h, rows, _dptr(X), _dptr(W), _dptr(y),
                                               _dptr(t), _dptr(h1), _dptr(h2), _dptr(grad),
                                               _stream(stream)))

    def mlp_adam(self, master, W, bias, m, v, grad, lr, beta1, beta2, eps, step, stream=None):
        """bbtn_mlp_adam: one bias-corrected Adam step."""
        self._check(self.lib.bbtn_mlp_adam(self.h, _dptr(master), _dptr(W), _dptr(bias), _dptr(m),
                                           _dptr(v), _dptr(grad), lr, beta1, beta2, eps, step,
                                           _stream(stream)))

    def scorer_load(self, path):
        """bbtn_scorer_load."""
        self._check(self.lib.bbtn_scorer_load(self.h, path.encode()))

    def scorer_collect(self, kind, n, edges, weights, h=None, log2_target=10, max_nodes=64,
                       cand_per_node=8):
        """bbtn_scorer_collect -> (X [rows, 32] float32, y [rows] float32)."""
        edges = _i32(edges).reshape(-1, 2)
        w = None if weights is None else _i32(weights)
        hh = None if h is None else _i32(h)
        rows = C.c_int64(0)
        args = (self.h, kind, n, len(edges), _ptr(edges), _ptr(w), _ptr(hh), log2_target,
                max_nodes, cand_per_node)
        self._check(self.lib.bbtn_scorer_collect(*args, None, None, 0, C.byref(rows)))
        X = np.zeros((rows.value, MLP_IN), np.float32)
        y = np.zeros(rows.value, np.float32)
        if rows.value:
            self._check(self.lib.bbtn_scorer_collect(*args, _ptr(X), _ptr(y), rows.value,
                                                     C.byref(rows)))
        return X, y

    def scorer_train(self, X, y, epochs=20, batch=1024, lr=1e-3, seed=0, save_path=None):
        """bbtn_scorer_train -> per-epoch standardised MSE."""
        X = np.ascontiguousarray(X, np.float32)
        y = np.ascontiguousarray(y, np.float32)
        loss = np.zeros(epochs, np.float32)
        self._check(self.lib.bbtn_scorer_train(self.h, _ptr(X), _ptr(y), len(y), epochs, batch,
                                               lr, seed, _ptr(loss),
                                               save_path.encode() if save_path else None))
        return loss


def plan_leaves(kind, n, edges, weights, h=None, log2_target=10, region_max=8, local_search=100,
                values_only=False, order_refine=0):
    """bbtn_plan_leaves without a device context: the leaves of the
    branch-and-bound search as an int8 array [leaves, n] (-1 = free, else the
    fixed state), and the local-search incumbent's value (None if none)."""
    lib = load()
    edges = _i32(edges).reshape(-1, 2)
    w = None if weights is None else _i32(weights)
    hh = None if h is None else _i32(h)
    nl = C.c_int64(0)
    inc = C.c_int64(0)
    args = (None, kind, n, len(edges), _ptr(edges), _ptr(w), _ptr(hh), log2_target, region_max,
            local_search, int(bool(values_only)), order_refine)
    s = lib.bbtn_plan_leaves(*args, None, 0, C.byref(nl), C.byref(inc))
    if s != 0:
        raise BBTNError(s, "bbtn_plan_leaves failed")
    out = np.zeros((nl.value, n), np.int8)
    if nl.value:
        s = lib.bbtn_plan_leaves(*args, out.ctypes.data_as(C.c_void_p), nl.value, C.byref(nl),
                                 C.byref(inc))
        if s != 0:
            raise BBTNError(s, "bbtn_plan_leaves failed")
    incumbent = None if inc.value == -(1 << 63) else int(inc.value)
    return out, incumbent


def order_complexity(kind, n, edges, weights, h=None, order_refine=0, log2_target=10,
                     region_max=8):
    """bbtn_order_complexity: (tc_log2, sc, rho) of the contraction order the
    planner uses for the instance (host only)."""
    lib = load()
    edges = _i32(edges).reshape(-1, 2)
    w = None if weights is None else _i32(weights)
    hh = None if h is None else _i32(h)
    tc = C.c_double(0)
    sc = C.c_int32(0)
    rho = C.c_int64(0)
    s = lib.bbtn_order_complexity(kind, n, len(edges), _ptr(edges), _ptr(w), _ptr(hh),
                                  order_refine, log2_target, region_max, C.byref(tc),
                                  C.byref(sc), C.byref(rho))
    if s != 0:
        raise BBTNError(s, "bbtn_order_complexity failed")
    return tc.value, sc.value, rho.value


def scorer_collect(kind, n, edges, weights, h=None, log2_target=10, max_nodes=64, cand_per_node=8):
    """bbtn_scorer_collect without a device context (host-only search)."""
    lib = load()
    edges = _i32(edges).reshape(-1, 2)
    w = None if weights is None else _i32(weights)
    hh = None if h is None else _i32(h)
    rows = C.c_int64(0)
    args = (None, kind, n, len(edges), _ptr(edges), _ptr(w), _ptr(hh), log2_target, max_nodes,
            cand_per_node)
    s = lib.bbtn_scorer_collect(*args, None, None, 0, C.byref(rows))
    if s != 0:
        raise BBTNError(s, "bbtn_scorer_collect failed")
    X = np.zeros((rows.value, MLP_IN), np.float32)
    y = np.zeros(rows.value, np.float32)
    if rows.value:
        s = lib.bbtn_scorer_collect(*args, _ptr(X), _ptr(y), rows.value, C.byref(rows))
        if s != 0:
            raise BBTNError(s, "bbtn_scorer_collect failed")
    return X, y
