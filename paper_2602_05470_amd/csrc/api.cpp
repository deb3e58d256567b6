// C ABI of the library (include/bbtn.h) and the solve driver:
// build network -> contraction tree -> branch-and-bound search -> batched
// contraction of every branch sub-network per prime pass -> tropical sum of
// the branch results -> CRT + certification -> one optimal configuration.
#include <chrono>
#include <cmath>
#include <cstring>
#include <fstream>
#include <future>

#include "crt.h"
#include "ctx.h"
#include "exec.h"
#include "persist.h"
#include "scorer.h"
#include "search.h"
#include "solve.h"
#include "trace.h"

using namespace bbtn;

namespace {

template <class F>
bbtn_status guard(bbtn_ctx* ctx, F&& f) {
  try {
    f();
    if (ctx) ctx->err.clear();
    return BBTN_OK;
  } catch (const Error& e) {
    if (ctx) ctx->err = e.what();
    return e.status;
  } catch (const std::bad_alloc&) {
    if (ctx) ctx->err = "host allocation failed";
    return BBTN_E_OOM;
  } catch (const std::exception& e) {
    if (ctx) ctx->err = e.what();
    return BBTN_E_INTERNAL;
  }
}

// Kernel-level entry points run on the caller's stream; NULL is the null
// (default) stream, as everywhere in HIP.
hipStream_t pick_stream(bbtn_ctx*, void* s) { return (hipStream_t)s; }

// One instance through the shared pipeline; its own failure becomes this
// call's status.
void solve_network(bbtn_ctx* ctx, Network&& net, std::vector<uint8_t>&& ls_x, bbtn_result* res) {
  std::vector<Instance> one(1);
  one[0].net = std::move(net);
  one[0].ls_x = std::move(ls_x);
  one[0].res = res;
  solve_instances(ctx, one);
  if (one[0].status != BBTN_OK) throw Error(one[0].status, one[0].err);
}

void check_graph(int32_t n, int32_t m, const int32_t* uv) {
  BBTN_REQUIRE(n >= 1 && n <= (1 << 22), "n out of range");
  BBTN_REQUIRE(m >= 0, "m out of range");
  BBTN_REQUIRE(m == 0 || uv != nullptr, "edge list is NULL");
}

}  // namespace

extern "C" {

void bbtn_default_options(bbtn_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->device = 0;
  o->residues_per_pass = 3;
  o->max_primes = 16;
  o->log2_target = 0;
  o->branching = 1;
  o->batched = 1;
  o->region_max = 8;
  o->local_search = 100;
  o->graphs = 1;
  o->scorer_weights = nullptr;
  o->autotune_cache = nullptr;
  o->time_limit_s = 0;
  o->stream = nullptr;
  o->host_threads = 0;
  o->order_refine = 0;
  o->device_mem_cap = 0;
  o->spin_flip = 0;
}

bbtn_status bbtn_create(const bbtn_options* opt, bbtn_ctx** out) {
  if (!out) return BBTN_E_INVALID_ARG;
  *out = nullptr;
  bbtn_ctx* ctx = new (std::nothrow) bbtn_ctx();
  if (!ctx) return BBTN_E_OOM;
  if (opt) ctx->opt = *opt; else bbtn_default_options(&ctx->opt);
  ctx->attach_memcap(std::make_shared<MemCap>());
  ctx->memcap->cap = (size_t)ctx->opt.device_mem_cap;
  bbtn_status s = guard(ctx, [&] {
    BBTN_REQUIRE(ctx->opt.residues_per_pass >= 0 && ctx->opt.residues_per_pass <= KUSER,
                 "residues_per_pass must be in [0, 4]");
    BBTN_REQUIRE(ctx->opt.batched >= 0 && ctx->opt.batched <= 2, "batched must be 0, 1 or 2");
    int ndev = 0;
    BBTN_HIP(hipGetDeviceCount(&ndev));
    BBTN_REQUIRE(ctx->opt.device >= 0 && ctx->opt.device < ndev, "no such device");
    BBTN_HIP(hipSetDevice(ctx->opt.device));
    if (ctx->opt.stream) {
      ctx->stream = (hipStream_t)ctx->opt.stream;
    } else {
      BBTN_HIP(hipStreamCreateWithFlags(&ctx->own, hipStreamNonBlocking));
      ctx->stream = ctx->own;
    }
    (void)prime_table();
    // once per device, with the device current: the address of its copy of
    // the allocation-free product's scratch array
    noalloc_scratch_init(ctx->opt.device);
    if (ctx->opt.autotune_cache) load_tune_cache(ctx, ctx->opt.autotune_cache);
    if (ctx->opt.scorer_weights) load_scorer(ctx, ctx->opt.scorer_weights);
  });
  if (s != BBTN_OK) {
    bbtn_destroy(ctx);
    return s;
  }
  *out = ctx;
  return BBTN_OK;
}

void bbtn_destroy(bbtn_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->opt.device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  ctx->work.release();
  ctx->shared_ws.release();
  ctx->partial.release();
  ctx->base.release();
  ctx->fixbits.release();
  ctx->leafconst.release();
  ctx->leafout.release();
  ctx->misc.release();
  ctx->persist.release();
  ctx->pin_base.release();
  ctx->pin_persist.release();
  ctx->clear_graphs();
  if (ctx->own) (void)hipStreamDestroy(ctx->own);
  bbtn_destroy(ctx->aux);
  delete ctx;
}

const char* bbtn_last_error(const bbtn_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

uint64_t bbtn_last_macs(const bbtn_ctx* ctx) { return ctx ? ctx->last_macs : 0; }

bbtn_status bbtn_profile(bbtn_ctx* ctx, int32_t enable) {
  return bbtn_profile_mask(ctx, enable != 0 ? ~0u : 0u);
}

bbtn_status bbtn_profile_mask(bbtn_ctx* ctx, uint32_t mask) {
  if (!ctx) return BBTN_E_INVALID_ARG;
  return guard(ctx, [&] {
    BBTN_HIP(hipSetDevice(ctx->opt.device));
    ctx->prof.clear();
    ctx->prof.on = (mask & ((1u << K_COUNT) - 1)) != 0;
    ctx->prof.mask = mask;
  });
}

bbtn_status bbtn_get_kernel_stats(bbtn_ctx* ctx, int32_t kernel, bbtn_kernel_stats* out) {
  if (!ctx || !out) return BBTN_E_INVALID_ARG;
  return guard(ctx, [&] {
    BBTN_REQUIRE(kernel >= 0 && kernel < K_COUNT, "unknown kernel id");
    BBTN_HIP(hipSetDevice(ctx->opt.device));
    ctx->prof.resolve();
    const KStat& s = ctx->prof.stat[kernel];
    out->launches = s.launches;
    out->seconds = s.seconds;
    out->ops = s.ops;
    out->bytes = s.bytes;
  });
}

bbtn_status bbtn_solve_spinglass(bbtn_ctx* ctx, int32_t n, int32_t m, const int32_t* edge_uv,
                                 const int32_t* J, const int32_t* h, bbtn_result* res) {
  if (!ctx || !res) return BBTN_E_INVALID_ARG;
  return guard(ctx, [&] {
    check_graph(n, m, edge_uv);
    BBTN_REQUIRE(m == 0 || J != nullptr, "J is NULL");
    BBTN_HIP(hipSetDevice(ctx->opt.device));
    Network net = build_spinglass(n, m, edge_uv, J, h);
    std::vector<uint8_t> x;
    if (ctx->opt.local_search > 0)
      x = local_search_spinglass(n, m, edge_uv, J, h, ctx->opt.local_search, 12345);
    solve_network(ctx, std::move(net), std::move(x), res);
  });
}

bbtn_status bbtn_solve_batch(bbtn_ctx* ctx, int32_t kind, int32_t n_inst, const int32_t* n,
                             const int32_t* m, const int32_t* const* edge_uv,
                             const int32_t* const* weights, const int32_t* const* h,
                             bbtn_result* results, bbtn_status* status) {
  if (!ctx || !results || !status || n_inst < 0) return BBTN_E_INVALID_ARG;
  if (n_inst > 0 && (!n || !m || !edge_uv || !weights)) return BBTN_E_INVALID_ARG;
  return guard(ctx, [&] {
    BBTN_REQUIRE(kind == 0 || kind == 1, "kind must be 0 (spin glass) or 1 (MWIS)");
    BBTN_HIP(hipSetDevice(ctx->opt.device));
    std::vector<Instance> insts(n_inst);
    const int ls = ctx->opt.local_search;
    for (int32_t i = 0; i < n_inst; ++i) {
      insts[i].res = &results[i];
      const int32_t ni = n[i], mi = m[i];
      const int32_t* uv = edge_uv[i];
      const int32_t* w = weights[i];
      const int32_t* hi = h ? h[i] : nullptr;
      insts[i].build = [kind, ni, mi, uv, w, hi, ls](Instance& in) {
        check_graph(ni, mi, uv);
        if (kind == 0) {
          BBTN_REQUIRE(mi == 0 || w != nullptr, "J is NULL");
          in.net = build_spinglass(ni, mi, uv, w, hi);
          if (ls > 0) in.ls_x = local_search_spinglass(ni, mi, uv, w, hi, ls, 12345);
        } else {
          in.net = build_mwis(ni, mi, uv, w);
          if (ls > 0) in.ls_x = local_search_mwis(ni, mi, uv, w, std::max(1, ls / 20), 12345);
        }
      };
    }
    solve_instances(ctx, insts);
    bbtn_status first = BBTN_OK;
    std::string msg;
    for (int32_t i = 0; i < n_inst; ++i) {
      status[i] = insts[i].status;
      if (first == BBTN_OK && insts[i].status != BBTN_OK) {
        first = insts[i].status;
        msg = "instance " + std::to_string(i) + ": " + insts[i].err;
      }
    }
    if (first != BBTN_OK) throw Error(first, msg);
  });
}

bbtn_status bbtn_solve_mwis(bbtn_ctx* ctx, int32_t n, int32_t m, const int32_t* edge_uv,
                            const int32_t* w, bbtn_result* res) {
  if (!ctx || !res) return BBTN_E_INVALID_ARG;
  return guard(ctx, [&] {
    check_graph(n, m, edge_uv);
    BBTN_HIP(hipSetDevice(ctx->opt.device));
    Network net = build_mwis(n, m, edge_uv, w);
    std::vector<uint8_t> x;
    if (ctx->opt.local_search > 0)
      x = local_search_mwis(n, m, edge_uv, w, std::max(1, ctx->opt.local_search / 20), 12345);
    solve_network(ctx, std::move(net), std::move(x), res);
  });
}

bbtn_status bbtn_tgemm(bbtn_ctx* ctx, int32_t k, const uint32_t* primes, int64_t batch, int64_t M,
                       int64_t N, int64_t K, const void* A, const void* B, void* C, void* stream) {
  if (!ctx) return BBTN_E_INVALID_ARG;
  return guard(ctx, [&] {
    BBTN_REQUIRE(k >= 1 && k <= KUSER, "k must be in [1, 4]");
    BBTN_REQUIRE(primes != nullptr, "primes is NULL");
    BBTN_REQUIRE(batch >= 1 && M >= 1 && N >= 1 && K >= 1, "empty product");
    BBTN_REQUIRE(A && B && C, "NULL operand");
    BBTN_REQUIRE(batch * M * K < (1ll << 40) && batch * K * N < (1ll << 40) &&
                     batch * M * N < (1ll << 40), "operand too large");
    BBTN_HIP(hipSetDevice(ctx->opt.device));
    const Moduli mod = make_moduli(k, primes);
    const TuneVal tv = choose_tiles(ctx, k, batch, M, N, K);
    DevTensor part{};
    if (tv.splits > 1) {
      const int64_t ent = (int64_t)tv.splits * batch * M * N;
      ctx->partial.ensure((size_t)(1 + k) * ent * 4);
      part = DevTensor{ctx->partial.as<uint32_t>(), ent};
    }
    GemmShape sh{batch, M, N, K, M * K, K * N, M * N};
    hipStream_t st = pick_stream(ctx, stream);
    const int kid = tv.splits <= 1 && tgemm_is_thin(sh, 1) ? K_THIN : K_TGEMM;
    const int ph = ctx->prof.begin(st, kid);
    launch_tgemm(k, mod, sh, DevTensor{(uint32_t*)A, batch * M * K},
                 DevTensor{(uint32_t*)B, batch * K * N}, DevTensor{(uint32_t*)C, batch * M * N},
                 tv.cfg, tv.splits, part, st);
    ctx->prof.end(ph, st, kid, (double)batch * M * N * K * (2 + 2 * k),
                  (double)(1 + k) * 4 * (double)batch * (double)(M * K + K * N + M * N));
  });
}

bbtn_status bbtn_tgemm_values(bbtn_ctx* ctx, int64_t batch, int64_t M, int64_t N, int64_t K,
                              const int32_t* A, const int32_t* B, int32_t* C, int32_t max_abs,
                              void* stream) {
  if (!ctx) return BBTN_E_INVALID_ARG;
  return guard(ctx, [&] {
    BBTN_REQUIRE(batch >= 1 && M >= 1 && N >= 1 && K >= 1, "empty product");
    BBTN_REQUIRE(A && B && C, "NULL operand");
    BBTN_REQUIRE(max_abs >= 0 && max_abs < (1 << 28), "max_abs out of range");
    BBTN_REQUIRE(batch * M * K < (1ll << 40) && batch * K * N < (1ll << 40) &&
                     batch * M * N < (1ll << 40), "operand too large");
    BBTN_HIP(hipSetDevice(ctx->opt.device));
    const TuneVal tv = cached_or_heuristic_tiles(ctx, 1, batch, M, N, K);
    DevTensor part{};
    if (tv.splits > 1) {
      const int64_t ent = (int64_t)tv.splits * batch * M * N;
      ctx->partial.ensure((size_t)ent * 4);
      part = DevTensor{ctx->partial.as<uint32_t>(), ent};
    }
    GemmShape sh{batch, M, N, K, M * K, K * N, M * N};
    const DevTensor dA{(uint32_t*)A, batch * M * K}, dB{(uint32_t*)B, batch * K * N},
        dC{(uint32_t*)C, batch * M * N};
    hipStream_t st = pick_stream(ctx, stream);
    const bool packed = max_abs < kValues16Bound;
    const int kid = !packed && tgemm_is_thin(sh, tv.splits) ? K_THIN : K_TGEMM;
    const int ph = ctx->prof.begin(st, kid);
    if (packed)
      launch_tgemm_values16(sh, dA, dB, dC, tv.splits, part, st);
    else
      launch_tgemm(0, make_moduli(0, nullptr), sh, dA, dB, dC, tv.cfg, tv.splits, part, st);
    ctx->prof.end(ph, st, kid, 2.0 * batch * M * N * K,
                  4.0 * (double)batch * (double)(M * K + K * N + M * N));
  });
}

bbtn_status bbtn_tgemm_noalloc(bbtn_ctx* ctx, int32_t k, const uint32_t* primes, int64_t batch,
                               int64_t M, int64_t N, int64_t K, const void* A, const void* B,
                               void* C, void* stream) {
  if (!ctx) return BBTN_E_INVALID_ARG;
  return guard(ctx, [&] {
    BBTN_REQUIRE(k >= 1 && k <= KUSER, "k must be in [1, 4]");
    BBTN_REQUIRE(primes != nullptr, "primes is NULL");
    BBTN_REQUIRE(batch >= 1 && M >= 1 && N >= 1 && K >= 1, "empty product");
    BBTN_REQUIRE(A && B && C, "NULL operand");
    BBTN_REQUIRE(batch * M * K < (1ll << 40) && batch * K * N < (1ll << 40) &&
                     batch * M * N < (1ll << 40), "operand too large");
    BBTN_HIP(hipSetDevice(ctx->opt.device));
    uint32_t* scr = noalloc_scratch(ctx->opt.device);
    BBTN_REQUIRE(scr != nullptr, "scratch array not set up on this device");
    const Moduli mod = make_moduli(k, primes);
    // no tuning here (it allocates): the cached choice or the heuristic, with
    // the split-K factor lowered until the partial results fit the scratch
    TuneVal tv = cached_or_heuristic_tiles(ctx, k, batch, M, N, K);
    const int64_t outer = batch * M * N;
    int splits = tv.splits;
    while (splits > 1 &&
           (int64_t)(1 + k) * tgemm_partial_entries(tv.cfg, splits, K, outer) > kNoAllocScratchWords)
      splits = splits / 2;
    const int64_t pe = tgemm_partial_entries(tv.cfg, splits, K, outer);
    DevTensor part{};
    if (pe > 0) part = DevTensor{scr, pe};
    GemmShape sh{batch, M, N, K, M * K, K * N, M * N};
    launch_tgemm(k, mod, sh, DevTensor{(uint32_t*)A, batch * M * K},
                 DevTensor{(uint32_t*)B, batch * K * N}, DevTensor{(uint32_t*)C, outer}, tv.cfg,
                 splits, part, pick_stream(ctx, stream));
  });
}

bbtn_status bbtn_gather(bbtn_ctx* ctx, int32_t k, int32_t r_in, int32_t r_out,
                        const int32_t* src_bits, int64_t L, int64_t in_stride,
                        const uint64_t* fixed_bits, const void* in, int64_t in_entries, void* out,
                        void* stream) {
  if (!ctx) return BBTN_E_INVALID_ARG;
  return guard(ctx, [&] {
    BBTN_REQUIRE(k >= 0 && k <= KUSER, "k must be in [0, 4]");
    BBTN_REQUIRE(L >= 1 && in && out, "bad gather arguments");
    BBTN_REQUIRE(r_out == 0 || src_bits != nullptr, "src_bits is NULL");
    BBTN_REQUIRE(r_in <= 36, "r_in too large");
    const int64_t sz = 1ll << r_in;
    BBTN_REQUIRE(in_stride == 0 || in_stride == sz, "in_stride must be 0 or 2^r_in");
    BBTN_REQUIRE(in_entries >= (in_stride == 0 ? sz : L * sz), "input buffer too small");
    BBTN_HIP(hipSetDevice(ctx->opt.device));
    const GatherPlan gp = make_gather_plan(r_in, r_out, src_bits);
    hipStream_t st = pick_stream(ctx, stream);
    const int ph = ctx->prof.begin(st, K_GATHER);
    launch_gather(k, gp, L, in_stride, fixed_bits, DevTensor{(uint32_t*)in, in_entries},
                  DevTensor{(uint32_t*)out, L << r_out}, st);
    ctx->prof.end(ph, st, K_GATHER, 0, 2.0 * (1 + k) * 4 * (double)(L << r_out));
  });
}

bbtn_status bbtn_reduce(bbtn_ctx* ctx, int32_t k, const uint32_t* primes, int64_t outer,
                        int64_t S, int64_t seg_stride, int64_t elem_stride, const void* in,
                        int64_t in_entries, void* out, void* stream) {
  if (!ctx) return BBTN_E_INVALID_ARG;
  return guard(ctx, [&] {
    BBTN_REQUIRE(k >= 1 && k <= KUSER, "k must be in [1, 4]");
    BBTN_REQUIRE(primes && in && out, "NULL argument");
    BBTN_REQUIRE(outer >= 1 && S >= 1 && seg_stride >= 0 && elem_stride >= 0, "bad sizes");
    BBTN_REQUIRE((S - 1) * seg_stride + (outer - 1) * elem_stride < in_entries,
                 "input buffer too small");
    BBTN_HIP(hipSetDevice(ctx->opt.device));
    const Moduli mod = make_moduli(k, primes);
    launch_reduce(k, mod, outer, S, seg_stride, elem_stride, DevTensor{(uint32_t*)in, in_entries},
                  DevTensor{(uint32_t*)out, outer}, pick_stream(ctx, stream));
  });
}

bbtn_status bbtn_bound(bbtn_ctx* ctx, int64_t n_branch, int32_t tensors_per_branch,
                       const int32_t* values, const int64_t* tensor_off, const int32_t* tensor_len,
                       const int64_t* offset, int64_t incumbent, int64_t* bound,
                       int32_t* keep_idx, int32_t* n_keep, void* stream) {
  if (!ctx) return BBTN_E_INVALID_ARG;
  return guard(ctx, [&] {
    BBTN_REQUIRE(n_branch >= 0 && tensors_per_branch >= 0, "bad sizes");
    BBTN_REQUIRE(n_keep && (n_branch == 0 || (values && tensor_off && tensor_len && offset &&
                                              bound && keep_idx)), "NULL argument");
    BBTN_HIP(hipSetDevice(ctx->opt.device));
    ctx->misc.ensure((size_t)std::max<int64_t>(n_branch, 1) * 4);
    launch_bound(n_branch, tensors_per_branch, values, tensor_off, tensor_len, offset, incumbent,
                 bound, ctx->misc.as<int32_t>(), keep_idx, n_keep, pick_stream(ctx, stream));
  });
}

}  // extern "C"

// ------------------------------------------------------------------ scorer
#include <random>

#include "mlp.h"

extern "C" {

bbtn_status bbtn_mlp_forward(bbtn_ctx* ctx, int64_t rows, const uint16_t* X, const uint16_t* W,
                             const float* bias, float* y, float* h1, float* h2, void* stream) {
  if (!ctx) return BBTN_E_INVALID_ARG;
  return guard(ctx, [&] {
    BBTN_REQUIRE(rows >= 0 && (rows == 0 || (X && W && bias && y)), "bad arguments");
    BBTN_REQUIRE((h1 == nullptr) == (h2 == nullptr), "h1 and h2 go together");
    BBTN_HIP(hipSetDevice(ctx->opt.device));
    launch_mlp_forward(rows, X, W, bias, y, h1, h2, pick_stream(ctx, stream));
  });
}

bbtn_status bbtn_mlp_backward(bbtn_ctx* ctx, int64_t rows, const uint16_t* X, const uint16_t* W,
                              const float* y, const float* t, const float* h1, const float* h2,
                              float* grad, void* stream) {
  if (!ctx) return BBTN_E_INVALID_ARG;
  return guard(ctx, [&] {
    BBTN_REQUIRE(rows >= 1 && X && W && y && t && h1 && h2 && grad, "bad arguments");
    BBTN_HIP(hipSetDevice(ctx->opt.device));
    ctx->partial.ensure((size_t)mlp_partial_floats(rows) * 4);
    launch_mlp_backward(rows, X, W, y, t, h1, h2, ctx->partial.as<float>(), grad,
                        pick_stream(ctx, stream));
  });
}

bbtn_status bbtn_mlp_adam(bbtn_ctx* ctx, float* master, uint16_t* wbf, float* bias, float* m,
                          float* v, const float* grad, float lr, float beta1, float beta2,
                          float eps, int32_t step, void* stream) {
  if (!ctx) return BBTN_E_INVALID_ARG;
  return guard(ctx, [&] {
    BBTN_REQUIRE(master && wbf && bias && m && v && grad && step >= 1, "bad arguments");
    BBTN_HIP(hipSetDevice(ctx->opt.device));
    launch_mlp_adam(master, wbf, bias, m, v, grad, lr, beta1, beta2, eps, step,
                    pick_stream(ctx, stream));
  });
}

bbtn_status bbtn_scorer_load(bbtn_ctx* ctx, const char* path) {
  if (!ctx || !path) return BBTN_E_INVALID_ARG;
  return guard(ctx, [&] {
    BBTN_HIP(hipSetDevice(ctx->opt.device));
    load_scorer(ctx, path);
  });
}

bbtn_status bbtn_plan_leaves(bbtn_ctx* ctx, int32_t kind, int32_t n, int32_t m,
                             const int32_t* edge_uv, const int32_t* weights, const int32_t* h,
                             int32_t log2_target, int32_t region_max, int32_t local_search,
                             int32_t values_only, int32_t order_refine, int8_t* leaves,
                             int64_t capacity, int64_t* n_leaves, int64_t* incumbent) {
  if (!n_leaves || !incumbent) return BBTN_E_INVALID_ARG;
  return guard(ctx, [&] {  // host-only: ctx may be NULL
    check_graph(n, m, edge_uv);
    BBTN_REQUIRE(kind == 0 || kind == 1, "kind must be 0 (spin glass) or 1 (MWIS)");
    BBTN_REQUIRE(log2_target > 0 && region_max >= 1 && local_search >= 0, "bad options");
    BBTN_REQUIRE(order_refine >= -1 && order_refine <= 64, "order_refine must be in [-1, 64]");
    if (kind == 0) BBTN_REQUIRE(weights != nullptr, "J is NULL");
    Network net = kind == 0 ? build_spinglass(n, m, edge_uv, weights, h)
                            : build_mwis(n, m, edge_uv, weights);
    SearchOptions probe;
    probe.log2_target = log2_target;
    probe.region_max = std::min(16, region_max);
    probe.values_only = values_only != 0;
    Tree tree = choose_order(net, order_refine, probe);
    std::vector<uint8_t> x;
    if (local_search > 0)
      x = kind == 0 ? local_search_spinglass(n, m, edge_uv, weights, h, local_search, 12345)
                    : local_search_mwis(n, m, edge_uv, weights, std::max(1, local_search / 20), 12345);
    SearchOptions so;
    so.log2_target = log2_target;
    so.region_max = std::min(16, region_max);
    so.incumbent = x.empty() ? INT64_MIN : network_value(net, x);
    so.values_only = values_only != 0;
    std::vector<LeafGroup> groups;
    SearchStats stats;
    bb_search(net, tree, so, groups, stats);
    int64_t total = 0;
    for (const auto& g : groups) total += g.count;
    *n_leaves = total;
    *incumbent = so.incumbent == INT64_MIN ? INT64_MIN
                 : (net.spin ? -so.incumbent : so.incumbent);
    if (!leaves) return;
    if (capacity < total) throw Error(BBTN_E_BUFFER_TOO_SMALL, "leaf buffer too small");
    int64_t row = 0;
    for (const auto& g : groups)
      for (int64_t l = 0; l < g.count; ++l, ++row) {
        int8_t* out = leaves + row * n;
        std::memset(out, -1, (size_t)n);
        for (size_t j = 0; j < g.vars.size(); ++j)
          out[g.vars[j]] = (int8_t)g.assign[(size_t)l * g.vars.size() + j];
      }
  });
}

bbtn_status bbtn_order_complexity(int32_t kind, int32_t n, int32_t m, const int32_t* edge_uv,
                                  const int32_t* weights, const int32_t* h, int32_t order_refine,
                                  int32_t log2_target, int32_t region_max, double* tc_log2,
                                  int32_t* sc, int64_t* rho) {
  if (!tc_log2 || !sc || !rho) return BBTN_E_INVALID_ARG;
  return guard(nullptr, [&] {
    check_graph(n, m, edge_uv);
    BBTN_REQUIRE(kind == 0 || kind == 1, "kind must be 0 (spin glass) or 1 (MWIS)");
    BBTN_REQUIRE(log2_target > 0 && region_max >= 1, "bad options");
    BBTN_REQUIRE(order_refine >= -1 && order_refine <= 64, "order_refine must be in [-1, 64]");
    if (kind == 0) BBTN_REQUIRE(weights != nullptr, "J is NULL");
    Network net = kind == 0 ? build_spinglass(n, m, edge_uv, weights, h)
                            : build_mwis(n, m, edge_uv, weights);
    SearchOptions probe;
    probe.log2_target = log2_target;
    probe.region_max = std::min(16, region_max);
    const Tree tree = choose_order(net, order_refine, probe);
    const Complexity c = complexity(tree, {});
    *tc_log2 = c.tc_log2;
    *sc = c.sc;
    int64_t r = 0;
    for (int id : tree.postorder)
      r += std::max(0, (int)tree.nodes[id].vars.size() - log2_target);
    *rho = r;
  });
}

static Network order_network(bbtn_ctx* ctx, int32_t kind, int32_t n, int32_t m,
                             const int32_t* edge_uv, const int32_t* weights, const int32_t* h) {
  BBTN_REQUIRE(ctx != nullptr, "NULL context");
  check_graph(n, m, edge_uv);
  BBTN_REQUIRE(kind == 0 || kind == 1, "kind must be 0 (spin glass) or 1 (MWIS)");
  BBTN_REQUIRE(ctx->opt.log2_target > 0, "order candidates need log2_target > 0");
  if (kind == 0) BBTN_REQUIRE(weights != nullptr, "J is NULL");
  return kind == 0 ? build_spinglass(n, m, edge_uv, weights, h) : build_mwis(n, m, edge_uv, weights);
}

bbtn_status bbtn_order_candidates(bbtn_ctx* ctx, int32_t kind, int32_t n, int32_t m,
                                  const int32_t* edge_uv, const int32_t* weights,
                                  const int32_t* h, int32_t* n_out) {
  if (!ctx || !n_out) return BBTN_E_INVALID_ARG;
  return guard(ctx, [&] {
    const Network net = order_network(ctx, kind, n, m, edge_uv, weights, h);
    *n_out = order_candidates(ctx, net);
  });
}

bbtn_status bbtn_order_use(bbtn_ctx* ctx, int32_t kind, int32_t n, int32_t m,
                           const int32_t* edge_uv, const int32_t* weights, const int32_t* h,
                           int32_t which) {
  if (!ctx) return BBTN_E_INVALID_ARG;
  return guard(ctx, [&] {
    const Network net = order_network(ctx, kind, n, m, edge_uv, weights, h);
    order_use(ctx, net, which);
  });
}

bbtn_status bbtn_scorer_collect(bbtn_ctx* ctx, int32_t kind, int32_t n, int32_t m,
                                const int32_t* edge_uv, const int32_t* weights, const int32_t* h,
                                int32_t log2_target, int32_t max_nodes, int32_t cand_per_node,
                                float* X, float* y, int64_t capacity, int64_t* rows) {
  if (!rows) return BBTN_E_INVALID_ARG;
  return guard(ctx, [&] {  // host-only: ctx may be NULL
    check_graph(n, m, edge_uv);
    BBTN_REQUIRE(kind == 0 || kind == 1, "kind must be 0 (spin glass) or 1 (MWIS)");
    BBTN_REQUIRE(log2_target > 0 && max_nodes >= 1 && cand_per_node >= 1, "bad sizes");
    Network net = kind == 0 ? build_spinglass(n, m, edge_uv, weights, h)
                            : build_mwis(n, m, edge_uv, weights);
    Tree tree = greedy_tree(net);
    std::vector<uint8_t> x = kind == 0 ? local_search_spinglass(n, m, edge_uv, weights, h, 200, 12345)
                                       : local_search_mwis(n, m, edge_uv, weights, 10, 12345);
    std::vector<float> fx, fy;
    const int rmax = ctx ? std::max(1, std::min(16, ctx->opt.region_max)) : 8;
    collect_training(net, tree, log2_target, rmax,
                     network_value(net, x), max_nodes, cand_per_node, fx, fy);
    *rows = (int64_t)fy.size();
    if (X && y) {
      BBTN_REQUIRE(capacity >= (int64_t)fy.size(), "capacity too small");
      std::memcpy(X, fx.data(), fx.size() * 4);
      std::memcpy(y, fy.data(), fy.size() * 4);
    }
  });
}

bbtn_status bbtn_scorer_train(bbtn_ctx* ctx, const float* X, const float* y, int64_t rows,
                              int32_t epochs, int32_t batch, float lr, uint64_t seed,
                              float* loss_out, const char* save_path) {
  if (!ctx) return BBTN_E_INVALID_ARG;
  return guard(ctx, [&] {
    BBTN_REQUIRE(X && y && rows >= 1 && epochs >= 1 && batch >= 1 && lr > 0, "bad arguments");
    BBTN_HIP(hipSetDevice(ctx->opt.device));
    hipStream_t st = ctx->stream;
    ScorerModel mdl;
    // standardisation
    for (int q = 0; q < N_FEAT; ++q) {
      double s = 0, s2 = 0;
      for (int64_t r = 0; r < rows; ++r) { s += X[r * N_FEAT + q]; s2 += (double)X[r * N_FEAT + q] * X[r * N_FEAT + q]; }
      const double mu = s / rows, var = std::max(0.0, s2 / rows - mu * mu);
      mdl.fmean[q] = (float)mu;
      mdl.fstd[q] = var > 1e-12 ? (float)std::sqrt(var) : 1.f;
    }
    {
      double s = 0, s2 = 0;
      for (int64_t r = 0; r < rows; ++r) { s += y[r]; s2 += (double)y[r] * y[r]; }
      const double mu = s / rows, var = std::max(0.0, s2 / rows - mu * mu);
      mdl.ymean = (float)mu;
      mdl.ystd = var > 1e-12 ? (float)std::sqrt(var) : 1.f;
    }
    // shuffled, standardised data (bf16 inputs, f32 targets)
    std::mt19937_64 rng(seed);
    std::vector<int64_t> perm(rows);
    for (int64_t r = 0; r < rows; ++r) perm[r] = r;
    std::shuffle(perm.begin(), perm.end(), rng);
    std::vector<uint16_t> xb((size_t)rows * N_FEAT);
    std::vector<float> yt(rows);
    for (int64_t i = 0; i < rows; ++i) {
      const int64_t r = perm[i];
      for (int q = 0; q < N_FEAT; ++q) {
        float v = (X[r * N_FEAT + q] - mdl.fmean[q]) / mdl.fstd[q];
        uint32_t u;
        std::memcpy(&u, &v, 4);
        xb[i * N_FEAT + q] = (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
      }
      yt[i] = (y[r] - mdl.ymean) / mdl.ystd;
    }
    // parameters: uniform +-1/sqrt(fan_in) weights, zero biases
    std::vector<float> master(MLP_NPARAM, 0.f);
    std::uniform_real_distribution<float> U(-1.f, 1.f);
    for (int i = 0; i < MLP_H * MLP_IN; ++i) master[MLP_W1 + i] = U(rng) / std::sqrt((float)MLP_IN);
    for (int i = 0; i < MLP_H * MLP_H; ++i) master[MLP_W2 + i] = U(rng) / std::sqrt((float)MLP_H);
    for (int i = 0; i < MLP_H; ++i) master[MLP_W3 + i] = U(rng) / std::sqrt((float)MLP_H);
    const int64_t B = std::min<int64_t>(batch, rows);
    // device buffers
    DevBuf dbuf;
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    size_t off = 0;
    const size_t o_x = off; off += al(xb.size() * 2);
    const size_t o_y = off; off += al(yt.size() * 4);
    const size_t o_p = off; off += al((size_t)rows * 4);
    const size_t o_h1 = off; off += al((size_t)rows * MLP_H * 4);
    const size_t o_h2 = off; off += al((size_t)rows * MLP_H * 4);
    const size_t o_ms = off; off += al(MLP_NPARAM * 4);
    const size_t o_m = off; off += al(MLP_NPARAM * 4);
    const size_t o_v = off; off += al(MLP_NPARAM * 4);
    const size_t o_g = off; off += al(MLP_NPART * 4);
    const size_t o_w = off; off += al(MLP_NW * 2);
    const size_t o_b = off; off += al(MLP_NB * 4);
    dbuf.ensure(off);
    char* d = dbuf.as<char>();
    std::vector<uint16_t> wb(MLP_NW);
    for (int i = 0; i < MLP_NW; ++i) {
      uint32_t u;
      std::memcpy(&u, &master[i], 4);
      wb[i] = (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
    }
    std::vector<float> zeros(MLP_NPARAM, 0.f);
    BBTN_HIP(hipMemcpyAsync(d + o_x, xb.data(), xb.size() * 2, hipMemcpyHostToDevice, st));
    BBTN_HIP(hipMemcpyAsync(d + o_y, yt.data(), yt.size() * 4, hipMemcpyHostToDevice, st));
    BBTN_HIP(hipMemcpyAsync(d + o_ms, master.data(), MLP_NPARAM * 4, hipMemcpyHostToDevice, st));
    BBTN_HIP(hipMemcpyAsync(d + o_m, zeros.data(), MLP_NPARAM * 4, hipMemcpyHostToDevice, st));
    BBTN_HIP(hipMemcpyAsync(d + o_v, zeros.data(), MLP_NPARAM * 4, hipMemcpyHostToDevice, st));
    BBTN_HIP(hipMemcpyAsync(d + o_w, wb.data(), MLP_NW * 2, hipMemcpyHostToDevice, st));
    BBTN_HIP(hipMemcpyAsync(d + o_b, master.data() + MLP_NW, MLP_NB * 4, hipMemcpyHostToDevice, st));
    ctx->partial.ensure((size_t)mlp_partial_floats(B) * 4);
    const uint16_t* dX = (const uint16_t*)(d + o_x);
    const float* dY = (const float*)(d + o_y);
    float* dP = (float*)(d + o_p);
    float* dH1 = (float*)(d + o_h1);
    float* dH2 = (float*)(d + o_h2);
    int step = 0;
    std::vector<float> pred(rows);
    for (int e = 0; e < epochs; ++e) {
      for (int64_t r0 = 0; r0 < rows; r0 += B) {
        const int64_t nb = std::min<int64_t>(B, rows - r0);
        launch_mlp_forward(nb, dX + r0 * N_FEAT, (const uint16_t*)(d + o_w),
                           (const float*)(d + o_b), dP + r0, dH1 + r0 * MLP_H, dH2 + r0 * MLP_H, st);
        launch_mlp_backward(nb, dX + r0 * N_FEAT, (const uint16_t*)(d + o_w), dP + r0, dY + r0,
                            dH1 + r0 * MLP_H, dH2 + r0 * MLP_H, ctx->partial.as<float>(),
                            (float*)(d + o_g), st);
        launch_mlp_adam((float*)(d + o_ms), (uint16_t*)(d + o_w), (float*)(d + o_b),
                        (float*)(d + o_m), (float*)(d + o_v), (const float*)(d + o_g), lr, 0.9f,
                        0.999f, 1e-8f, ++step, st);
      }
      if (loss_out) {
        launch_mlp_forward(rows, dX, (const uint16_t*)(d + o_w), (const float*)(d + o_b), dP,
                           nullptr, nullptr, st);
        BBTN_HIP(hipMemcpyAsync(pred.data(), dP, rows * 4, hipMemcpyDeviceToHost, st));
        BBTN_HIP(hipStreamSynchronize(st));
        double l = 0;
        for (int64_t r = 0; r < rows; ++r) l += (double)(pred[r] - yt[r]) * (pred[r] - yt[r]);
        loss_out[e] = (float)(l / rows);
      }
    }
    mdl.params.resize(MLP_NPARAM);
    BBTN_HIP(hipMemcpyAsync(mdl.params.data(), d + o_ms, MLP_NPARAM * 4, hipMemcpyDeviceToHost, st));
    BBTN_HIP(hipStreamSynchronize(st));
    dbuf.release();
    if (save_path) {
      if (!write_model(save_path, mdl)) throw Error(BBTN_E_INVALID_ARG, "cannot write scorer weights");
      load_scorer(ctx, save_path);
    }
  });
}

}  // extern "C"
