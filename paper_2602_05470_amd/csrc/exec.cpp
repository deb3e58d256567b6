#include "exec.h"
#include "persist.h"

#include <cstring>

namespace bbtn {

void upload_base(bbtn_ctx* ctx, const Network& net, const int* prime_idx, int k, BaseDev& bd,
                 DevBuf& buf) {
  bd.k = k;
  bd.off.resize(net.tensors.size());
  int64_t total = 0;
  for (size_t i = 0; i < net.tensors.size(); ++i) {
    bd.off[i] = total;
    total += net.tensors[i].size();
  }
  bd.total = std::max<int64_t>(total, 1);
  std::vector<uint32_t> host((size_t)(1 + k) * bd.total, 0);
  for (size_t i = 0; i < net.tensors.size(); ++i) {
    const BaseTensor& T = net.tensors[i];
    for (int64_t e = 0; e < T.size(); ++e) {
      host[bd.off[i] + e] = (uint32_t)T.val[e];
      for (int p = 0; p < k; ++p)
        host[(size_t)(p + 1) * bd.total + bd.off[i] + e] = T.res[(size_t)prime_idx[p] * T.size() + e];
    }
  }
  buf.ensure(host.size() * 4);
  BBTN_HIP(hipMemcpyAsync(buf.p, host.data(), host.size() * 4, hipMemcpyHostToDevice, ctx->stream));
  BBTN_HIP(hipStreamSynchronize(ctx->stream));
  bd.t = DevTensor{buf.as<uint32_t>(), bd.total};
}

void upload_bases(bbtn_ctx* ctx, const std::vector<const Network*>& nets, const int* prime_idx,
                  int k, BaseDev& bd, std::vector<std::vector<int64_t>>& offs, DevBuf& buf) {
  bd.k = k;
  bd.off.clear();
  offs.assign(nets.size(), {});
  int64_t total = 0;
  for (size_t i = 0; i < nets.size(); ++i) {
    offs[i].resize(nets[i]->tensors.size());
    for (size_t t = 0; t < nets[i]->tensors.size(); ++t) {
      offs[i][t] = total;
      total += nets[i]->tensors[t].size();
    }
  }
  bd.total = std::max<int64_t>(total, 1);
  // staged in pinned memory: the copy is asynchronous, and the staging
  // buffer is next written after a later synchronisation of the stream
  const size_t words = (size_t)(1 + k) * bd.total;
  BBTN_HIP(hipStreamSynchronize(ctx->stream));
  ctx->pin_base.ensure(words * 4);
  uint32_t* host = ctx->pin_base.as<uint32_t>();
  for (size_t i = 0; i < nets.size(); ++i) {
    const Network& net = *nets[i];
    if (net.tensors.empty()) continue;
    const int64_t o = offs[i][0];
    const bool flat = net.flat_total > 0 && net.flat.size() == (size_t)(1 + NP_FLAT) * net.flat_total;
    // whole planes from the network's flat copy where it holds them
    for (int p = -1; p < k; ++p) {
      const int plane = p < 0 ? 0 : p + 1;
      if (flat && (p < 0 || prime_idx[p] < NP_FLAT)) {
        const int src_plane = p < 0 ? 0 : prime_idx[p] + 1;
        std::memcpy(host + (size_t)plane * bd.total + o,
                    net.flat.data() + (size_t)src_plane * net.flat_total,
                    (size_t)net.flat_total * 4);
        continue;
      }
      for (size_t t = 0; t < net.tensors.size(); ++t) {
        const BaseTensor& T = net.tensors[t];
        const int64_t n = T.size();
        uint32_t* dst = host + (size_t)plane * bd.total + offs[i][t];
        if (p < 0) std::memcpy(dst, T.val.data(), (size_t)n * 4);
        else std::memcpy(dst, &T.res[(size_t)prime_idx[p] * n], (size_t)n * 4);
      }
    }
  }
  if (total == 0)
    for (size_t p = 0; p < words; ++p) host[p] = 0;
  buf.ensure(words * 4);
  BBTN_HIP(hipMemcpyAsync(buf.p, host, words * 4, hipMemcpyHostToDevice, ctx->stream));
  bd.t = DevTensor{buf.as<uint32_t>(), bd.total};
}

static int ilog2_bucket(int64_t x) {
  int b = 0;
  while ((1ll << (b + 1)) <= x) ++b;
  return b;
}

static TuneKey tune_key(int k, int64_t batch, int64_t M, int64_t N, int64_t K) {
  return TuneKey{k, std::min(ilog2_bucket(batch), 20), ilog2_bucket(M), ilog2_bucket(N),
                 ilog2_bucket(K)};
}

TuneVal cached_or_heuristic_tiles(const bbtn_ctx* ctx, int k, int64_t batch, int64_t M,
                                  int64_t N, int64_t K) {
  auto it = ctx->tune.find(tune_key(k, batch, M, N, K));
  if (it != ctx->tune.end()) return it->second;
  TuneVal tv{2, 1};
  if (M == 1 && N >= 64) tv.cfg = 5;
  else if (N == 1 && M >= 64) tv.cfg = 6;
  // measured best for counting products (four-word staging when aligned)
  else if (k >= 5 && M >= 32 && N >= 64) tv.cfg = 12;
  else if (k >= 4 && M >= 32 && N >= 64) tv.cfg = 11;
  else if (k >= 1 && M >= 64 && N >= 32) tv.cfg = 10;
  else if (k >= 1 && M >= 32 && N >= 64) tv.cfg = 8;
  else if (M >= 64 && N >= 64) tv.cfg = 0;
  else if (M >= 32 && N >= 32) tv.cfg = 1;
  else if (M <= 8 && N >= 64) tv.cfg = 3;
  else if (N <= 8 && M >= 64) tv.cfg = 4;
  const TileCfg& c = kTileCfgs[tv.cfg];
  const int64_t tiles = ((M + c.tm - 1) / c.tm) * ((N + c.tn - 1) / c.tn) * batch;
  if (tiles < 1024 && K >= 256) {
    int64_t sp = std::min<int64_t>(K / 64, (2048 + tiles - 1) / tiles);
    tv.splits = (int)std::max<int64_t>(1, std::min<int64_t>(sp, 256));
  }
  return tv;
}

TuneVal choose_tiles(bbtn_ctx* ctx, int k, int64_t batch, int64_t M, int64_t N, int64_t K) {
  const TuneKey key = tune_key(k, batch, M, N, K);
  if (ctx->tune.count(key)) return ctx->tune[key];
  TuneVal tv = cached_or_heuristic_tiles(ctx, k, batch, M, N, K);
  // measured choice for products large enough to matter
  if (ctx->opt.autotune_cache && (double)batch * M * N * K >= (double)(1 << 24)) {
    tv = autotune_shape(ctx, k, batch, M, N, K, tv);
    ctx->tune[key] = tv;
    save_tune_cache(ctx, ctx->opt.autotune_cache);
  }
  return tv;
}

void leaf_constants(const Network& net, const GroupPlan& g, const int* prime_idx, int k,
                    const uint8_t* assign, int64_t L, std::vector<uint32_t>& host) {
  const auto& P = prime_table();
  const size_t S = g.fixed_vars.size();
  host.assign((size_t)(1 + k) * L, 0);
  std::vector<int> pos_of(net.n, -1);
  for (size_t j = 0; j < S; ++j) pos_of[g.fixed_vars[j]] = (int)j;
  for (int64_t l = 0; l < L; ++l) {
    int64_t v = 0;
    uint32_t r[KMAX];
    for (int p = 0; p < k; ++p) r[p] = 1;
    bool feas = true;
    for (int t : g.folded) {
      const BaseTensor& T = net.tensors[t];
      int64_t e = 0;
      for (size_t j = 0; j < T.vars.size(); ++j) e |= (int64_t)(assign[l * S + pos_of[T.vars[j]]] & 1) << j;
      if (T.val[e] <= NEG_CUT) { feas = false; break; }
      v += T.val[e];
      for (int p = 0; p < k; ++p)
        r[p] = mulmod(r[p], T.res[(size_t)prime_idx[p] * T.size() + e], P[prime_idx[p]]);
    }
    host[l] = (uint32_t)(feas ? (int32_t)v : NEG);
    for (int p = 0; p < k; ++p) host[(size_t)(p + 1) * L + l] = feas ? r[p] : 0u;
  }
}

void run_group(bbtn_ctx* ctx, const Network& net, const GroupPlan& g, const BaseDev& bd,
               const Moduli& mod, const uint8_t* assign, int64_t L, DevTensor out,
               hipStream_t st, bool reuse, bool shared_ready, int64_t L_group) {
  if (L_group < 0) L_group = L;
  const int k = bd.k;
  const int W = 1 + k;  // words per entry
  const size_t S = g.fixed_vars.size();
  // workspaces: branch buffers scale with L; shared subtrees (scratch and
  // roots) are computed once
  ctx->work.ensure((size_t)W * L * std::max<int64_t>(g.peak, 1) * 4);
  ctx->shared_ws.ensure((size_t)W * std::max<int64_t>(g.subtree_peak + g.shared_total, 1) * 4);
  uint32_t* ws = ctx->work.as<uint32_t>();
  uint32_t* sw = ctx->shared_ws.as<uint32_t>();
  // small steps that run once per pass: one persistent launch (a forest of
  // subtrees, one workgroup each) instead of a launch per step and operand;
  // their subtree roots live in the forest's root region
  SmallForest fr;
  if (ctx->opt.batched == 1) fr = plan_small_forest(g, bd.off, k, L_group);
  std::vector<uint8_t> fimg;
  uint8_t* fdev = nullptr;
  if (!fr.tasks.empty()) {
    fimg = small_forest_image(fr);
    ctx->forest.ensure(small_forest_bytes(fr, k));
    fdev = ctx->forest.as<uint8_t>();
    BBTN_HIP(hipMemcpyAsync(fdev + small_forest_prog_off(fr, k), fimg.data(), fimg.size(),
                            hipMemcpyHostToDevice, st));
  }
  auto buf = [&](int id) {
    if (!fr.root_off.empty() && fr.root_off[id] >= 0)
      return DevTensor{(uint32_t*)fdev + (size_t)W * fr.root_off[id], g.buf_entries[id]};
    switch (g.buf_region[id]) {
      case R_SUBTREE: return DevTensor{sw + (size_t)W * g.buf_off[id], g.buf_entries[id]};
      case R_SHARED:
        return DevTensor{sw + (size_t)W * (g.subtree_peak + g.buf_off[id]), g.buf_entries[id]};
      default: return DevTensor{ws + (size_t)W * L * g.buf_off[id], L * g.buf_entries[id]};
    }
  };
  // fixed bits of every base operand for every branch
  std::vector<int> pos_of(net.n, -1);
  for (size_t j = 0; j < S; ++j) pos_of[g.fixed_vars[j]] = (int)j;
  const size_t nbo = g.base_ops.size();
  std::vector<uint64_t> fb(std::max<size_t>(nbo, 1) * L, 0);
  for (size_t i = 0; i < nbo; ++i) {
    const Step& s = g.steps[g.base_ops[i].first];
    const Operand& op = g.base_ops[i].second == 0 ? s.a : s.b;
    for (int64_t l = 0; l < L; ++l) {
      uint64_t bits = 0;
      for (auto& fp : op.fixed_pos) bits |= (uint64_t)(assign[l * S + pos_of[fp.second]] & 1) << fp.first;
      fb[i * L + l] = bits;
    }
  }
  ctx->fixbits.ensure(fb.size() * 8);
  BBTN_HIP(hipMemcpyAsync(ctx->fixbits.p, fb.data(), fb.size() * 8, hipMemcpyHostToDevice, st));
  // folded constants per branch
  std::vector<uint32_t> lc;
  std::vector<int> pidx(k);
  for (int p = 0; p < k; ++p) {
    // recover prime-table indices from the moduli
    const auto& P = prime_table();
    pidx[p] = (int)(std::find(P.begin(), P.end(), mod.p[p]) - P.begin());
  }
  leaf_constants(net, g, pidx.data(), k, assign, L, lc);
  ctx->leafconst.ensure(lc.size() * 4);
  BBTN_HIP(hipMemcpyAsync(ctx->leafconst.p, lc.data(), lc.size() * 4, hipMemcpyHostToDevice, st));
  BBTN_HIP(hipStreamSynchronize(st));  // host staging vectors die with this scope
  const DevTensor lconst{ctx->leafconst.as<uint32_t>(), L};

  // tile choices (possibly autotuned, which allocates) and split-K space are
  // settled before any capture
  std::vector<TuneVal> tvs(g.steps.size());
  int64_t part_entries = 0;
  for (size_t si = 0; si < g.steps.size(); ++si) {
    const Step& s = g.steps[si];
    const int64_t Ls = s.shared ? 1 : L;
    const int64_t M = 1ll << s.rm, N = 1ll << s.rn, K = 1ll << s.rk;
    tvs[si] = choose_tiles(ctx, k, Ls << s.rb, M, N, K);
    if (tvs[si].splits > 1) part_entries = std::max<int64_t>(part_entries, (int64_t)tvs[si].splits * (Ls << s.rb) * M * N);
  }
  if (part_entries > 0) ctx->partial.ensure((size_t)W * part_entries * 4);
  // values pass: every partial sum of the network is bounded by the sum of
  // its |couplings| and |fields| (or weights), so small networks take the
  // packed 16-bit product for steps with M and N of at least 32
  const bool vals16 = k == 0 && net.abs_sum < kValues16Bound;
  // shared steps first (once), then the branch steps
  std::vector<size_t> order;
  for (size_t si = 0; si < g.steps.size(); ++si)
    if (g.steps[si].shared) order.push_back(si);
  for (size_t si = 0; si < g.steps.size(); ++si)
    if (!g.steps[si].shared) order.push_back(si);
  auto issue = [&]() {
    if (!fr.tasks.empty() && !shared_ready) {
      const int ph = ctx->prof.begin(st, K_PERSIST);
      launch_small_forest(fr, k, mod, bd, fdev, st, ws);
      ctx->prof.end(ph, st, K_PERSIST, fr.ops, fr.bytes);
    }
    for (size_t si : order) {
      if (!fr.in.empty() && fr.in[si]) continue;
      const Step& s = g.steps[si];
      if (s.shared && shared_ready) continue;
      const int64_t Ls = s.shared ? 1 : L;
      DevTensor opnd[2];
      const Operand* ops[2] = {&s.a, &s.b};
      const int ranks[2] = {(int)s.a_vars.size(), (int)s.b_vars.size()};
      const TuneVal tv = tvs[si];
      const bool packed = vals16 && s.rm >= 5 && s.rn >= 5;
      // packed products read a permuted intermediate operand in place (no
      // gathered copy) when a tile's rows and k slice cover the 64 lowest
      // source entries; lanes walk whichever of the two covers more
      bool fuse[2] = {false, false};
      FusedOp fop[2]{};
      // (not in programs that keep every operand for the traceback)
      if (packed && tv.splits <= 1 && !g.keep_all) {
        const bool small = s.rm < 7 || s.rn < 7;  // 64-wide tiles, else 128
        const int tb = small ? 6 : 7;
        for (int w = 0; w < 2; ++w) {
          const Operand& op = *ops[w];
          if (op.base || op.direct || !op.fixed_pos.empty() ||
              (int)op.src_bits.size() != op.r_in || op.r_in > 30)
            continue;
          // layout bits of the row index (m of A, n of B) and of k
          const int row_lo = w == 0 ? s.rk : 0, row_n = std::min(tb, w == 0 ? s.rm : s.rn);
          const int k_lo = w == 0 ? 0 : s.rn, k_n = std::min(5, s.rk);
          // lowest source bits 0, 1, ... that are images of the given
          // layout bit ranges
          auto cover = [&](int lo1, int n1, int lo2, int n2) {
            int c = 0;
            for (;; ++c) {
              bool hit = false;
              for (int j = lo1; j < lo1 + n1; ++j) hit |= op.src_bits[j] == c;
              for (int j = lo2; j < lo2 + n2; ++j) hit |= op.src_bits[j] == c;
              if (!hit) return c;
            }
          };
          // the tile's rows and k slice together cover the lowest 64 source
          // entries: every source line a tile touches is used whole while
          // the tile is staged
          if (cover(row_lo, row_n, k_lo, k_n) < 6) continue;
          const int cr = cover(row_lo, row_n, 0, 0), ck = cover(k_lo, k_n, 0, 0);
          FusedOp& f = fop[w];
          f.src = buf(op.id).ptr;
          f.stride = g.buf_region[op.id] == R_SHARED ? 0 : (1ll << op.r_in);
          f.rb = s.rb;
          f.fast = cr >= ck ? 1 : 0;
          for (int j = 0; j < op.r_in; ++j) f.bits[j] = (int8_t)op.src_bits[j];
          fuse[w] = true;
        }
      }
      for (int w = 0; w < 2; ++w) {
        const Operand& op = *ops[w];
        if (fuse[w]) continue;
        if (op.base) {
          const GatherPlan gp = make_gather_plan(op.r_in, ranks[w], op.src_bits.data());
          const DevTensor src{bd.t.ptr + bd.off[op.id], bd.total};
          const uint64_t* fbits =
              s.shared ? nullptr : ctx->fixbits.as<uint64_t>() + (size_t)op.base_op * L;
          const int ph = ctx->prof.begin(st, K_GATHER);
          launch_gather(k, gp, Ls, 0, fbits, src, buf(op.temp), st);
          ctx->prof.end(ph, st, K_GATHER, 0, 2.0 * W * 4 * (double)(Ls << ranks[w]));
          opnd[w] = buf(op.temp);
        } else if (!op.direct) {
          const GatherPlan gp = make_gather_plan(op.r_in, ranks[w], op.src_bits.data());
          // a shared root is read by every branch: no branch stride; the root
          // of a deferred subtree is sliced by each branch's fixed bits
          const int64_t stride = g.buf_region[op.id] == R_SHARED ? 0 : (1ll << op.r_in);
          const uint64_t* fbits = (op.base_op >= 0 && !s.shared)
                                      ? ctx->fixbits.as<uint64_t>() + (size_t)op.base_op * L
                                      : nullptr;
          const int ph = ctx->prof.begin(st, K_GATHER);
          launch_gather(k, gp, Ls, stride, fbits, buf(op.id), buf(op.temp), st);
          ctx->prof.end(ph, st, K_GATHER, 0, 2.0 * W * 4 * (double)(Ls << ranks[w]));
          opnd[w] = buf(op.temp);
        } else {
          opnd[w] = buf(op.id);
        }
      }
      const int64_t M = 1ll << s.rm, N = 1ll << s.rn, K = 1ll << s.rk;
      const int64_t batch = Ls << s.rb;
      GemmShape sh{batch, M, N, K, M * K, K * N, M * N};
      DevTensor part{};
      if (tv.splits > 1) part = DevTensor{ctx->partial.as<uint32_t>(), (int64_t)tv.splits * batch * M * N};
      const int kid = !packed && tgemm_is_thin(sh, tv.splits) ? K_THIN : K_TGEMM;
      const int ph = ctx->prof.begin(st, kid);
      if (fuse[0] || fuse[1])
        launch_tgemm_values16_fused(sh, fuse[0] ? &fop[0] : nullptr, opnd[0],
                                    fuse[1] ? &fop[1] : nullptr, opnd[1], buf(s.out), st);
      else if (packed)
        launch_tgemm_values16(sh, opnd[0], opnd[1], buf(s.out), tv.splits, part, st);
      else
        launch_tgemm(k, mod, sh, opnd[0], opnd[1], buf(s.out), tv.cfg, tv.splits, part, st);
      ctx->prof.end(ph, st, kid, (double)Ls * s.macs() * (2 + 2 * k),
                    (double)W * 4 * (double)batch * (double)(M * K + K * N + M * N));
    }
    if (g.root_buf >= 0) {
      launch_otimes(k, mod, L, buf(g.root_buf), lconst, out, st);
    } else {
      // the whole sub-network folded into constants: copy them
      const GatherPlan id = make_gather_plan(0, 0, nullptr);
      launch_gather(k, id, L, 1, nullptr, lconst, out, st);
    }
  };
  for (const Step& s : g.steps)
    if (!(s.shared && shared_ready)) ctx->last_macs += (uint64_t)((s.shared ? 1 : L) * s.macs());
  // A program that runs more than once with the same shapes (chunks of a
  // group, or one branch at a time) is captured into a hipGraph on first use
  // and replayed: its device inputs (fixed bits, constants) sit in the same
  // buffers, refreshed before every replay.
  if (reuse && ctx->opt.graphs && !ctx->prof.on && g.steps.size() >= 2) {
    uint64_t off_hash = 1469598103934665603ull;  // FNV-1a over the base offsets
    for (int64_t o : bd.off) off_hash = (off_hash ^ (uint64_t)o) * 1099511628211ull;
    // keyed by the program's unique id, not its address: a program freed
    // from the cache and another allocated at the same address must not
    // replay the first one's graph
    const GraphKey key{(const void*)(uintptr_t)g.uid, L, k, ctx->work.p, ctx->partial.p, ctx->fixbits.p,
                       ctx->leafconst.p, (void*)out.ptr, (void*)bd.t.ptr, mod.p[0],
                       ctx->shared_ws.p, (void*)fdev, off_hash, shared_ready};
    auto it = ctx->graphs.find(key);
    if (it == ctx->graphs.end()) {
      hipGraph_t graph;
      BBTN_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      try {
        issue();
      } catch (...) {
        hipGraph_t dead;
        (void)hipStreamEndCapture(st, &dead);
        if (dead) (void)hipGraphDestroy(dead);
        throw;
      }
      BBTN_HIP(hipStreamEndCapture(st, &graph));
      hipGraphExec_t exec;
      BBTN_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
      (void)hipGraphDestroy(graph);
      it = ctx->graphs.emplace(key, exec).first;
    }
    BBTN_HIP(hipGraphLaunch(it->second, st));
  } else {
    issue();
  }
}

}  // namespace bbtn
