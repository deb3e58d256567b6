// Tile autotuner for the counting tropical product: for a shape bucket
// (k, log2 batch, log2 M, log2 N, log2 K) it times every candidate tile
// configuration (and split-K factor) on the device with synthetic operands
// and keeps the fastest.  Results persist in a text cache file, one line per
// bucket: "k lb lm ln lk cfg splits".
#include <cstdio>
#include <fstream>
#include <random>
#include <sstream>

#include "exec.h"
#include "scorer.h"

namespace bbtn {

void load_tune_cache(bbtn_ctx* ctx, const char* path) {
  ctx->tune_loaded = true;
  std::ifstream f(path);
  if (!f) return;  // no cache yet
  std::string line;
  while (std::getline(f, line)) {
    if (line.empty() || line[0] == '#') continue;
    std::istringstream is(line);
    int k, lb, lm, ln, lk, cfg, sp;
    if (is >> k >> lb >> lm >> ln >> lk >> cfg >> sp) {
      if (cfg >= 0 && cfg < N_TILE_CFGS && sp >= 1) ctx->tune[TuneKey{k, lb, lm, ln, lk}] = TuneVal{cfg, sp};
    }
  }
}

void save_tune_cache(bbtn_ctx* ctx, const char* path) {
  std::ofstream f(path);
  if (!f) return;
  f << "# k log2batch log2M log2N log2K cfg splits\n";
  for (auto& kv : ctx->tune) {
    const auto& k = kv.first;
    f << std::get<0>(k) << ' ' << std::get<1>(k) << ' ' << std::get<2>(k) << ' '
      << std::get<3>(k) << ' ' << std::get<4>(k) << ' ' << kv.second.cfg << ' '
      << kv.second.splits << '\n';
  }
}

TuneVal autotune_shape(bbtn_ctx* ctx, int k, int64_t batch, int64_t M, int64_t N, int64_t K,
                       const TuneVal& heuristic) {
  hipStream_t st = ctx->stream;
  // a proxy no larger than 2^28 entries per operand and 2^33 MACs
  int64_t b = batch;
  while (b > 1 && (b * M * N * K > (1ll << 33) || b * std::max({M * K, K * N, M * N}) > (1ll << 28))) b >>= 1;
  const int64_t eA = b * M * K, eB = b * K * N, eC = b * M * N;
  if (std::max({eA, eB, eC}) > (1ll << 28)) return heuristic;
  const int W = 1 + k;
  DevBuf buf;
  buf.ensure((size_t)W * (eA + eB + eC) * 4);
  uint32_t* pA = buf.as<uint32_t>();
  uint32_t* pB = pA + W * eA;
  uint32_t* pC = pB + W * eB;
  {
    // operands: small values (dense ties) and residues < 2^30
    std::vector<uint32_t> h((size_t)W * (eA + eB));
    std::mt19937 rng(1234);
    for (int64_t i = 0; i < eA; ++i) h[i] = (uint32_t)(int32_t)(rng() % 17) - 8;
    for (int64_t i = eA; i < W * eA; ++i) h[i] = rng() >> 2;
    for (int64_t i = 0; i < eB; ++i) h[W * eA + i] = (uint32_t)(int32_t)(rng() % 17) - 8;
    for (int64_t i = eB; i < W * eB; ++i) h[W * eA + i] = rng() >> 2;
    BBTN_HIP(hipMemcpyAsync(pA, h.data(), h.size() * 4, hipMemcpyHostToDevice, st));
    BBTN_HIP(hipStreamSynchronize(st));
  }
  const auto& P = prime_table();
  const Moduli mod = make_moduli(k, P.data());
  GemmShape sh{b, M, N, K, M * K, K * N, M * N};
  std::vector<TuneVal> cands;
  for (int c = 0; c < N_TILE_CFGS; ++c) {
    const TileCfg& tc = kTileCfgs[c];
    if ((tc.tm == 1 && M > 1 && N < 64) || (tc.tn == 1 && N > 1 && M < 64)) continue;
    cands.push_back(TuneVal{c, 1});
    const int64_t tiles = ((M + tc.tm - 1) / tc.tm) * ((N + tc.tn - 1) / tc.tn) * b;
    if (K >= 128 && tiles < 2048)
      for (int sp : {4, 16, 64})
        if (K / sp >= 16) cands.push_back(TuneVal{c, sp});
  }
  hipEvent_t e0, e1;
  BBTN_HIP(hipEventCreate(&e0));
  BBTN_HIP(hipEventCreate(&e1));
  TuneVal best = heuristic;
  float best_ms = 1e30f;
  DevBuf part;
  for (const TuneVal& c : cands) {
    DevTensor pt{};
    if (c.splits > 1) {
      const int64_t ent = (int64_t)c.splits * eC;
      part.ensure((size_t)W * ent * 4);
      pt = DevTensor{part.as<uint32_t>(), ent};
    }
    // warm up, then time two launches
    launch_tgemm(k, mod, sh, DevTensor{pA, eA}, DevTensor{pB, eB}, DevTensor{pC, eC}, c.cfg,
                 c.splits, pt, st);
    BBTN_HIP(hipEventRecord(e0, st));
    for (int r = 0; r < 2; ++r)
      launch_tgemm(k, mod, sh, DevTensor{pA, eA}, DevTensor{pB, eB}, DevTensor{pC, eC}, c.cfg,
                   c.splits, pt, st);
    BBTN_HIP(hipEventRecord(e1, st));
    BBTN_HIP(hipEventSynchronize(e1));
    float ms = 0;
    BBTN_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best_ms) { best_ms = ms; best = c; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  buf.release();
  part.release();
  return best;
}

}  // namespace bbtn
