#include "scorer.h"

#include <cmath>
#include <cstring>
#include <fstream>
#include <memory>

namespace bbtn {

FeatureCtx::FeatureCtx(const Network& n, const Tree& tr, int log2_target)
    : net(&n), tree(&tr), t(log2_target) {
  var_tensors.assign(n.n, {});
  nbr.assign(n.n, {});
  spread.assign(n.n, 0.0);
  for (int i = 0; i < (int)n.tensors.size(); ++i) {
    const BaseTensor& T = n.tensors[i];
    int32_t mx = INT32_MIN, mn = INT32_MAX;
    for (int32_t v : T.val)
      if (v > NEG_CUT) { mx = std::max(mx, v); mn = std::min(mn, v); }
    for (int v : T.vars) {
      var_tensors[v].push_back(i);
      if (mx >= mn) spread[v] += (double)(mx - mn);
    }
  }
  for (int v = 0; v < n.n; ++v) {
    for (int ti : var_tensors[v])
      for (int u : n.tensors[ti].vars)
        if (u != v) nbr[v].push_back(u);
    std::sort(nbr[v].begin(), nbr[v].end());
    nbr[v].erase(std::unique(nbr[v].begin(), nbr[v].end()), nbr[v].end());
  }
  post_index.assign(tr.nodes.size(), 0);
  for (size_t i = 0; i < tr.postorder.size(); ++i) post_index[tr.postorder[i]] = (int32_t)i;
}

void FeatureCtx::features(int v, const std::vector<uint64_t>& fixed,
                          const std::vector<int16_t>& sizes, const std::vector<double>& heur,
                          int64_t rho, float* f) const {
  for (int i = 0; i < N_FEAT; ++i) f[i] = 0.f;
  const auto& vn = tree->var_nodes[v];
  double over = 0, over2 = 0, mean_size = 0;
  int n_over = 0, max_over = 0, first = INT32_MAX, last = -1;
  for (int id : vn) {
    const int s = sizes[id];
    const int o = std::max(0, s - t);
    over += o;
    over2 += (double)o * o;
    n_over += o > 0;
    max_over = std::max(max_over, o);
    mean_size += s;
    first = std::min(first, post_index[id]);
    last = std::max(last, post_index[id]);
  }
  const double nn = std::max<size_t>(1, tree->postorder.size());
  mean_size /= std::max<size_t>(1, vn.size());
  int free_nb = 0, fixed_nb = 0, pos_nb = 0;
  double nb_mean = 0, nb_max = 0;
  for (int u : nbr[v]) {
    if (bit_get(fixed, u)) { ++fixed_nb; continue; }
    ++free_nb;
    nb_mean += heur[u];
    nb_max = std::max(nb_max, heur[u]);
    pos_nb += heur[u] > 0;
  }
  if (free_nb) nb_mean /= free_nb;
  double hmax = 0;
  int n_free = 0, rank = 0;
  for (int u = 0; u < net->n; ++u) {
    if (bit_get(fixed, u)) continue;
    ++n_free;
    hmax = std::max(hmax, heur[u]);
    if (heur[u] > heur[v]) ++rank;
  }
  // rho reduction when v alone is fixed
  double drho = 0;
  for (int id : vn) drho += (sizes[id] > t) ? 1.0 : 0.0;
  const double rr = std::max<double>(1.0, (double)rho);
  const double hm = std::max(1.0, hmax);
  f[0] = (float)(heur[v] / rr);
  f[1] = (float)std::log2(1.0 + heur[v]);
  f[2] = (float)std::log2(1.0 + n_over);
  f[3] = (float)(max_over / 16.0);
  f[4] = (float)(mean_size / 32.0);
  f[5] = (float)std::log2(1.0 + vn.size());
  f[6] = (float)(first == INT32_MAX ? 0.0 : first / nn);
  f[7] = (float)(last < 0 ? 0.0 : last / nn);
  f[8] = (float)(free_nb / 8.0);
  f[9] = (float)(fixed_nb / 8.0);
  f[10] = (float)(var_tensors[v].size() / 8.0);
  f[11] = (float)(spread[v] / 8.0);
  f[12] = (float)(drho / rr);
  f[13] = (float)std::log2(1.0 + drho);
  f[14] = (float)std::log2(1.0 + (double)rho);
  f[15] = (float)((double)(net->n - n_free) / std::max(1, net->n));
  f[16] = (float)(t / 32.0);
  f[17] = (float)(std::log2((double)std::max(2, net->n)) / 16.0);
  f[18] = (float)(nb_mean / hm);
  f[19] = (float)(nb_max / hm);
  f[20] = (float)((double)rank / std::max(1, n_free));
  f[21] = (float)(heur[v] / hm);
  f[22] = (float)(vn.empty() ? 0.0 : (double)n_over / vn.size());
  f[23] = net->spin ? 1.f : 0.f;
  f[24] = (float)(pos_nb / 8.0);
  f[25] = (float)(over2 / (1.0 + rr));
}

// ---------------------------------------------------------------- model IO
static const char MAGIC[8] = {'B', 'B', 'T', 'N', 'M', 'L', 'P', '1'};

bool read_model(const char* path, ScorerModel& m) {
  std::ifstream f(path, std::ios::binary);
  if (!f) return false;
  char mg[8];
  int32_t nin = 0, nh = 0;
  f.read(mg, 8);
  f.read((char*)&nin, 4);
  f.read((char*)&nh, 4);
  if (!f || std::memcmp(mg, MAGIC, 8) != 0 || nin != MLP_IN || nh != MLP_H) return false;
  f.read((char*)m.fmean, sizeof m.fmean);
  f.read((char*)m.fstd, sizeof m.fstd);
  f.read((char*)&m.ymean, 4);
  f.read((char*)&m.ystd, 4);
  m.params.resize(MLP_NPARAM);
  f.read((char*)m.params.data(), MLP_NPARAM * 4);
  return (bool)f;
}

bool write_model(const char* path, const ScorerModel& m) {
  std::ofstream f(path, std::ios::binary);
  if (!f) return false;
  const int32_t nin = MLP_IN, nh = MLP_H;
  f.write(MAGIC, 8);
  f.write((const char*)&nin, 4);
  f.write((const char*)&nh, 4);
  f.write((const char*)m.fmean, sizeof m.fmean);
  f.write((const char*)m.fstd, sizeof m.fstd);
  f.write((const char*)&m.ymean, 4);
  f.write((const char*)&m.ystd, 4);
  f.write((const char*)m.params.data(), MLP_NPARAM * 4);
  return (bool)f;
}

static uint16_t to_bf16(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

void load_scorer(bbtn_ctx* ctx, const char* path) {
  ScorerModel m;
  if (!read_model(path, m)) throw Error(BBTN_E_INVALID_ARG, std::string("cannot read scorer weights: ") + path);
  ctx->scorer_model.assign(2 * N_FEAT + 2 + MLP_NPARAM, 0.f);
  float* s = ctx->scorer_model.data();
  std::memcpy(s, m.fmean, sizeof m.fmean);
  std::memcpy(s + N_FEAT, m.fstd, sizeof m.fstd);
  s[2 * N_FEAT] = m.ymean;
  s[2 * N_FEAT + 1] = m.ystd;
  std::memcpy(s + 2 * N_FEAT + 2, m.params.data(), MLP_NPARAM * 4);
  // device copy: bf16 weights, f32 biases
  std::vector<uint16_t> w(MLP_NW);
  for (int i = 0; i < MLP_NW; ++i) w[i] = to_bf16(m.params[i]);
  const size_t wbytes = (MLP_NW * 2 + 255) / 256 * 256;
  ctx->scorer_dev.ensure(wbytes + MLP_NB * 4);
  BBTN_HIP(hipMemcpyAsync(ctx->scorer_dev.p, w.data(), MLP_NW * 2, hipMemcpyHostToDevice, ctx->stream));
  BBTN_HIP(hipMemcpyAsync(ctx->scorer_dev.as<char>() + wbytes, m.params.data() + MLP_NW, MLP_NB * 4,
                          hipMemcpyHostToDevice, ctx->stream));
  BBTN_HIP(hipStreamSynchronize(ctx->stream));
  ctx->scorer_loaded = true;
}

// Scores every free variable of a node with the MLP on the device: the score
// is minus the predicted (standardised) log branching factor, so seeds with
// the smallest predicted gamma come first.
VarScorer make_var_scorer(bbtn_ctx* ctx, const Network& net, const Tree& tree, int log2_target) {
  auto fc = std::make_shared<FeatureCtx>(net, tree, log2_target);
  const int64_t t = log2_target;
  return [ctx, fc, t](const std::vector<uint64_t>& fixed, const std::vector<int16_t>& sizes,
                      const std::vector<double>& heur, std::vector<double>& score) {
    const Network& n = *fc->net;
    std::vector<int32_t> vs;
    for (int v = 0; v < n.n; ++v)
      if (!bit_get(fixed, v)) vs.push_back(v);
    if (vs.empty()) return;
    int64_t rho = 0;
    for (int id : fc->tree->postorder) rho += std::max<int64_t>(0, sizes[id] - t);
    const float* mdl = ctx->scorer_model.data();
    std::vector<uint16_t> X(vs.size() * N_FEAT);
    float f[N_FEAT];
    for (size_t i = 0; i < vs.size(); ++i) {
      fc->features(vs[i], fixed, sizes, heur, rho, f);
      for (int q = 0; q < N_FEAT; ++q)
        X[i * N_FEAT + q] = to_bf16((f[q] - mdl[q]) / mdl[N_FEAT + q]);
    }
    const size_t wbytes = (MLP_NW * 2 + 255) / 256 * 256;
    const size_t bbytes = (MLP_NB * 4 + 255) / 256 * 256;
    const size_t xbytes = (X.size() * 2 + 255) / 256 * 256;
    const size_t need = wbytes + bbytes + xbytes + vs.size() * 4;
    if (ctx->scorer_dev.bytes < need) {
      // grow while keeping the weights: reload them after the reallocation
      std::vector<char> keep(wbytes + MLP_NB * 4);
      BBTN_HIP(hipMemcpy(keep.data(), ctx->scorer_dev.p, keep.size(), hipMemcpyDeviceToHost));
      ctx->scorer_dev.ensure(need * 2);
      BBTN_HIP(hipMemcpy(ctx->scorer_dev.p, keep.data(), keep.size(), hipMemcpyHostToDevice));
    }
    char* base = ctx->scorer_dev.as<char>();
    uint16_t* dX = (uint16_t*)(base + wbytes + bbytes);
    float* dy = (float*)(base + wbytes + bbytes + xbytes);
    hipStream_t st = ctx->stream;
    BBTN_HIP(hipMemcpyAsync(dX, X.data(), X.size() * 2, hipMemcpyHostToDevice, st));
    launch_mlp_forward((int64_t)vs.size(), dX, (const uint16_t*)base, (const float*)(base + wbytes),
                       dy, nullptr, nullptr, st);
    std::vector<float> y(vs.size());
    BBTN_HIP(hipMemcpyAsync(y.data(), dy, y.size() * 4, hipMemcpyDeviceToHost, st));
    BBTN_HIP(hipStreamSynchronize(st));
    for (size_t i = 0; i < vs.size(); ++i) score[vs[i]] = -(double)y[i];
  };
}

}  // namespace bbtn
