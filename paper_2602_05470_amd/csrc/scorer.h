// Learned branching scorer (host side): per-variable features of a search
// node, the training-data collector, the training driver and the inference
// hook used by the planner.  The scorer only orders branching variables (the
// seeds and growth order of the region); the planner still evaluates F(R),
// D(R) and gamma for whatever region it grows, so results are unchanged.
#pragma once
#include <vector>
#include "ctx.h"
#include "mlp.h"
#include "search.h"

namespace bbtn {

constexpr int N_FEAT = MLP_IN;

// Precomputed per-network data for feature extraction.
struct FeatureCtx {
  const Network* net;
  const Tree* tree;
  int t;
  std::vector<std::vector<int32_t>> nbr, var_tensors;
  std::vector<int32_t> post_index;  // tree node id -> position in postorder
  std::vector<double> spread;       // per var: sum over its tensors of (max - min)
  FeatureCtx(const Network& n, const Tree& tr, int log2_target);
  // features of variable v at a node (fixed mask, node sizes, heuristic
  // scores of every variable, rho of the node)
  void features(int v, const std::vector<uint64_t>& fixed, const std::vector<int16_t>& sizes,
                const std::vector<double>& heur, int64_t rho, float* out) const;
};

// Loaded scorer: standardisation and parameters (float32 master copy).
struct ScorerModel {
  float fmean[N_FEAT], fstd[N_FEAT];
  float ymean = 0, ystd = 1;
  std::vector<float> params;  // MLP_NPARAM
};
bool read_model(const char* path, ScorerModel& m);
bool write_model(const char* path, const ScorerModel& m);

void load_scorer(bbtn_ctx* ctx, const char* path);
VarScorer make_var_scorer(bbtn_ctx* ctx, const Network& net, const Tree& tree, int log2_target);
void load_tune_cache(bbtn_ctx* ctx, const char* path);

// Run the search on a network and record, for sampled nodes and candidate
// seeds, (features, label): the label is log2 of the branching factor gamma
// of the best rule grown from the seed (the characteristic equation, which
// folds the problem-size reduction and the pruning of F(R) together), minus
// the smallest label among the node's candidates.
void collect_training(const Network& net, const Tree& tree, int log2_target, int region_max,
                      int64_t incumbent, int max_nodes, int cand_per_node,
                      std::vector<float>& X, std::vector<float>& y);

}  // namespace bbtn
