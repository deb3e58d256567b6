// Pairwise contraction tree of a tensor network and its complexity
// (time complexity = total semiring operations, space complexity = largest
// intermediate; "Tropical Tensor Networks" section).
#pragma once
#include <vector>
#include "network.h"

namespace bbtn {

struct TNode {
  int32_t left = -1, right = -1;  // children (internal nodes)
  int32_t base = -1;              // base tensor id (leaves)
  int32_t parent = -1;
  std::vector<int32_t> vars;      // ascending; variables the node's tensor keeps
};

struct Tree {
  std::vector<TNode> nodes;       // leaves first (node i = base tensor i)
  int32_t root = -1;
  int32_t n_base = 0;
  std::vector<int32_t> postorder; // internal nodes in merge order (children first)
  std::vector<int32_t> dfs_post;  // internal nodes in depth-first post-order:
                                  // every subtree is a contiguous range
  // var -> internal nodes whose tensor holds it
  std::vector<std::vector<int32_t>> var_nodes;
};

// Greedy pairwise order: repeatedly contract the pair of tensors sharing a
// variable that minimises |out| - |A| - |B| (sizes in entries), lowest ids on
// ties; a variable is summed out as soon as no other tensor holds it.
// Disconnected scalars are joined at the end.
Tree greedy_tree(const Network& net);

// Tree from a min-fill elimination order of the variables: the tensors
// holding the eliminated variable are contracted pairwise (smallest result
// first); deterministic.
Tree minfill_tree(const Network& net);

// Simulated-annealing refinement of a contraction tree by local rotations
// (the tree-annealing approach to contraction orders).  Each sweep visits
// every internal node once in random order and proposes one rotation; the
// local change of log2(MACs) of the two affected contractions, plus the
// space terms, is accepted with probability min(1, exp(-beta * change)),
// beta rising linearly from beta0 to beta1.
struct RefineOptions {
  int sweeps = 0;          // 0: return the input tree
  double beta0 = 1.0, beta1 = 30.0;
  int sc_target = 0;       // <= 0: the input tree's space complexity
  double sc_weight = 4.0;  // per log2 entry above sc_target
  int log2_target = 0;     // T_target of the overflow measure rho
  double rho_weight = 0.0; // per log2 entry above log2_target
  uint64_t seed = 1;
  double deadline = 0;     // absolute wall time (s) or 0: stop sweeping past it
  // memory traffic in the move score: a contraction costs its
  // multiply-accumulates plus kappa per entry it moves (operands read,
  // permuted into layout and read again, output written); 0: MACs only
  double kappa = 0;
};
Tree refine_tree(const Network& net, const Tree& t, const RefineOptions& o);

// log2 of time (multiply-accumulates) and space (largest intermediate) of the
// tree when the variables in `fixed` (bitmask over vars, may be empty) are
// sliced away.
struct Complexity {
  double tc_log2 = 0;
  int32_t sc = 0;
};
Complexity complexity(const Tree& t, const std::vector<uint64_t>& fixed);

// Cost model of the tree with the variables in `fixed` sliced away, in
// multiply-accumulate units: per contraction its multiply-accumulates plus
// kappa per entry moved (3 |A| + 3 |B| + |C|: each operand read, permuted
// into the product's layout and read again, the output written).  Splits
// into the contractions of subtrees without a fixed variable, which run once
// however many branches fix it ("shared"), and the others, once per branch.
struct TimeCost {
  double shared = 0, branch = 0;
};
TimeCost time_cost(const Tree& t, const std::vector<uint64_t>& fixed, double kappa);

inline bool bit_get(const std::vector<uint64_t>& b, int v) {
  return (size_t)(v >> 6) < b.size() && ((b[v >> 6] >> (v & 63)) & 1);
}
inline void bit_set(std::vector<uint64_t>& b, int v) {
  if ((size_t)(v >> 6) >= b.size()) b.resize((v >> 6) + 1, 0);
  b[v >> 6] |= 1ull << (v & 63);
}

}  // namespace bbtn
