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

// log2 of time (multiply-accumulates) and space (largest intermediate) of the
// tree when the variables in `fixed` (bitmask over vars, may be empty) are
// sliced away.
struct Complexity {
  double tc_log2 = 0;
  int32_t sc = 0;
};
Complexity complexity(const Tree& t, const std::vector<uint64_t>& fixed);

inline bool bit_get(const std::vector<uint64_t>& b, int v) {
  return (size_t)(v >> 6) < b.size() && ((b[v >> 6] >> (v & 63)) & 1);
}
inline void bit_set(std::vector<uint64_t>& b, int v) {
  if ((size_t)(v >> 6) >= b.size()) b.resize((v >> 6) + 1, 0);
  b[v >> 6] |= 1ull << (v & 63);
}

}  // namespace bbtn
