// Step program for the contraction of one branch sub-network
// T|_{s_S = x} (Eq. 3): the contraction tree of the whole network with the
// fixed variables S removed from every tensor.  Every branch that fixes the
// same variable set S shares this program (same topology, different
// contents), so the program runs batched over all of them.
#pragma once
#include <cmath>
#include <vector>
#include "tree.h"

namespace bbtn {

// Where a buffer lives.  Subtrees of the contraction tree that hold no fixed
// variable are the same for every branch: their steps ("shared" steps) run
// once per pass.  Their intermediates live in a per-subtree scratch and the
// root of each such subtree in a shared region that every branch reads; the
// remaining ("branch") steps run per branch in the branch workspace.
enum Region { R_BRANCH = 0, R_SUBTREE = 1, R_SHARED = 2 };

// One operand of a step: a base tensor sliced per branch, or an
// intermediate buffer; gathered into the step's required layout unless it
// is already stored that way.
struct Operand {
  bool base = false;
  int32_t id = -1;                  // base tensor id or buffer id
  bool direct = false;              // intermediate already in required layout
  int32_t r_in = 0;                 // rank of the source (all vars for base)
  std::vector<int32_t> src_bits;    // required-layout bit j <- source bit
  int32_t temp = -1;                // buffer receiving the gathered operand
  std::vector<std::pair<int32_t, int32_t>> fixed_pos;  // (source bit, var) of fixed vars sliced per branch
  int32_t base_op = -1;             // index into GroupPlan::base_ops, or -1
};

// C[b, m, n] = (+)_k A[b, m, k] (.) B[b, k, n], bit layouts (low bits first):
//   A: [K][M][batch], B: [N][K][batch], C: [N][M][batch].
struct Step {
  int32_t node = -1;
  bool shared = false;              // runs once per pass (no fixed variable below)
  int32_t rb = 0, rm = 0, rn = 0, rk = 0;
  Operand a, b;
  int32_t out = -1;                 // buffer id of C
  std::vector<int32_t> a_vars, b_vars, c_vars;  // layouts (variable ids)
  double macs() const { return std::ldexp(1.0, rb + rm + rn + rk); }
};

struct GroupPlan {
  std::vector<uint64_t> fixed;      // bitmask of fixed variables S
  std::vector<int32_t> fixed_vars;  // S, ascending
  std::vector<Step> steps;          // children before parents
  std::vector<int64_t> buf_entries; // entries of every buffer (per branch for R_BRANCH)
  std::vector<int64_t> buf_off;     // entry offset of every buffer within its region
  std::vector<int32_t> buf_region;  // Region of every buffer
  int64_t peak = 0;                 // per-branch entries of the branch workspace
  int64_t subtree_peak = 0;         // entries of the subtree scratch
  int64_t shared_total = 0;         // entries of the shared region
  // maximal shared subtrees as [begin, end) ranges of `steps`
  std::vector<std::pair<int32_t, int32_t>> shared_ranges;
  std::vector<int32_t> folded;      // base tensors with every variable fixed
  int32_t root_buf = -1;            // buffer of the final scalar, -1 if none
  // operands read with per-branch fixed bits (base tensors, and roots of
  // deferred subtrees): (step, 0=A / 1=B)
  std::vector<std::pair<int32_t, int32_t>> base_ops;
  int32_t max_rank = 0;             // largest tensor rank in the program
  bool keep_all = false;            // every buffer kept, operands materialised
  double macs = 0;                  // per branch (branch steps)
  double shared_macs = 0;           // per pass (shared steps)
  int32_t n_branch_steps = 0;
  uint64_t uid = 0;                 // unique over the process (keys of captured graphs)
};

// keep_all: never reuse buffers and materialise every operand in its
// required layout (values-only recontraction for configuration recovery);
// keep_all plans share nothing.  defer_log2 > 0: subtrees holding fixed
// variables whose tensors, with those variables kept, have at most
// 2^defer_log2 entries are contracted once per pass and sliced per branch
// afterwards (their steps are shared).
GroupPlan build_plan(const Network& net, const Tree& tree,
                     const std::vector<uint64_t>& fixed, bool keep_all, int defer_log2 = 0);

}  // namespace bbtn
