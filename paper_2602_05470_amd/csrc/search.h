// Branch-and-bound over the tensor network ("Branch-and-Bound Tensor
// Network" section): a node fixes a set of variables; its sub-network's
// problem size rho (Eq. 4) is the total overflow of the intermediates of the
// contraction tree above T_target; a node with rho = 0 is a leaf whose
// sub-network is contracted on the device.  Other nodes branch on a region R:
// the feasible set F(R) keeps, for every boundary state, only the
// locally-optimal interiors (ties kept) that also pass global pruning; the
// branches D(R) are disjoint cubes covering F(R), chosen to minimise the
// branching factor gamma of the characteristic equation.
#pragma once
#include <atomic>
#include <functional>
#include <vector>
#include "tree.h"

namespace bbtn {

struct LeafGroup {
  std::vector<uint64_t> mask;     // fixed variables S
  std::vector<int32_t> vars;      // S ascending
  std::vector<uint8_t> assign;    // count * |S| states
  int64_t count = 0;
};

struct SearchStats {
  uint64_t nodes = 0, pruned = 0, leaves = 0;
  double gamma_sum = 0;
};

// Orders candidate branching variables: returns one score per variable
// (higher = branch earlier) for the free variables of a node.  Empty
// function: the overflow-participation heuristic.
using VarScorer = std::function<void(const std::vector<uint64_t>& fixed,
                                     const std::vector<int16_t>& sizes,
                                     const std::vector<double>& heuristic,
                                     std::vector<double>& score)>;

struct SearchOptions {
  int log2_target = 10;
  int region_max = 8;
  int64_t incumbent = INT64_MIN;  // value of a known configuration (max form)
  // values only (no counts): branches that cannot beat the incumbent are
  // pruned (non-strict; the caller keeps the incumbent's configuration) and
  // boundary equivalence keeps one optimal interior per boundary state
  bool values_only = false;
  double deadline = 0;            // absolute wall time (s) or 0
  // when set: the search stops with BBTN_E_TIMEOUT once it has expanded more
  // nodes than this (read at every node; may be lowered while it runs)
  const std::atomic<uint64_t>* node_limit = nullptr;
  VarScorer scorer;
  // variables fixed at the root, with their states (the spin fixed by the
  // spin-flip symmetry)
  std::vector<std::pair<int32_t, uint8_t>> prefix;
};

void bb_search(const Network& net, const Tree& tree, const SearchOptions& opt,
               std::vector<LeafGroup>& leaves, SearchStats& stats);

// Upper bound (max form) of a node: constant + sum over tensors of the
// largest finite entry consistent with the fixed states.  INT64_MIN if a
// tensor has no consistent finite entry.
int64_t node_bound(const Network& net, const std::vector<uint64_t>& fixed,
                   const std::vector<uint8_t>& x);

// The spin whose fixing saves the most contraction work: largest overflow
// participation sum over intermediates of max(0, log2 size - log2_target)
// (the search's own branching priority), then largest MAC share sum over
// contractions holding it of 2^(log2 MACs - the largest); lowest id on ties.
// -1 for a network without variables.
int32_t flip_variable(const Network& net, const Tree& tree, int log2_target);

// Upper bound on the weight of an independent set that agrees with the
// fixed states (independent-set networks; INT64_MAX otherwise): the fixed
// vertices in the set, plus, per clique of the network's clique partition,
// the largest weight of a vertex that can still join (free, no neighbour in
// the set); nothing for a clique that already holds a vertex of the set.
int64_t clique_bound(const Network& net, const std::vector<uint64_t>& fixed,
                     const std::vector<uint8_t>& x);

// rho of Eq. 4 given per-internal-node free-variable counts.
int64_t rho_of(const Tree& t, const std::vector<int16_t>& sizes, int log2_target);

// Free-variable counts of the tree's internal nodes (indexed by node id)
// for a fixed-variable mask.
std::vector<int16_t> node_sizes(const Tree& t, const std::vector<uint64_t>& fixed);

// Value (max form, including the folded constant) of a full assignment of
// the network's variables, or INT64_MIN if infeasible.
int64_t network_value(const Network& net, const std::vector<uint8_t>& x);

// Local search for a good configuration of the original instance; returns
// states per variable (0/1).
std::vector<uint8_t> local_search_spinglass(int32_t n, int32_t m, const int32_t* uv,
                                            const int32_t* J, const int32_t* h, int sweeps,
                                            uint64_t seed);
std::vector<uint8_t> local_search_mwis(int32_t n, int32_t m, const int32_t* uv,
                                       const int32_t* w, int restarts, uint64_t seed);

// The contraction order used for a structure: the greedy tree (n = 0), the
// min-fill tree (n < 0), or the cheapest of the greedy tree, n <= 64
// annealed refinements of it, the min-fill tree and one refinement of that,
// each scored by a branch-and-bound search of `net` with `probe`: a cost
// model of its leaves (multiply-accumulates plus memory traffic) plus a
// fixed weight per search node.  The choice is deterministic.  `complete`
// (optional) is set to false when probe.deadline cut the choice short (the
// greedy tree is then returned).
Tree choose_order(const Network& net, int n, const SearchOptions& probe,
                  bool* complete = nullptr);

// The candidates of choose_order with n refinements (n >= 1) and n more
// refinements under varied annealing objectives (overflow weight 0.25 or
// 0.1, memory weight 0, 4 or 6), each probed with a budget of 2^22 search
// nodes, those that finish ranked by their score, cheapest first (ties in
// candidate order).  For choosing among the first few by measurement.
std::vector<Tree> rank_orders(const Network& net, int n, const SearchOptions& probe);

}  // namespace bbtn
