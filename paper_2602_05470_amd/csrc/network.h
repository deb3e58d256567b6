// Tensor network of a spin glass or MWIS instance in the counting tropical
// algebra, max form ("Tropical Tensor Networks" section: edge matrices B^ij,
// vertex vectors w^i, bond index s_i shared by every tensor touching i).
#pragma once
#include <array>
#include <memory>
#include <vector>
#include "common.h"

namespace bbtn {

// The 32 largest primes below 2^31, descending (computed once).
const std::vector<uint32_t>& prime_table();

// Exact modular helpers (host).
inline uint32_t addmod(uint32_t a, uint32_t b, uint32_t p) {
  uint64_t s = (uint64_t)a + b;
  return (uint32_t)(s >= p ? s - p : s);
}
inline uint32_t mulmod(uint32_t a, uint32_t b, uint32_t p) {
  return (uint32_t)((uint64_t)a * b % p);
}

constexpr int NP = BBTN_MAX_PRIMES;

// A base tensor over `vars` (ascending ids).  Entry e (bit j = state of
// vars[j]) has value val[e] (NEG = infeasible) and count residues
// res[p * size + e] modulo prime_table()[p] for every p < NP.
struct BaseTensor {
  std::vector<int32_t> vars;
  std::vector<int32_t> val;
  std::vector<uint32_t> res;
  int64_t size() const { return (int64_t)val.size(); }
};

// One exact elimination done while simplifying the network: `var` was
// summed out of a tensor over `tvars` with values `tval`.  Replaying these in
// reverse, choosing the best state of `var` given the others, recovers an
// optimal configuration of the eliminated variables.
struct PeelRec {
  int32_t var;
  std::vector<int32_t> tvars;
  std::vector<int32_t> tval;
};

// The graph of an independent-set instance, kept for a bound the tensors do
// not give: a partition of the vertices into cliques (an independent set
// holds at most one vertex of each), built greedily.
struct MisGraph {
  std::vector<std::vector<int32_t>> adj;      // neighbours, ascending
  std::vector<int64_t> w;                     // vertex weights
  std::vector<std::vector<int32_t>> cliques;  // disjoint, covering every vertex
};

struct Network {
  int32_t n = 0;
  bool spin = true;                 // spin glass (true) or MWIS (false)
  std::vector<BaseTensor> tensors;  // after simplification
  int64_t const_val = 0;            // folded scalar factor (max form)
  std::array<uint32_t, NP> const_res{};
  bool infeasible = false;
  std::vector<PeelRec> peel;        // in elimination order
  int64_t abs_sum = 0;              // sum |J| + |h| (or sum w)
  bool zero_field = false;
  std::shared_ptr<const MisGraph> mis;  // independent-set instances only          // spin glass without fields: H(sigma) = H(-sigma)
  // every tensor's entries back to back, in tensor order: the value plane
  // then the residue planes of the first NP_FLAT primes (flat_total entries
  // each), for uploads of whole planes
  std::vector<uint32_t> flat;
  int64_t flat_total = 0;
};

constexpr int NP_FLAT = KMAX + 1;  // one pass's primes and its check prime

Network build_spinglass(int32_t n, int32_t m, const int32_t* uv, const int32_t* J,
                        const int32_t* h);
Network build_mwis(int32_t n, int32_t m, const int32_t* uv, const int32_t* w);

// Exact simplification: absorb tensors whose variables are a subset of
// another's (tropical product), sum out variables held by a single tensor
// (tropical sum, recorded in `peel`), fold scalars into the constant.
void simplify(Network& net);

// Fill net.flat from the tensors (done by the builders).
void flatten(Network& net);

}  // namespace bbtn
