#include "search.h"

#include <thread>

#include "scorer.h"

#include <chrono>
#include <cmath>
#include <map>
#include <random>
#include <unordered_map>

namespace bbtn {

static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

std::vector<int16_t> node_sizes(const Tree& t, const std::vector<uint64_t>& fixed) {
  std::vector<int16_t> s(t.nodes.size(), 0);
  for (int id : t.postorder) {
    int c = 0;
    for (int v : t.nodes[id].vars) c += !bit_get(fixed, v);
    s[id] = (int16_t)c;
  }
  return s;
}

int64_t rho_of(const Tree& t, const std::vector<int16_t>& sizes, int log2_target) {
  int64_t r = 0;
  for (int id : t.postorder) r += std::max(0, sizes[id] - log2_target);
  return r;
}

// Largest finite entry of tensor T consistent with the fixed states (and
// with the region assignment: vars in `rvars` take the bits of `rx`).
static int64_t tensor_max(const BaseTensor& T, const std::vector<uint64_t>& fixed,
                          const std::vector<uint8_t>& x, const int32_t* rpos = nullptr,
                          uint32_t rx = 0) {
  const int r = (int)T.vars.size();
  uint32_t cmask = 0, cval = 0;  // constrained positions and their states
  for (int j = 0; j < r; ++j) {
    const int v = T.vars[j];
    if (rpos && rpos[j] >= 0) {
      cmask |= 1u << j;
      cval |= ((rx >> rpos[j]) & 1u) << j;
    } else if (bit_get(fixed, v)) {
      cmask |= 1u << j;
      cval |= (uint32_t)(x[v] & 1) << j;
    }
  }
  int64_t best = INT64_MIN;
  for (int64_t e = 0; e < T.size(); ++e) {
    if (((uint32_t)e & cmask) != cval) continue;
    const int32_t v = T.val[e];
    if (v > NEG_CUT && v > best) best = v;
  }
  return best;
}

int64_t node_bound(const Network& net, const std::vector<uint64_t>& fixed,
                   const std::vector<uint8_t>& x) {
  int64_t b = net.const_val;
  for (const auto& T : net.tensors) {
    const int64_t m = tensor_max(T, fixed, x);
    if (m == INT64_MIN) return INT64_MIN;
    b += m;
  }
  return b;
}

int64_t clique_bound(const Network& net, const std::vector<uint64_t>& fixed,
                     const std::vector<uint8_t>& x) {
  if (!net.mis) return INT64_MAX;
  const MisGraph& g = *net.mis;
  const int n = (int)g.w.size();
  // a vertex can still join the set iff it is free and no neighbour is in
  std::vector<char> out(n, 0);
  int64_t b = 0;
  for (int v = 0; v < n; ++v) {
    if (!bit_get(fixed, v)) continue;
    out[v] = 1;
    if (x[v] & 1) {
      b += g.w[v];
      for (int u : g.adj[v]) out[u] = 1;
    }
  }
  // at most one vertex of each clique; a clique holding a chosen vertex
  // adds nothing more
  for (const auto& q : g.cliques) {
    int64_t best = 0;
    bool has = false;
    for (int v : q) {
      if (bit_get(fixed, v) && (x[v] & 1)) { has = true; break; }
      if (!out[v]) best = std::max(best, g.w[v]);
    }
    if (!has) b += best;
  }
  return b;
}

int32_t flip_variable(const Network& net, const Tree& tree, int log2_target) {
  if (net.n <= 0) return -1;
  std::vector<double> over(net.n, 0.0), mac(net.n, 0.0);
  double top = 0;
  for (int32_t id : tree.postorder) {
    const TNode& nd = tree.nodes[id];
    const auto& A = tree.nodes[nd.left].vars;
    const auto& Bv = tree.nodes[nd.right].vars;
    std::vector<int32_t> u;
    std::set_union(A.begin(), A.end(), Bv.begin(), Bv.end(), std::back_inserter(u));
    top = std::max(top, (double)u.size());
  }
  for (int32_t id : tree.postorder) {
    const TNode& nd = tree.nodes[id];
    const double ov = std::max(0, (int)nd.vars.size() - log2_target);
    for (int32_t v : nd.vars) over[v] += ov;
    const auto& A = tree.nodes[nd.left].vars;
    const auto& Bv = tree.nodes[nd.right].vars;
    std::vector<int32_t> u;
    std::set_union(A.begin(), A.end(), Bv.begin(), Bv.end(), std::back_inserter(u));
    const double w = std::ldexp(1.0, (int)u.size() - (int)top);
    for (int32_t v : u) mac[v] += w;
  }
  int32_t best = -1;
  for (int32_t v = 0; v < net.n; ++v) {
    if (mac[v] == 0 && over[v] == 0) continue;
    if (best < 0 || over[v] > over[best] || (over[v] == over[best] && mac[v] > mac[best]))
      best = v;
  }
  return best;
}

int64_t network_value(const Network& net, const std::vector<uint8_t>& x) {
  if (net.infeasible) return INT64_MIN;
  int64_t v = net.const_val;
  for (const auto& T : net.tensors) {
    int64_t e = 0;
    for (size_t j = 0; j < T.vars.size(); ++j) e |= (int64_t)(x[T.vars[j]] & 1) << j;
    if (T.val[e] <= NEG_CUT) return INT64_MIN;
    v += T.val[e];
  }
  return v;
}

namespace {

struct Node {
  std::vector<uint64_t> fixed;
  std::vector<uint8_t> x;
  std::vector<int16_t> sizes;
  int64_t rho = 0;
  int64_t bound = 0;
};

struct Cube {
  uint32_t mask, val;  // over region positions
};

struct Searcher {
  const Network& net;
  const Tree& tree;
  const SearchOptions& opt;
  std::vector<std::vector<int32_t>> var_tensors, nbr;
  std::vector<int32_t> dec;      // scratch: decrements per tree node
  std::vector<int32_t> touched;  // scratch: tree nodes with dec > 0
  std::map<std::vector<uint64_t>, int> group_of;
  std::map<std::vector<uint64_t>, std::vector<int32_t>> rule_memo;  // fixed set -> region

  Searcher(const Network& n, const Tree& t, const SearchOptions& o) : net(n), tree(t), opt(o) {
    var_tensors.assign(net.n, {});
    nbr.assign(net.n, {});
    for (int i = 0; i < (int)net.tensors.size(); ++i)
      for (int v : net.tensors[i].vars) var_tensors[v].push_back(i);
    for (int v = 0; v < net.n; ++v) {
      for (int ti : var_tensors[v])
        for (int u : net.tensors[ti].vars)
          if (u != v) nbr[v].push_back(u);
      std::sort(nbr[v].begin(), nbr[v].end());
      nbr[v].erase(std::unique(nbr[v].begin(), nbr[v].end()), nbr[v].end());
    }
    dec.assign(tree.nodes.size(), 0);
    // largest entry of every tensor of rank <= 3 under each constraint
    // pattern (per variable: free, fixed to 0, fixed to 1)
    tm_off.assign(net.tensors.size(), -1);
    for (size_t i = 0; i < net.tensors.size(); ++i) {
      const BaseTensor& T = net.tensors[i];
      const int r = (int)T.vars.size();
      if (r > 3) continue;
      int patterns = 1;
      for (int j = 0; j < r; ++j) patterns *= 3;
      tm_off[i] = (int32_t)tm_tab.size();
      for (int code = 0; code < patterns; ++code) {
        uint32_t cmask = 0, cval = 0;
        for (int j = 0, c = code; j < r; ++j, c /= 3)
          if (c % 3) {
            cmask |= 1u << j;
            cval |= (uint32_t)(c % 3 - 1) << j;
          }
        int64_t best = INT64_MIN;
        for (int64_t e = 0; e < T.size(); ++e)
          if (((uint32_t)e & cmask) == cval && T.val[e] > NEG_CUT && T.val[e] > best) best = T.val[e];
        tm_tab.push_back(best);
      }
    }
  }

  std::vector<int64_t> tm_tab;
  std::vector<int32_t> tm_off;
  // tensor_max of tensor t through the pattern table (same result)
  int64_t tmax(int t, const std::vector<uint64_t>& fixed, const std::vector<uint8_t>& x,
               const int32_t* rpos = nullptr, uint32_t rx = 0) const {
    const BaseTensor& T = net.tensors[t];
    if (tm_off[t] < 0) return tensor_max(T, fixed, x, rpos, rx);
    int code = 0, mul = 1;
    for (size_t j = 0; j < T.vars.size(); ++j, mul *= 3) {
      const int v = T.vars[j];
      if (rpos && rpos[j] >= 0) code += mul * (1 + (int)((rx >> rpos[j]) & 1u));
      else if (bit_get(fixed, v)) code += mul * (1 + (x[v] & 1));
    }
    return tm_tab[tm_off[t] + code];
  }

  // rho reduction when the variables vs (all free at `n`) are fixed too.
  int64_t drho(const Node& n, const std::vector<int32_t>& vs) {
    for (int v : vs)
      for (int id : tree.var_nodes[v]) {
        if (dec[id]++ == 0) touched.push_back(id);
      }
    int64_t d = 0;
    const int t = opt.log2_target;
    for (int id : touched) {
      const int s0 = n.sizes[id], s1 = s0 - dec[id];
      d += std::max(0, s0 - t) - std::max(0, s1 - t);
      dec[id] = 0;
    }
    touched.clear();
    return d;
  }

  // Branching factor of the characteristic equation: gamma >= 1 with
  // sum_i gamma^(-delta rho_i) = 1, solved for lambda = ln gamma by Newton's
  // method (the sum is convex and decreasing in lambda; starting left of the
  // root, the iterates increase monotonically to it).
  static double gamma_of(const std::vector<std::pair<int64_t, int64_t>>& terms) {
    int64_t total = 0;
    for (auto& t : terms) {
      if (t.first <= 0) return INFINITY;
      total += t.second;
    }
    if (total == 0) return 0.0;
    if (total == 1) return 1.0;
    // one term: count * gamma^(-d) = 1 has the closed form gamma = count^(1/d)
    if (terms.size() == 1)
      return std::exp(std::log((double)terms[0].second) / (double)terms[0].first);
    double lam = 0;
    for (int it = 0; it < 60; ++it) {
      double f = -1, df = 0;
      for (auto& t : terms) {
        const double e = (double)t.second * std::exp(-lam * (double)t.first);
        f += e;
        df -= (double)t.first * e;
      }
      const double step = f / df;
      lam -= step;
      if (std::fabs(step) <= 1e-12 * std::max(1.0, lam)) break;
    }
    return std::exp(lam);
  }

  struct Eval {
    double gamma = INFINITY;
    std::vector<int32_t> region;
    std::vector<Cube> cubes;
    // rho reduction per fixed subset of the region (few distinct subsets)
    std::vector<std::pair<uint32_t, int64_t>> drho;
    const int64_t* drho_of(uint32_t mask) const {
      for (const auto& d : drho)
        if (d.first == mask) return &d.second;
      return nullptr;
    }
  };

  // evaluation scratch, reused across calls (one search runs on one thread)
  std::vector<int32_t> e_tt;                 // tensors touching the region
  std::vector<int32_t> e_rpos, e_rpos_off;   // region position of each tensor var, or -1
  std::vector<char> e_inside;                // tensor has no free variable outside R
  std::vector<int64_t> e_base;               // tensor's largest consistent entry at the node
  std::vector<int32_t> e_tpos, e_tpos_off;   // region positions of a tensor's region vars
  std::vector<int64_t> e_tval;               // largest entry per state of those vars
  std::vector<int64_t> e_tval_off;
  std::vector<int64_t> e_local, e_bnd, e_gmax;
  std::vector<char> e_taken;
  std::vector<uint32_t> e_masks;
  std::vector<uint64_t> e_keys;
  std::vector<int32_t> e_vs;

  Eval evaluate(const Node& n, const std::vector<int32_t>& R) {
    Eval ev;
    ev.region = R;
    const int r = (int)R.size();
    std::vector<int32_t>& tt = e_tt;
    tt.clear();
    for (int v : R) tt.insert(tt.end(), var_tensors[v].begin(), var_tensors[v].end());
    if (R.size() > 1) {  // one variable's tensor list is already ascending
      std::sort(tt.begin(), tt.end());
      tt.erase(std::unique(tt.begin(), tt.end()), tt.end());
    }
    const size_t nt = tt.size();
    // per touching tensor: region positions of its vars; inside/cross; base max
    e_rpos.clear();
    e_rpos_off.assign(nt + 1, 0);
    e_inside.assign(nt, 1);
    e_base.resize(nt);
    uint32_t bmask = 0;
    for (size_t i = 0; i < nt; ++i) {
      const BaseTensor& T = net.tensors[tt[i]];
      e_rpos_off[i] = (int32_t)e_rpos.size();
      bool cross = false;
      for (size_t j = 0; j < T.vars.size(); ++j) {
        const int v = T.vars[j];
        int pos = -1;
        for (int q = 0; q < r; ++q)
          if (R[q] == v) { pos = q; break; }
        e_rpos.push_back(pos);
        if (pos < 0 && !bit_get(n.fixed, v)) cross = true;
      }
      e_inside[i] = !cross;
      if (cross)
        for (size_t j = 0; j < T.vars.size(); ++j)
          if (e_rpos[e_rpos_off[i] + j] >= 0) bmask |= 1u << e_rpos[e_rpos_off[i] + j];
      e_base[i] = tmax(tt[i], n.fixed, n.x);
    }
    e_rpos_off[nt] = (int32_t)e_rpos.size();
    const uint32_t nx = 1u << r;
    // per touching tensor: table of its largest consistent entry over the
    // states of its region variables (at most 2^|T| entries), so that every
    // region configuration costs one table lookup per tensor
    e_tpos.clear();
    e_tpos_off.assign(nt + 1, 0);
    e_tval.clear();
    e_tval_off.assign(nt + 1, 0);
    for (size_t i = 0; i < nt; ++i) {
      const BaseTensor& T = net.tensors[tt[i]];
      const int32_t* rp = &e_rpos[e_rpos_off[i]];
      e_tpos_off[i] = (int32_t)e_tpos.size();
      for (size_t j = 0; j < T.vars.size(); ++j)
        if (rp[j] >= 0) e_tpos.push_back(rp[j]);
      const int nj = (int)e_tpos.size() - e_tpos_off[i];
      e_tval_off[i] = (int64_t)e_tval.size();
      for (uint32_t y = 0; y < (1u << nj); ++y) {
        uint32_t rx = 0;
        for (int q = 0; q < nj; ++q) rx |= ((y >> q) & 1u) << e_tpos[e_tpos_off[i] + q];
        e_tval.push_back(tmax(tt[i], n.fixed, n.x, rp, rx));
      }
    }
    e_tpos_off[nt] = (int32_t)e_tpos.size();
    e_tval_off[nt] = (int64_t)e_tval.size();
    // Nothing can be pruned when every region variable is on the boundary
    // (boundary equivalence has one configuration per boundary state), no
    // tensor has an infeasible entry under any region state, and even the
    // smallest bound over region states reaches the incumbent.  Then F(R) is
    // every configuration and the enumeration below is skipped.
    {
      bool may_prune = bmask != nx - 1;
      int64_t minb = n.bound;
      for (size_t i = 0; i < nt; ++i) {
        int64_t mn = INT64_MAX;
        for (int64_t q = e_tval_off[i]; q < e_tval_off[i + 1]; ++q) mn = std::min(mn, e_tval[q]);
        if (mn == INT64_MIN) { may_prune = true; break; }
        minb += mn - e_base[i];
      }
      if (!may_prune && (opt.values_only ? minb > opt.incumbent : minb >= opt.incumbent)) {
        ev.cubes.reserve(nx);
        for (uint32_t x = 0; x < nx; ++x) ev.cubes.push_back(Cube{nx - 1, x});
        const int64_t d = drho(n, R);
        ev.drho.push_back({nx - 1, d});
        ev.gamma = gamma_of({{d, (int64_t)nx}});
        return ev;
      }
    }
    e_local.resize(nx);
    e_bnd.resize(nx);
    e_gmax.assign(nx, INT64_MIN);  // indexed by x & bmask
    for (uint32_t x = 0; x < nx; ++x) {
      int64_t lc = 0, b = n.bound;
      bool feas = true;
      for (size_t i = 0; i < nt; ++i) {
        uint32_t y = 0;
        const int32_t q0 = e_tpos_off[i], nq = e_tpos_off[i + 1] - q0;
        for (int q = 0; q < nq; ++q) y |= ((x >> e_tpos[q0 + q]) & 1u) << q;
        const int64_t m = e_tval[e_tval_off[i] + y];
        if (m == INT64_MIN) { feas = false; break; }
        b += m - e_base[i];
        if (e_inside[i]) lc += m;
      }
      e_local[x] = feas ? lc : INT64_MIN;
      e_bnd[x] = feas ? b : INT64_MIN;
      if (feas && lc > e_gmax[x & bmask]) e_gmax[x & bmask] = lc;
    }
    const uint32_t full = nx - 1;
    if (opt.values_only) e_taken.assign(nx, 0);
    for (uint32_t x = 0; x < nx; ++x) {
      if (e_local[x] == INT64_MIN) continue;
      if (e_local[x] != e_gmax[x & bmask]) continue;    // boundary equivalence
      if (opt.values_only) {
        // one optimal interior per boundary state; prune what cannot beat
        // the incumbent
        if (e_taken[x & bmask] || e_bnd[x] <= opt.incumbent) continue;
        e_taken[x & bmask] = 1;
      } else if (e_bnd[x] < opt.incumbent) {
        continue;                                        // global pruning (strict)
      }
      ev.cubes.push_back(Cube{full, x});
    }
    // delta rho per fixed subset of the region (cached in ev.drho)
    auto dr = [&](uint32_t mask) {
      if (const int64_t* d = ev.drho_of(mask)) return *d;
      e_vs.clear();
      for (int j = 0; j < r; ++j)
        if (mask >> j & 1) e_vs.push_back(R[j]);
      const int64_t d = drho(n, e_vs);
      ev.drho.push_back({mask, d});
      return d;
    };
    // gamma of a cover: one term per distinct fixed subset, ascending
    auto gam = [&](const std::vector<Cube>& cs) {
      e_masks.clear();
      for (auto& c : cs) e_masks.push_back(c.mask);
      std::sort(e_masks.begin(), e_masks.end());
      std::vector<std::pair<int64_t, int64_t>> terms;
      for (size_t i = 0; i < e_masks.size();) {
        size_t j = i;
        while (j < e_masks.size() && e_masks[j] == e_masks[i]) ++j;
        terms.push_back({dr(e_masks[i]), (int64_t)(j - i)});
        i = j;
      }
      return gamma_of(terms);
    };
    ev.gamma = gam(ev.cubes);
    // with nothing pruned, freeing variables only reproduces a smaller region
    // (evaluated separately); otherwise free variables of the cover
    if (ev.cubes.size() == nx) return ev;
    // free variables of the cover while it lowers gamma (cubes stay disjoint
    // and cover exactly the same configurations)
    for (;;) {
      int bestj = -1;
      double bestg = ev.gamma;
      std::vector<Cube> bestc;
      e_keys.clear();
      for (auto& c : ev.cubes) e_keys.push_back(((uint64_t)c.mask << 32) | c.val);
      std::sort(e_keys.begin(), e_keys.end());
      for (int j = 0; j < r; ++j) {
        const uint32_t bj = 1u << j;
        std::vector<Cube> merged;
        bool any = false;
        for (auto& c : ev.cubes) {
          if (!(c.mask & bj)) { merged.push_back(c); continue; }
          const uint64_t partner = ((uint64_t)c.mask << 32) | (c.val ^ bj);
          if (std::binary_search(e_keys.begin(), e_keys.end(), partner)) {
            if (!(c.val & bj)) { merged.push_back(Cube{c.mask & ~bj, c.val}); any = true; }
          } else {
            merged.push_back(c);
          }
        }
        if (!any) continue;
        const double g = gam(merged);
        if (g < bestg - 1e-12) { bestg = g; bestj = j; bestc = std::move(merged); }
      }
      if (bestj < 0) break;
      ev.gamma = bestg;
      ev.cubes = std::move(bestc);
    }
    return ev;
  }

  // lowest gamma; on a tie (within 1e-9 relative) the larger step, which
  // reaches the same leaves through fewer search nodes
  static bool better(const Eval& ev, const Eval& best) {
    const double tol = 1e-9 * std::max(1.0, std::isfinite(best.gamma) ? best.gamma : 1.0);
    return ev.gamma < best.gamma - tol ||
           (std::fabs(ev.gamma - best.gamma) <= tol && ev.cubes.size() > best.cubes.size());
  }

  // Grow a region from `seed` by adjacency (highest score first, lowest id on
  // ties) and keep the best branching rule over its prefixes.
  Eval best_from_seed(const Node& n, int seed, const std::vector<double>& score) {
    std::vector<int32_t> order{seed};
    while ((int)order.size() < opt.region_max) {
      int pick = -1;
      for (int v : order)
        for (int u : nbr[v]) {
          if (bit_get(n.fixed, u)) continue;
          if (std::find(order.begin(), order.end(), u) != order.end()) continue;
          if (pick < 0 || score[u] > score[pick] || (score[u] == score[pick] && u < pick)) pick = u;
        }
      if (pick < 0) break;
      order.push_back(pick);
    }
    Eval best;
    for (int r = 1; r <= (int)order.size(); ++r) {
      std::vector<int32_t> R(order.begin(), order.begin() + r);
      Eval ev = evaluate(n, R);
      if (better(ev, best)) best = std::move(ev);
      if (best.gamma == 0.0) break;
    }
    return best;
  }

  void heuristic(const Node& n, std::vector<double>& heur, std::vector<int32_t>& cand) {
    cand.clear();
    for (int v = 0; v < net.n; ++v) {
      heur[v] = 0;
      if (bit_get(n.fixed, v)) continue;
      double s = 0;
      for (int id : tree.var_nodes[v]) s += std::max(0, n.sizes[id] - opt.log2_target);
      heur[v] = s;
      if (s > 0) cand.push_back(v);
    }
  }

  // Children of a node under a branching rule: bounded, pruned if below the
  // incumbent (strict).
  // nodes already expanded or pruned: their buffers are reused for new
  // children (the search makes a few thousand nodes per instance)
  std::vector<Node> spare;
  Node take() {
    if (spare.empty()) return Node();
    Node nd = std::move(spare.back());
    spare.pop_back();
    return nd;
  }
  std::vector<int32_t> c_tt, c_newly;
  std::vector<int64_t> c_base;

  void children(const Node& n, const Eval& best, std::vector<Node>& out, SearchStats& st) {
    // tensors touched by the region and their largest entries at the node
    std::vector<int32_t>& tt = c_tt;
    tt.clear();
    for (int v : best.region) tt.insert(tt.end(), var_tensors[v].begin(), var_tensors[v].end());
    std::sort(tt.begin(), tt.end());
    tt.erase(std::unique(tt.begin(), tt.end()), tt.end());
    std::vector<int64_t>& base_max = c_base;
    base_max.resize(tt.size());
    for (size_t i = 0; i < tt.size(); ++i) base_max[i] = tmax(tt[i], n.fixed, n.x);
    for (int ci = (int)best.cubes.size() - 1; ci >= 0; --ci) {
      const Cube& c = best.cubes[ci];
      Node ch = take();
      ch.fixed = n.fixed;
      ch.x = n.x;
      std::vector<int32_t>& newly = c_newly;
      newly.clear();
      for (int j = 0; j < (int)best.region.size(); ++j)
        if (c.mask >> j & 1) {
          const int v = best.region[j];
          bit_set(ch.fixed, v);
          ch.x[v] = (uint8_t)((c.val >> j) & 1);
          newly.push_back(v);
        }
      // bound: only tensors holding a newly fixed variable change
      int64_t b = n.bound;
      for (size_t i = 0; i < tt.size() && b != INT64_MIN; ++i) {
        const BaseTensor& T = net.tensors[tt[i]];
        bool hit = false;
        for (int v : T.vars)
          if (std::find(newly.begin(), newly.end(), v) != newly.end()) { hit = true; break; }
        if (!hit) continue;
        const int64_t m = tmax(tt[i], ch.fixed, ch.x);
        b = (m == INT64_MIN) ? INT64_MIN : b + (m - base_max[i]);
      }
      ch.bound = b;
      if (ch.bound == INT64_MIN || ch.bound < opt.incumbent ||
          (opt.values_only && ch.bound == opt.incumbent)) {
        st.pruned++;
        spare.push_back(std::move(ch));
        continue;
      }
      // sizes are kept for nodes that branch again; a leaf (rho = 0) only
      // needs its fixed states
      const int64_t* d = best.drho_of(c.mask);
      if (d && n.rho - *d == 0) {
        ch.rho = 0;
        ch.sizes.clear();
      } else {
        ch.sizes = n.sizes;
        for (int v : newly)
          for (int id : tree.var_nodes[v]) ch.sizes[id]--;
        ch.rho = d ? n.rho - *d : rho_of(tree, ch.sizes, opt.log2_target);
      }
      out.push_back(std::move(ch));
    }
  }

  void emit(const Node& n, std::vector<LeafGroup>& leaves) {
    auto it = group_of.find(n.fixed);
    int gi;
    if (it == group_of.end()) {
      gi = (int)leaves.size();
      LeafGroup g;
      g.mask = n.fixed;
      for (int v = 0; v < net.n; ++v)
        if (bit_get(n.fixed, v)) g.vars.push_back(v);
      leaves.push_back(std::move(g));
      group_of[n.fixed] = gi;
    } else {
      gi = it->second;
    }
    LeafGroup& g = leaves[gi];
    for (int v : g.vars) g.assign.push_back(n.x[v]);
    g.count++;
  }

  // The node being expanded: fixed set, states and sizes are changed in
  // place on the way down and restored on the way up (a child differs from
  // its parent by the few variables of one cube).  Depth-first, children in
  // cube order: the same visiting order as an explicit stack with the first
  // cube on top.
  Node cur;
  std::vector<double> heur, score;

  // the branching rule of the current node (empty cubes: nothing to branch)
  Eval rule_of() {
    Eval best;
    // Nodes with the same fixed-variable set have the same rho structure.
    // When the rule chosen for an earlier such node pruned nothing, try it
    // first: if it again prunes nothing it is taken as is (the branches
    // are complete and disjoint either way; only the choice of rule is
    // shared).
    auto memo = rule_memo.find(cur.fixed);
    if (memo != rule_memo.end()) {
      Eval ev = evaluate(cur, memo->second);
      if (ev.cubes.size() == ((size_t)1 << memo->second.size())) best = std::move(ev);
    }
    if (best.cubes.empty()) {
      // overflow participation of every free variable
      std::vector<int32_t> cand;
      heuristic(cur, heur, cand);
      if (cand.empty()) throw Error(BBTN_E_INTERNAL, "rho > 0 but no overflowing variable");
      // seeds: the heuristic's two best candidates; with the learned
      // scorer, also its two best (the scorer ranks seeds only; regions
      // always grow in the heuristic's order, the order its training labels
      // were measured with).  The lowest gamma over all seeds wins, so the
      // scorer's picks add to the heuristic's and never displace them.
      std::stable_sort(cand.begin(), cand.end(), [&](int a, int b) {
        if (heur[a] != heur[b]) return heur[a] > heur[b];
        return a < b;
      });
      std::vector<int32_t> seeds;
      for (int si = 0; si < std::min<int>(2, (int)cand.size()); ++si) seeds.push_back(cand[si]);
      if (opt.scorer) {
        score = heur;
        opt.scorer(cur.fixed, cur.sizes, heur, score);
        std::vector<int32_t> by_score(cand);
        std::stable_sort(by_score.begin(), by_score.end(),
                         [&](int a, int b) { return score[a] > score[b]; });
        for (int si = 0; si < std::min<int>(2, (int)by_score.size()); ++si)
          if (std::find(seeds.begin(), seeds.end(), by_score[si]) == seeds.end())
            seeds.push_back(by_score[si]);
      }
      for (int sd : seeds) {
        Eval ev = best_from_seed(cur, sd, heur);
        if (better(ev, best)) best = std::move(ev);
        if (best.gamma == 0.0) break;  // every configuration pruned
      }
      if (!best.cubes.empty() && best.cubes.size() == ((size_t)1 << best.region.size()))
        rule_memo[cur.fixed] = best.region;
    }
    return best;
  }

  void visit(std::vector<LeafGroup>& leaves, SearchStats& st) {
    if (opt.deadline > 0 && now_s() > opt.deadline)
      throw Error(BBTN_E_TIMEOUT, "time limit reached during the search");
    if (opt.node_limit && st.nodes >= opt.node_limit->load(std::memory_order_relaxed))
      throw Error(BBTN_E_TIMEOUT, "node limit reached during the search");
    st.nodes++;
    if (cur.rho == 0 || opt.log2_target <= 0) {
      emit(cur, leaves);
      st.leaves++;
      return;
    }
    const Eval best = rule_of();
    if (best.cubes.empty()) { st.pruned++; return; }
    if (!std::isfinite(best.gamma)) throw Error(BBTN_E_INTERNAL, "no branching rule reduces rho");
    st.gamma_sum += best.gamma;
    // tensors touched by the region and their largest entries at the node
    std::vector<int32_t> tt;
    for (int v : best.region) tt.insert(tt.end(), var_tensors[v].begin(), var_tensors[v].end());
    std::sort(tt.begin(), tt.end());
    tt.erase(std::unique(tt.begin(), tt.end()), tt.end());
    std::vector<int64_t> base_max(tt.size());
    for (size_t i = 0; i < tt.size(); ++i) base_max[i] = tmax(tt[i], cur.fixed, cur.x);
    const int64_t rho0 = cur.rho, bound0 = cur.bound;
    std::vector<int32_t> newly;
    for (const Cube& c : best.cubes) {
      newly.clear();
      for (int j = 0; j < (int)best.region.size(); ++j)
        if (c.mask >> j & 1) {
          const int v = best.region[j];
          bit_set(cur.fixed, v);
          cur.x[v] = (uint8_t)((c.val >> j) & 1);
          newly.push_back(v);
        }
      // bound: only tensors holding a newly fixed variable change
      int64_t b = bound0;
      for (size_t i = 0; i < tt.size() && b != INT64_MIN; ++i) {
        const BaseTensor& T = net.tensors[tt[i]];
        bool hit = false;
        for (int v : T.vars)
          if (std::find(newly.begin(), newly.end(), v) != newly.end()) { hit = true; break; }
        if (!hit) continue;
        const int64_t m = tmax(tt[i], cur.fixed, cur.x);
        b = (m == INT64_MIN) ? INT64_MIN : b + (m - base_max[i]);
      }
      // the node keeps its tensor bound (later bounds update it in place);
      // an independent-set network may also be pruned by the clique bound
      int64_t bp = b;
      if (b != INT64_MIN && net.mis) bp = std::min(b, clique_bound(net, cur.fixed, cur.x));
      if (bp == INT64_MIN || bp < opt.incumbent || (opt.values_only && bp == opt.incumbent)) {
        st.pruned++;
      } else {
        // sizes follow the fixed set for a node that branches again; a leaf
        // (rho = 0) only needs its fixed states
        const int64_t* d = best.drho_of(c.mask);
        const bool leaf = d && rho0 - *d == 0;
        if (!leaf)
          for (int v : newly)
            for (int id : tree.var_nodes[v]) cur.sizes[id]--;
        cur.rho = leaf ? 0 : (d ? rho0 - *d : rho_of(tree, cur.sizes, opt.log2_target));
        cur.bound = b;
        visit(leaves, st);
        if (!leaf)
          for (int v : newly)
            for (int id : tree.var_nodes[v]) cur.sizes[id]++;
      }
      for (int v : newly) cur.fixed[v >> 6] &= ~(1ull << (v & 63));
    }
    cur.rho = rho0;
    cur.bound = bound0;
  }

  void run(std::vector<LeafGroup>& leaves, SearchStats& st) {
    cur.fixed.assign((net.n + 63) / 64, 0);
    cur.x.assign(net.n, 0);
    for (const auto& pv : opt.prefix) {
      BBTN_REQUIRE(pv.first >= 0 && pv.first < net.n, "prefixed variable out of range");
      bit_set(cur.fixed, pv.first);
      cur.x[pv.first] = pv.second & 1;
    }
    cur.sizes = node_sizes(tree, cur.fixed);
    cur.rho = rho_of(tree, cur.sizes, opt.log2_target);
    cur.bound = node_bound(net, cur.fixed, cur.x);
    int64_t bp = cur.bound;
    if (bp != INT64_MIN && net.mis) bp = std::min(bp, clique_bound(net, cur.fixed, cur.x));
    if (bp < opt.incumbent || bp == INT64_MIN || (opt.values_only && bp == opt.incumbent)) {
      st.pruned++;
      return;
    }
    heur.assign(net.n, 0);
    score.assign(net.n, 0);
    visit(leaves, st);
  }
};

}  // namespace

void collect_training(const Network& net, const Tree& tree, int log2_target, int region_max,
                      int64_t incumbent, int max_nodes, int cand_per_node,
                      std::vector<float>& X, std::vector<float>& y) {
  SearchOptions opt;
  opt.log2_target = log2_target;
  opt.region_max = region_max;
  opt.incumbent = incumbent;
  Searcher s(net, tree, opt);
  FeatureCtx fc(net, tree, log2_target);
  Node root;
  root.fixed.assign((net.n + 63) / 64, 0);
  root.x.assign(net.n, 0);
  root.sizes = node_sizes(tree, root.fixed);
  root.rho = rho_of(tree, root.sizes, log2_target);
  root.bound = node_bound(net, root.fixed, root.x);
  if (root.bound == INT64_MIN || root.bound < incumbent || root.rho == 0) return;
  std::vector<Node> stack;
  stack.push_back(std::move(root));
  std::vector<double> heur(net.n);
  std::vector<int32_t> cand;
  SearchStats st;
  uint64_t rng = 0x9E3779B97F4A7C15ull ^ (uint64_t)net.n;
  auto next = [&]() {
    rng ^= rng << 13; rng ^= rng >> 7; rng ^= rng << 17;
    return rng;
  };
  int done = 0;
  float f[N_FEAT];
  while (!stack.empty() && done < max_nodes) {
    Node n = std::move(stack.back());
    stack.pop_back();
    if (n.rho == 0) continue;
    s.heuristic(n, heur, cand);
    if (cand.empty()) continue;
    std::stable_sort(cand.begin(), cand.end(), [&](int a, int b) {
      if (heur[a] != heur[b]) return heur[a] > heur[b];
      return a < b;
    });
    // candidates: the best half by the heuristic and a random other half
    std::vector<int32_t> pick;
    for (int i = 0; i < (int)cand.size() && (int)pick.size() < cand_per_node / 2; ++i) pick.push_back(cand[i]);
    for (int tries = 0; tries < 4 * cand_per_node && (int)pick.size() < cand_per_node; ++tries) {
      const int v = cand[next() % cand.size()];
      if (std::find(pick.begin(), pick.end(), v) == pick.end()) pick.push_back(v);
    }
    Searcher::Eval chosen;
    const size_t row0 = y.size();
    for (int v : pick) {
      Searcher::Eval ev = s.best_from_seed(n, v, heur);
      // label: the branching factor (characteristic equation) of the best
      // rule the planner builds from this seed, in log2; it folds together
      // the problem-size reduction and the pruning of F(R).  A seed whose
      // rules reduce nothing gets the largest label seen at the node.
      const double lg = ev.gamma == 0.0 ? 0.0 : std::log2(std::max(1.0, ev.gamma));
      fc.features(v, n.fixed, n.sizes, heur, n.rho, f);
      X.insert(X.end(), f, f + N_FEAT);
      y.push_back(std::isfinite(lg) ? (float)lg : -1.f);
      if (v == cand[0] || (v == cand[std::min<size_t>(1, cand.size() - 1)] && Searcher::better(ev, chosen)))
        if (Searcher::better(ev, chosen)) chosen = std::move(ev);
    }
    // labels relative to the node's best candidate: the scorer only has to
    // rank the candidates of one node
    float lo = INFINITY, hi = 0.f;
    for (size_t i = row0; i < y.size(); ++i)
      if (y[i] >= 0) { lo = std::min(lo, y[i]); hi = std::max(hi, y[i]); }
    for (size_t i = row0; i < y.size(); ++i) y[i] = y[i] >= 0 ? y[i] - lo : hi - lo + 1.f;
    ++done;
    // continue the search with the heuristic's choice
    if (chosen.cubes.empty() || !std::isfinite(chosen.gamma)) continue;
    s.children(n, chosen, stack, st);
  }
}

void bb_search(const Network& net, const Tree& tree, const SearchOptions& opt,
               std::vector<LeafGroup>& leaves, SearchStats& stats) {
  Searcher s(net, tree, opt);
  s.run(leaves, stats);
}

// ------------------------------------------------------------ local search
std::vector<uint8_t> local_search_spinglass(int32_t n, int32_t m, const int32_t* uv,
                                            const int32_t* J, const int32_t* h, int sweeps,
                                            uint64_t seed) {
  // simulated annealing (single-spin Metropolis updates, geometric
  // temperature schedule), then zero-temperature sweeps; one restart per 100
  // sweeps.  Acceptance probabilities exp(-dE/T) for small dE are tabulated
  // per sweep as they are first needed.  Neighbours in compressed rows (edge
  // order), spins as bytes: a new best state is a 1-byte-per-spin copy.
  std::vector<int32_t> row(n + 1, 0), nb(2 * (size_t)m), wj(2 * (size_t)m);
  for (int e = 0; e < m; ++e) {
    row[uv[2 * e] + 1]++;
    row[uv[2 * e + 1] + 1]++;
  }
  for (int i = 0; i < n; ++i) row[i + 1] += row[i];
  {
    std::vector<int32_t> fill(row.begin(), row.end() - 1);
    for (int e = 0; e < m; ++e) {
      const int a = uv[2 * e], b = uv[2 * e + 1];
      nb[fill[a]] = b;
      wj[fill[a]++] = J[e];
      nb[fill[b]] = a;
      wj[fill[b]++] = J[e];
    }
  }
  std::mt19937_64 rng(seed);
  auto energy = [&](const std::vector<int8_t>& s) {
    int64_t E = 0;
    for (int e = 0; e < m; ++e) E -= (int64_t)J[e] * s[uv[2 * e]] * s[uv[2 * e + 1]];
    if (h) for (int i = 0; i < n; ++i) E -= (int64_t)h[i] * s[i];
    return E;
  };
  std::vector<int8_t> best_s(n, 1);
  int64_t bestE = energy(best_s);
  const int restarts = std::max(1, sweeps / 100);
  const int per = std::max(1, std::min(sweeps, 100));
  constexpr int TAB = 64;
  double acc[TAB];
  int acc_sweep[TAB];  // sweep whose temperature acc[d] was formed for
  std::vector<int8_t> s(n);
  for (int rs = 0; rs < restarts; ++rs) {
    for (int i = 0; i < n; ++i) s[i] = (rng() & 1) ? 1 : -1;
    int64_t E = energy(s);
    const double T0 = 2.0, T1 = 0.05;
    for (int sw = 0; sw < per + 10; ++sw) {
      const double T = sw < per ? T0 * std::pow(T1 / T0, (double)sw / std::max(1, per - 1)) : 0.0;
      const int tag = rs * (per + 10) + sw;
      if (tag == 0)
        for (int d = 0; d < TAB; ++d) acc_sweep[d] = -1;
      for (int i = 0; i < n; ++i) {
        // |J| + |h| sums are below 2^27, so local fields fit 32 bits
        int32_t f = h ? h[i] : 0;
        for (int q = row[i]; q < row[i + 1]; ++q) f += wj[q] * s[nb[q]];
        const int32_t dE = 2 * s[i] * f;
        bool flip = dE <= 0;
        if (!flip && T > 0) {
          // exp(-dE/T), formed the first time this sweep needs it
          if (dE < TAB && acc_sweep[dE] != tag) {
            acc[dE] = std::exp(-(double)dE / T);
            acc_sweep[dE] = tag;
          }
          const double p = dE < TAB ? acc[dE] : std::exp(-(double)dE / T);
          flip = (double)(rng() >> 11) * 0x1.0p-53 < p;
        }
        if (flip) {
          s[i] = (int8_t)-s[i];
          E += dE;
          if (E < bestE) {
            bestE = E;
            std::copy(s.begin(), s.end(), best_s.begin());
          }
        }
      }
    }
  }
  std::vector<uint8_t> x(n);
  for (int i = 0; i < n; ++i) x[i] = best_s[i] > 0 ? 1 : 0;
  return x;
}

// Iterated local search on an independent set (the swap moves and
// perturbations of Andrade, Resende and Werneck, 2012, in weighted form):
// insert free vertices (no neighbour in the set); replace a set vertex v by
// one or two non-adjacent neighbours whose only set neighbour is v when
// that adds weight; then perturb by forcing a random outside vertex in
// (dropping its set neighbours), re-optimise, and keep the result when it
// is no lighter.  x and W are updated to the best set found.
static void improve_independent_set(const std::vector<std::vector<int>>& adj,
                                    const int32_t* w, std::vector<uint8_t>& x, int64_t& W,
                                    int iterations, std::mt19937_64& rng) {
  const int n = (int)adj.size();
  if (n == 0) return;
  auto wt = [&](int v) -> int64_t { return w ? w[v] : 1; };
  std::vector<int> tau(n, 0);  // set neighbours of each vertex
  for (int v = 0; v < n; ++v)
    if (x[v])
      for (int u : adj[v]) tau[u]++;
  auto ins = [&](int v) {
    x[v] = 1;
    W += wt(v);
    for (int u : adj[v]) tau[u]++;
  };
  auto del = [&](int v) {
    x[v] = 0;
    W -= wt(v);
    for (int u : adj[v]) tau[u]--;
  };
  auto adjacent = [&](int a, int b) {
    const auto& A = adj[a].size() < adj[b].size() ? adj[a] : adj[b];
    const int o = adj[a].size() < adj[b].size() ? b : a;
    return std::find(A.begin(), A.end(), o) != A.end();
  };
  std::vector<int> cand;
  auto local_opt = [&]() {
    for (bool again = true; again;) {
      again = false;
      for (int v = 0; v < n; ++v)
        if (!x[v] && tau[v] == 0) ins(v);
      for (int v = 0; v < n; ++v) {
        if (!x[v]) continue;
        cand.clear();
        for (int u : adj[v])
          if (!x[u] && tau[u] == 1) cand.push_back(u);
        int b1 = -1, b2 = -1;
        int64_t gain = 0;
        for (size_t i = 0; i < cand.size(); ++i) {
          if (wt(cand[i]) - wt(v) > gain) { gain = wt(cand[i]) - wt(v); b1 = cand[i]; b2 = -1; }
          for (size_t j = i + 1; j < cand.size(); ++j)
            if (wt(cand[i]) + wt(cand[j]) - wt(v) > gain && !adjacent(cand[i], cand[j])) {
              gain = wt(cand[i]) + wt(cand[j]) - wt(v);
              b1 = cand[i];
              b2 = cand[j];
            }
        }
        if (b1 < 0) continue;
        del(v);
        ins(b1);
        if (b2 >= 0) ins(b2);
        again = true;
      }
    }
  };
  local_opt();
  std::vector<uint8_t> best = x;
  int64_t bestW = W;
  std::vector<uint8_t> keep;
  for (int it = 0; it < iterations; ++it) {
    keep = x;
    const int64_t W0 = W;
    int u = (int)(rng() % (uint64_t)n);
    for (int t = 0; t < n && x[u]; ++t) u = (u + 1) % n;
    if (x[u]) break;
    for (int nb : adj[u])
      if (x[nb]) del(nb);
    ins(u);
    local_opt();
    if (W < W0) {
      // restore the previous set and its neighbour counts
      for (int v = 0; v < n; ++v)
        if (x[v] != keep[v]) (keep[v] ? ins(v) : del(v));
    } else if (W > bestW) {
      bestW = W;
      best = x;
    }
  }
  x = best;
  W = bestW;
}

std::vector<uint8_t> local_search_mwis(int32_t n, int32_t m, const int32_t* uv,
                                       const int32_t* w, int restarts, uint64_t seed) {
  std::vector<std::vector<int>> adj(n);
  for (int e = 0; e < m; ++e) {
    adj[uv[2 * e]].push_back(uv[2 * e + 1]);
    adj[uv[2 * e + 1]].push_back(uv[2 * e]);
  }
  std::mt19937_64 rng(seed);
  std::vector<uint8_t> best(n, 0);
  int64_t bestW = -1;
  for (int rs = 0; rs < std::max(1, restarts); ++rs) {
    std::vector<double> key(n);
    for (int i = 0; i < n; ++i) {
      const double wi = w ? w[i] : 1;
      key[i] = wi / (double)(adj[i].size() + 1) + 1e-6 * (double)(rng() % 1000000) / 1e6 * (rs > 0);
    }
    std::vector<int> ord(n);
    for (int i = 0; i < n; ++i) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return key[a] > key[b]; });
    std::vector<uint8_t> x(n, 0), blocked(n, 0);
    int64_t W = 0;
    for (int i : ord) {
      if (blocked[i]) continue;
      x[i] = 1;
      W += w ? w[i] : 1;
      for (int j : adj[i]) blocked[j] = 1;
    }
    improve_independent_set(adj, w, x, W, 200, rng);
    if (W > bestW) { bestW = W; best = x; }
  }
  return best;
}

namespace {
constexpr double kNodeMacs = 131072.0;  // host time of a search node, in device MACs
// device time of moving one tensor entry (all its residue words) through
// HBM, in multiply-accumulates of the counting product: about 3.3e12 MACs
// against 1.75e11 entries of 20 bytes per second
constexpr double kKappa = 16.0;

// Candidate trees: the greedy tree, its n annealed refinements (seeds 1..n,
// overflow weight 0.25, multiply-accumulates alone), the min-fill tree and
// one refinement of that.  With `varied`, n more refinements of the greedy
// tree (seeds 1..n again) vary the annealer's objective: the overflow
// weight alternates between 0.25 and 0.1 (a lighter one trades more
// overflow, hence more leaves, for fewer multiply-accumulates) and the
// memory weight kappa cycles through 0, 4 and 6.  Their leaves cost less or
// more depending on the structure and on where the optimum lies, which a
// probe does not see, so they are offered only to a choice by measurement.
std::vector<Tree> order_candidates(const Network& net, int n, const SearchOptions& probe,
                                   bool varied) {
  const int nc = n + 3 + (varied ? n : 0);
  std::vector<Tree> cand(nc);
  cand[0] = greedy_tree(net);  // built before any thread reads it
  cand[n + 1] = minfill_tree(net);
  std::vector<std::thread> th;
  for (int c = 1; c < nc; ++c) {
    if (c == n + 1) continue;
    th.emplace_back([&, c] {
      RefineOptions o;
      o.sweeps = 200;
      o.log2_target = probe.log2_target;
      o.rho_weight = 0.25;
      o.deadline = probe.deadline;
      if (c <= n + 2) {
        o.seed = (uint64_t)c;
        cand[c] = refine_tree(net, c <= n ? cand[0] : cand[n + 1], o);
      } else {
        const int j = c - (n + 2);  // 1..n
        static const double kappas[3] = {0.0, 4.0, 6.0};
        o.rho_weight = j % 2 == 0 ? 0.1 : 0.25;
        o.kappa = kappas[(j / 2) % 3];
        o.seed = (uint64_t)j;
        cand[c] = refine_tree(net, cand[0], o);
      }
    });
  }
  for (auto& t : th) t.join();
  return cand;
}

// Probe score of a candidate: the cost model of its leaves (time_cost with
// kKappa, shared contractions once per group) plus kNodeMacs per search
// node; HUGE_VAL when the search passes `limit` nodes.
double probe_score(const Network& net, const Tree& t, const SearchOptions& probe,
                   std::atomic<uint64_t>* limit) {
  SearchOptions so = probe;
  so.node_limit = limit;
  std::vector<LeafGroup> groups;
  SearchStats st;
  try {
    bb_search(net, t, so, groups, st);
  } catch (const std::exception&) {
    return HUGE_VAL;  // over the budget (or cannot be planned)
  }
  double cost = 0;
  for (const auto& g : groups) {
    const TimeCost tc = time_cost(t, g.mask, kKappa);
    cost += (double)g.count * tc.branch + tc.shared;
  }
  return cost + kNodeMacs * (double)st.nodes;
}
}  // namespace

// The candidates are scored by a branch-and-bound search of `net` with
// `probe` (probe_score).  Probes run in parallel in rounds of growing node
// budgets, 2^10, 2^12, ... 2^22: a round re-runs every unfinished probe from
// the start with the round's budget, and the first round in which some probe
// finishes decides.  Every probe's outcome in a round depends on its budget
// only, so the choice is the same on every run.  Within a round a finished
// probe with score S stops the others past S / kNodeMacs nodes: they score
// worse than S, and could not have been chosen.  On zero-field +-J lattices
// the leaves depend on the structure only, so one instance's probe serves
// every instance of that structure.
Tree choose_order(const Network& net, int n, const SearchOptions& probe, bool* complete) {
  if (complete) *complete = true;
  if (n < 0) return minfill_tree(net);
  n = std::min(64, n);
  if (n == 0) return greedy_tree(net);
  std::vector<Tree> cand = order_candidates(net, n, probe, false);
  const int nc = (int)cand.size();
  std::vector<double> score(nc, HUGE_VAL);
  auto late = [&] { return probe.deadline > 0 && now_s() > probe.deadline; };
  for (int lb = 10; lb <= 22 && !late(); lb += 2) {
    std::atomic<uint64_t> limit{uint64_t(1) << lb};
    std::vector<std::thread> th;
    for (int c = 0; c < nc; ++c)
      th.emplace_back([&, c] {
        score[c] = probe_score(net, cand[c], probe, &limit);
        if (score[c] == HUGE_VAL) return;
        const uint64_t mine = (uint64_t)std::min(std::floor(score[c] / kNodeMacs) + 1, 1e18);
        uint64_t cur = limit.load();
        while (mine < cur && !limit.compare_exchange_weak(cur, mine)) {
        }
      });
    for (auto& t : th) t.join();
    if (late()) break;
    int best = -1;
    for (int c = 0; c < nc; ++c)
      if (score[c] < HUGE_VAL && (best < 0 || score[c] < score[best])) best = c;
    if (best >= 0) return std::move(cand[best]);
  }
  // no probe finished within 2^22 nodes, or the deadline came first
  if (complete) *complete = !late();
  return std::move(cand[0]);
}

std::vector<Tree> rank_orders(const Network& net, int n, const SearchOptions& probe) {
  n = std::max(1, std::min(64, n));
  std::vector<Tree> cand = order_candidates(net, n, probe, true);
  const int nc = (int)cand.size();
  std::vector<double> score(nc, HUGE_VAL);
  {
    std::vector<std::thread> th;
    for (int c = 0; c < nc; ++c)
      th.emplace_back([&, c] {
        std::atomic<uint64_t> limit{uint64_t(1) << 22};
        score[c] = probe_score(net, cand[c], probe, &limit);
      });
    for (auto& t : th) t.join();
  }
  std::vector<int> idx;
  for (int c = 0; c < nc; ++c)
    if (score[c] < HUGE_VAL) idx.push_back(c);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return score[a] < score[b]; });
  std::vector<Tree> out;
  for (int c : idx) out.push_back(std::move(cand[c]));
  return out;
}

}  // namespace bbtn
