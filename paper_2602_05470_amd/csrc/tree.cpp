#include "tree.h"

#include <chrono>
#include <cmath>
#include <queue>
#include <random>
#include <set>
#include <tuple>

namespace bbtn {

namespace {
struct Cand {
  int64_t cost;
  int32_t a, b;
  bool operator>(const Cand& o) const {
    return std::tie(cost, a, b) > std::tie(o.cost, o.a, o.b);
  }
};
int64_t sz(size_t r) { return r >= 62 ? (1ll << 62) : (1ll << r); }

// Depth-first post-order and the variable -> node index of a finished tree.
void finish_tree(Tree& t, int32_t n_vars) {
  t.dfs_post.clear();
  if (t.root >= 0) {
    std::vector<std::pair<int32_t, int>> st{{t.root, 0}};
    while (!st.empty()) {
      auto& top = st.back();
      const TNode& nd = t.nodes[top.first];
      if (nd.left < 0) { st.pop_back(); continue; }  // base tensor
      if (top.second == 0) { top.second = 1; st.push_back({nd.left, 0}); }
      else if (top.second == 1) { top.second = 2; st.push_back({nd.right, 0}); }
      else { t.dfs_post.push_back(top.first); st.pop_back(); }
    }
  }
  t.var_nodes.assign(n_vars, {});
  for (int id : t.postorder)
    for (int v : t.nodes[id].vars) t.var_nodes[v].push_back(id);
}
}  // namespace

Tree greedy_tree(const Network& net) {
  Tree t;
  const int T = (int)net.tensors.size();
  t.n_base = T;
  t.nodes.resize(T);
  std::vector<std::vector<int32_t>> hold(net.n);  // live holders per var
  for (int i = 0; i < T; ++i) {
    t.nodes[i].base = i;
    t.nodes[i].vars = net.tensors[i].vars;
    for (int v : t.nodes[i].vars) hold[v].push_back(i);
  }
  std::vector<char> live(T, 1);
  auto out_vars = [&](int a, int b) {
    std::vector<int32_t> u;
    const auto& A = t.nodes[a].vars;
    const auto& B = t.nodes[b].vars;
    std::set_union(A.begin(), A.end(), B.begin(), B.end(), std::back_inserter(u));
    std::vector<int32_t> o;
    for (int v : u) {
      bool elsewhere = false;
      for (int h : hold[v])
        if (h != a && h != b) { elsewhere = true; break; }
      if (elsewhere) o.push_back(v);
    }
    return o;
  };
  std::priority_queue<Cand, std::vector<Cand>, std::greater<Cand>> pq;
  auto push_pair = [&](int a, int b) {
    if (a > b) std::swap(a, b);
    const auto o = out_vars(a, b);
    const int64_t c = sz(o.size()) - sz(t.nodes[a].vars.size()) - sz(t.nodes[b].vars.size());
    pq.push(Cand{c, a, b});
  };
  for (int v = 0; v < net.n; ++v)
    for (size_t i = 0; i < hold[v].size(); ++i)
      for (size_t j = i + 1; j < hold[v].size(); ++j) push_pair(hold[v][i], hold[v][j]);
  auto merge = [&](int a, int b) {
    TNode n;
    n.left = a;
    n.right = b;
    n.vars = out_vars(a, b);
    const int id = (int)t.nodes.size();
    t.nodes[a].parent = id;
    t.nodes[b].parent = id;
    // update holders
    std::vector<int32_t> u;
    const auto& A = t.nodes[a].vars;
    const auto& B = t.nodes[b].vars;
    std::set_union(A.begin(), A.end(), B.begin(), B.end(), std::back_inserter(u));
    for (int v : u) {
      auto& h = hold[v];
      h.erase(std::remove_if(h.begin(), h.end(), [&](int x) { return x == a || x == b; }), h.end());
    }
    for (int v : n.vars) hold[v].push_back(id);
    t.nodes.push_back(std::move(n));
    live.push_back(1);
    live[a] = live[b] = 0;
    t.postorder.push_back(id);
    return id;
  };
  while (!pq.empty()) {
    const Cand c = pq.top();
    pq.pop();
    if (!live[c.a] || !live[c.b]) continue;
    const int id = merge(c.a, c.b);
    std::vector<int32_t> nb;
    for (int v : t.nodes[id].vars)
      for (int h : hold[v])
        if (h != id) nb.push_back(h);
    std::sort(nb.begin(), nb.end());
    nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
    for (int x : nb) push_pair(id, x);
  }
  // join what is left (scalars of disconnected components, in id order)
  std::vector<int> rest;
  for (int i = 0; i < (int)t.nodes.size(); ++i)
    if (live[i]) rest.push_back(i);
  if (rest.empty()) {
    t.root = -1;
  } else {
    int acc = rest[0];
    for (size_t i = 1; i < rest.size(); ++i) acc = merge(acc, rest[i]);
    t.root = acc;
  }
  finish_tree(t, net.n);
  return t;
}


// Min-fill elimination order turned into a pairwise tree.  The interaction
// graph joins variables that share a tensor; each step eliminates the
// variable whose elimination adds the fewest edges among its neighbours
// (fewest neighbours, then lowest id, on ties), and the tree contracts the
// tensors holding it, two at a time, smallest result first, so that the
// variable is summed out as soon as its last holder is formed.  On planar
// grids this follows the separators of the lattice, where the greedy pair
// order (smallest size increase first) can leave a much wider frontier.
Tree minfill_tree(const Network& net) {
  Tree t;
  const int T = (int)net.tensors.size();
  const int n = net.n;
  t.n_base = T;
  t.nodes.resize(T);
  std::vector<std::vector<int32_t>> hold(n);
  std::vector<std::set<int32_t>> g(n);
  for (int i = 0; i < T; ++i) {
    t.nodes[i].base = i;
    t.nodes[i].vars = net.tensors[i].vars;
    const auto& vs = t.nodes[i].vars;
    for (int v : vs) hold[v].push_back(i);
    for (size_t a = 0; a < vs.size(); ++a)
      for (size_t b = a + 1; b < vs.size(); ++b) {
        g[vs[a]].insert(vs[b]);
        g[vs[b]].insert(vs[a]);
      }
  }
  std::vector<char> live(T, 1);
  auto out_vars = [&](int a, int b) {
    std::vector<int32_t> u;
    const auto& A = t.nodes[a].vars;
    const auto& B = t.nodes[b].vars;
    std::set_union(A.begin(), A.end(), B.begin(), B.end(), std::back_inserter(u));
    std::vector<int32_t> o;
    for (int v : u) {
      bool elsewhere = false;
      for (int h : hold[v])
        if (h != a && h != b) { elsewhere = true; break; }
      if (elsewhere) o.push_back(v);
    }
    return o;
  };
  auto merge = [&](int a, int b) {
    TNode nd;
    nd.left = a;
    nd.right = b;
    nd.vars = out_vars(a, b);
    const int id = (int)t.nodes.size();
    t.nodes[a].parent = id;
    t.nodes[b].parent = id;
    std::vector<int32_t> u;
    std::set_union(t.nodes[a].vars.begin(), t.nodes[a].vars.end(), t.nodes[b].vars.begin(),
                   t.nodes[b].vars.end(), std::back_inserter(u));
    for (int v : u) {
      auto& h = hold[v];
      h.erase(std::remove_if(h.begin(), h.end(), [&](int x) { return x == a || x == b; }), h.end());
    }
    for (int v : nd.vars) hold[v].push_back(id);
    t.nodes.push_back(std::move(nd));
    live.push_back(1);
    live[a] = live[b] = 0;
    t.postorder.push_back(id);
    return id;
  };
  auto fill_of = [&](int v) {
    int64_t f = 0;
    for (auto i = g[v].begin(); i != g[v].end(); ++i) {
      auto j = i;
      for (++j; j != g[v].end(); ++j) f += !g[*i].count(*j);
    }
    return f;
  };
  // keys (fill, degree, id) of the remaining variables, updated for the
  // neighbourhood of each eliminated variable
  using Key = std::tuple<int64_t, int64_t, int32_t>;
  std::set<Key> order;
  std::vector<Key> key(n);
  for (int v = 0; v < n; ++v) {
    key[v] = Key{fill_of(v), (int64_t)g[v].size(), v};
    order.insert(key[v]);
  }
  std::vector<char> gone(n, 0);
  while (!order.empty()) {
    const int v = std::get<2>(*order.begin());
    order.erase(order.begin());
    gone[v] = 1;
    // contract the tensors holding v, smallest result first
    while (hold[v].size() > 1) {
      int ba = -1, bb = -1;
      size_t bs = 0;
      for (size_t i = 0; i < hold[v].size(); ++i)
        for (size_t j = i + 1; j < hold[v].size(); ++j) {
          const size_t o = out_vars(hold[v][i], hold[v][j]).size();
          if (ba < 0 || o < bs) { ba = hold[v][i]; bb = hold[v][j]; bs = o; }
        }
      merge(std::min(ba, bb), std::max(ba, bb));
    }
    for (int a : g[v])
      for (int b : g[v])
        if (a != b) g[a].insert(b);
    for (int a : g[v]) g[a].erase(v);
    std::set<int32_t> touched;
    for (int a : g[v]) {
      touched.insert(a);
      for (int b : g[a]) touched.insert(b);
    }
    g[v].clear();
    for (int u : touched) {
      if (gone[u]) continue;
      order.erase(key[u]);
      key[u] = Key{fill_of(u), (int64_t)g[u].size(), u};
      order.insert(key[u]);
    }
  }
  std::vector<int> rest;
  for (int i = 0; i < (int)t.nodes.size(); ++i)
    if (live[i]) rest.push_back(i);
  if (rest.empty()) {
    t.root = -1;
  } else {
    int acc = rest[0];
    for (size_t i = 1; i < rest.size(); ++i) acc = merge(acc, rest[i]);
    t.root = acc;
  }
  finish_tree(t, n);
  return t;
}

// Annealed local rotations of a contraction tree.  A rotation at internal
// node n with children (L, R), L = (A, B), turns n into ((A, R), B) or
// ((B, R), A) (and symmetrically through R); only the new inner node's
// variables change: they are the variables of its two children that are
// still held outside it, i.e. by the third subtree or by n's own output.
Tree refine_tree(const Network& net, const Tree& in, const RefineOptions& o) {
  Tree t = in;
  const int N = (int)t.nodes.size();
  if (t.root < 0 || o.sweeps <= 0 || N - t.n_base < 2) return t;
  Complexity c0 = complexity(in, {});
  const int sc_cap = o.sc_target > 0 ? o.sc_target : c0.sc;
  const int lt = o.log2_target;
  std::mt19937_64 rng(o.seed);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  using V = std::vector<int32_t>;
  auto uni = [](const V& a, const V& b, V& out) {
    out.clear();
    std::set_union(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(out));
  };
  auto inter = [](const V& a, const V& b, V& out) {
    out.clear();
    std::set_intersection(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(out));
  };
  // space term of a node of rank r: over the cap, and over T_target (rho)
  auto space = [&](int r) {
    return o.sc_weight * std::max(0, r - sc_cap) + o.rho_weight * std::max(0, r - lt);
  };
  V u1, u2, u3, nv;
  std::vector<int32_t> internal;
  for (int id = t.n_base; id < N; ++id) internal.push_back(id);
  for (int sw = 0; sw < o.sweeps; ++sw) {
    if (o.deadline > 0 &&
        std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
                .count() > o.deadline)
      break;
    const double beta = o.beta0 + (o.beta1 - o.beta0) * sw / std::max(1, o.sweeps - 1);
    std::shuffle(internal.begin(), internal.end(), rng);
    for (int n : internal) {
      TNode& nd = t.nodes[n];
      // pick a child to rotate through, and which of its children stays
      const int side = (int)(rng() & 1), keep = (int)((rng() >> 1) & 1);
      const int c = side ? nd.right : nd.left;   // inner child (L)
      const int r = side ? nd.left : nd.right;   // sibling moving in (R)
      if (t.nodes[c].left < 0) continue;         // base tensor: no rotation
      const int a = keep ? t.nodes[c].right : t.nodes[c].left;   // joins R
      const int b = keep ? t.nodes[c].left : t.nodes[c].right;   // moves up
      const V& va = t.nodes[a].vars;
      const V& vb = t.nodes[b].vars;
      const V& vr = t.nodes[r].vars;
      const V& vc = t.nodes[c].vars;
      // old: c = (a, b) of cost |va u vb|, n = (c, r) of cost |vc u vr|
      uni(va, vb, u1);
      const int old_c = (int)u1.size();
      uni(vc, vr, u1);
      const int old_n = (int)u1.size();
      // new: c' = (a, r) with vars (va u vr) n (vb u vn), n = (c', b)
      uni(va, vr, u2);
      uni(vb, nd.vars, u3);
      inter(u2, u3, nv);
      const int new_c = (int)u2.size();
      uni(nv, vb, u1);
      const int new_n = (int)u1.size();
      // entries moved by the two contractions (the parts that change)
      const double ka = o.kappa;
      const double ea = std::ldexp(1.0, (int)va.size()), eb = std::ldexp(1.0, (int)vb.size());
      const double er = std::ldexp(1.0, (int)vr.size());
      const double mem_old = ka * (3 * ea + 3 * eb + 4 * std::ldexp(1.0, (int)vc.size()) + 3 * er);
      const double mem_new = ka * (3 * ea + 3 * er + 4 * std::ldexp(1.0, (int)nv.size()) + 3 * eb);
      const double lo = std::log2(std::ldexp(1.0, old_c) + std::ldexp(1.0, old_n) + mem_old);
      const double ln = std::log2(std::ldexp(1.0, new_c) + std::ldexp(1.0, new_n) + mem_new);
      const double d = ln - lo + space((int)nv.size()) - space((int)vc.size());
      if (d > 0 && U(rng) >= std::exp(-beta * d)) continue;
      // apply: c keeps its id and becomes (a, r); n becomes (c, b)
      TNode& cn = t.nodes[c];
      cn.left = a;
      cn.right = r;
      cn.vars = nv;
      t.nodes[a].parent = c;
      t.nodes[r].parent = c;
      if (side) { nd.right = c; nd.left = b; } else { nd.left = c; nd.right = b; }
      t.nodes[b].parent = n;
    }
  }
  // renumber internal nodes in depth-first post-order (children first)
  Tree out;
  out.n_base = t.n_base;
  out.nodes.assign(t.nodes.begin(), t.nodes.begin() + t.n_base);
  std::vector<int32_t> id_of(N, -1);
  for (int i = 0; i < t.n_base; ++i) id_of[i] = i;
  std::vector<std::pair<int32_t, int>> st{{t.root, 0}};
  while (!st.empty()) {
    auto& top = st.back();
    const TNode& nd = t.nodes[top.first];
    if (nd.left < 0) { st.pop_back(); continue; }
    if (top.second == 0) { top.second = 1; st.push_back({nd.left, 0}); }
    else if (top.second == 1) { top.second = 2; st.push_back({nd.right, 0}); }
    else {
      TNode m;
      m.left = id_of[nd.left];
      m.right = id_of[nd.right];
      m.vars = nd.vars;
      const int id = (int)out.nodes.size();
      id_of[top.first] = id;
      out.nodes[m.left].parent = id;
      out.nodes[m.right].parent = id;
      out.nodes.push_back(std::move(m));
      out.postorder.push_back(id);
      st.pop_back();
    }
  }
  out.root = id_of[t.root];
  out.nodes[out.root].parent = -1;
  // check every node's variables against a recount: a variable stays open
  // while some base tensor outside the subtree still holds it
  std::vector<int32_t> total(net.n, 0);
  for (int i = 0; i < out.n_base; ++i)
    for (int v : out.nodes[i].vars) ++total[v];
  std::vector<std::vector<std::pair<int32_t, int32_t>>> held(out.nodes.size());
  for (int i = 0; i < out.n_base; ++i)
    for (int v : out.nodes[i].vars) held[i].push_back({v, 1});
  for (int id : out.postorder) {
    const auto& A = held[out.nodes[id].left];
    const auto& B = held[out.nodes[id].right];
    auto& H = held[id];
    size_t i = 0, j = 0;
    while (i < A.size() || j < B.size()) {
      std::pair<int32_t, int32_t> e;
      if (j == B.size() || (i < A.size() && A[i].first < B[j].first)) e = A[i++];
      else if (i == A.size() || B[j].first < A[i].first) e = B[j++];
      else { e = {A[i].first, A[i].second + B[j].second}; ++i; ++j; }
      if (e.second < total[e.first]) H.push_back(e);
    }
    std::vector<int32_t> open;
    for (const auto& e : H) open.push_back(e.first);
    if (open != out.nodes[id].vars) throw Error(BBTN_E_INTERNAL, "refined tree: inconsistent variables");
    held[out.nodes[id].left].clear();
    held[out.nodes[id].right].clear();
  }
  finish_tree(out, net.n);
  return out;
}

Complexity complexity(const Tree& t, const std::vector<uint64_t>& fixed) {
  Complexity c;
  double tc = 0;
  for (int id : t.postorder) {
    const TNode& n = t.nodes[id];
    auto free_count = [&](const std::vector<int32_t>& vs) {
      int k = 0;
      for (int v : vs) k += !bit_get(fixed, v);
      return k;
    };
    const int ro = free_count(n.vars);
    std::vector<int32_t> u;
    const auto& A = t.nodes[n.left].vars;
    const auto& B = t.nodes[n.right].vars;
    std::set_union(A.begin(), A.end(), B.begin(), B.end(), std::back_inserter(u));
    const int ru = free_count(u);
    tc += std::ldexp(1.0, ru);  // one multiply-accumulate per joint index
    c.sc = std::max(c.sc, ro);
  }
  c.tc_log2 = tc > 0 ? std::log2(tc) : 0;
  return c;
}

TimeCost time_cost(const Tree& t, const std::vector<uint64_t>& fixed, double kappa) {
  TimeCost c;
  const int N = (int)t.nodes.size();
  std::vector<char> hasfix(N, 0);
  std::vector<int> free_n(N, 0);
  for (int i = 0; i < N; ++i) {
    int f = 0;
    for (int v : t.nodes[i].vars) {
      const bool fx = bit_get(fixed, v);
      f += !fx;
      if (i < t.n_base && fx) hasfix[i] = 1;
    }
    free_n[i] = f;
  }
  std::vector<int32_t> u;
  for (int id : t.postorder) {
    const TNode& n = t.nodes[id];
    hasfix[id] = hasfix[n.left] | hasfix[n.right];
    const auto& A = t.nodes[n.left].vars;
    const auto& B = t.nodes[n.right].vars;
    u.clear();
    std::set_union(A.begin(), A.end(), B.begin(), B.end(), std::back_inserter(u));
    int ru = 0;
    for (int v : u) ru += !bit_get(fixed, v);
    const double cost = std::ldexp(1.0, ru) +
                        kappa * (3 * std::ldexp(1.0, free_n[n.left]) +
                                 3 * std::ldexp(1.0, free_n[n.right]) + std::ldexp(1.0, free_n[id]));
    (hasfix[id] ? c.branch : c.shared) += cost;
  }
  return c;
}

}  // namespace bbtn
