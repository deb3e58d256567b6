#include "tree.h"

#include <cmath>
#include <queue>
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
  // depth-first post-order from the root (iterative)
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
  t.var_nodes.assign(net.n, {});
  for (int id : t.postorder)
    for (int v : t.nodes[id].vars) t.var_nodes[v].push_back(id);
  return t;
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

}  // namespace bbtn
