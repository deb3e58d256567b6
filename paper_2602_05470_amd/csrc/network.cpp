#include "network.h"

#include <map>
#include <set>

namespace bbtn {

static bool is_prime32(uint64_t n) {
  if (n < 2) return false;
  for (uint64_t p : {2ull, 3ull, 5ull, 7ull, 11ull, 13ull})
    if (n % p == 0) return n == p;
  uint64_t d = n - 1;
  int s = 0;
  while ((d & 1) == 0) { d >>= 1; ++s; }
  auto powm = [&](uint64_t a, uint64_t e) {
    uint64_t r = 1;
    a %= n;
    while (e) {
      if (e & 1) r = r * a % n;
      a = a * a % n;
      e >>= 1;
    }
    return r;
  };
  // deterministic for n < 2^32 with bases 2, 7, 61
  for (uint64_t a : {2ull, 7ull, 61ull}) {
    if (a % n == 0) continue;
    uint64_t x = powm(a, d);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int i = 1; i < s; ++i) {
      x = x * x % n;
      if (x == n - 1) { comp = false; break; }
    }
    if (comp) return false;
  }
  return true;
}

const std::vector<uint32_t>& prime_table() {
  static const std::vector<uint32_t> table = [] {
    std::vector<uint32_t> t;
    for (uint64_t c = (1ull << 31) - 1; t.size() < (size_t)NP; --c)
      if (is_prime32(c)) t.push_back((uint32_t)c);
    return t;
  }();
  return table;
}

static BaseTensor make_tensor(std::vector<int32_t> vars) {
  BaseTensor t;
  t.vars = std::move(vars);
  const int64_t sz = 1ll << t.vars.size();
  t.val.assign(sz, 0);
  t.res.assign((size_t)NP * sz, 1u);
  return t;
}

static void set_infeasible(BaseTensor& t, int64_t e) {
  t.val[e] = NEG;
  for (int p = 0; p < NP; ++p) t.res[(size_t)p * t.size() + e] = 0;
}

Network build_spinglass(int32_t n, int32_t m, const int32_t* uv, const int32_t* J,
                        const int32_t* h) {
  Network net;
  net.n = n;
  net.spin = true;
  std::map<std::pair<int, int>, int64_t> coup;
  for (int32_t e = 0; e < m; ++e) {
    int a = uv[2 * e], b = uv[2 * e + 1];
    BBTN_REQUIRE(a >= 0 && a < n && b >= 0 && b < n, "vertex id out of range");
    BBTN_REQUIRE(a != b, "self-loop");
    if (a > b) std::swap(a, b);
    coup[{a, b}] += J[e];
    net.abs_sum += std::llabs((long long)J[e]);
    BBTN_REQUIRE(net.abs_sum < (1ll << 27), "sum |J| + |h| must be < 2^27");
  }
  std::vector<int> deg(n, 0);
  for (auto& kv : coup) {
    // B^ij = [[-J, J], [J, -J]] as energies; max form stores -energy:
    // +J when the two spins agree, -J otherwise.  Bit 0 = s_i, bit 1 = s_j.
    const int64_t Jij = kv.second;
    BaseTensor t = make_tensor({kv.first.first, kv.first.second});
    t.val[0] = (int32_t)Jij;
    t.val[1] = (int32_t)-Jij;
    t.val[2] = (int32_t)-Jij;
    t.val[3] = (int32_t)Jij;
    net.tensors.push_back(std::move(t));
    deg[kv.first.first]++;
    deg[kv.first.second]++;
  }
  for (int i = 0; i < n; ++i) {
    const int64_t hi = h ? h[i] : 0;
    net.abs_sum += std::llabs((long long)hi);
    BBTN_REQUIRE(net.abs_sum < (1ll << 27), "sum |J| + |h| must be < 2^27");
    if (hi != 0 || deg[i] == 0) {
      // w^i = (h, -h) as energies; -energy: s=0 (sigma=-1) -> -h, s=1 -> +h
      BaseTensor t = make_tensor({i});
      t.val[0] = (int32_t)-hi;
      t.val[1] = (int32_t)hi;
      net.tensors.push_back(std::move(t));
    }
  }
  for (int p = 0; p < NP; ++p) net.const_res[p] = 1;
  net.zero_field = true;
  for (int i = 0; h && i < n; ++i) net.zero_field &= h[i] == 0;
  simplify(net);
  flatten(net);
  return net;
}

Network build_mwis(int32_t n, int32_t m, const int32_t* uv, const int32_t* w) {
  Network net;
  net.n = n;
  net.spin = false;
  std::set<std::pair<int, int>> es;
  for (int32_t e = 0; e < m; ++e) {
    int a = uv[2 * e], b = uv[2 * e + 1];
    BBTN_REQUIRE(a >= 0 && a < n && b >= 0 && b < n, "vertex id out of range");
    BBTN_REQUIRE(a != b, "self-loop");
    if (a > b) std::swap(a, b);
    es.insert({a, b});
  }
  for (auto& e : es) {
    // independence constraint: state (1,1) is the tropical zero
    BaseTensor t = make_tensor({e.first, e.second});
    set_infeasible(t, 3);
    net.tensors.push_back(std::move(t));
  }
  for (int i = 0; i < n; ++i) {
    const int64_t wi = w ? w[i] : 1;
    BBTN_REQUIRE(wi > 0, "weights must be positive");
    net.abs_sum += wi;
    BBTN_REQUIRE(net.abs_sum < (1ll << 27), "sum of weights must be < 2^27");
    // vertex tensor (0, -w_i) as energies; max form (0, +w_i)
    BaseTensor t = make_tensor({i});
    t.val[1] = (int32_t)wi;
    net.tensors.push_back(std::move(t));
  }
  for (int p = 0; p < NP; ++p) net.const_res[p] = 1;
  // clique partition: each vertex in id order, with every later unassigned
  // neighbour adjacent to all members taken so far
  auto g = std::make_shared<MisGraph>();
  g->adj.assign(n, {});
  for (auto& e : es) {
    g->adj[e.first].push_back(e.second);
    g->adj[e.second].push_back(e.first);
  }
  for (auto& a : g->adj) std::sort(a.begin(), a.end());
  g->w.resize(n);
  for (int i = 0; i < n; ++i) g->w[i] = w ? w[i] : 1;
  std::vector<char> taken(n, 0);
  for (int v = 0; v < n; ++v) {
    if (taken[v]) continue;
    std::vector<int32_t> q{v};
    taken[v] = 1;
    for (int u : g->adj[v]) {
      if (taken[u]) continue;
      bool all = true;
      for (int x : q)
        if (x != v && !std::binary_search(g->adj[u].begin(), g->adj[u].end(), x)) { all = false; break; }
      if (all) { q.push_back(u); taken[u] = 1; }
    }
    g->cliques.push_back(std::move(q));
  }
  net.mis = std::move(g);
  simplify(net);
  flatten(net);
  return net;
}

// Tropical product of `small` into `big` (small.vars a subset of big.vars).
static void absorb(BaseTensor& big, const BaseTensor& small) {
  std::vector<int> pos;
  for (int v : small.vars) {
    auto it = std::find(big.vars.begin(), big.vars.end(), v);
    pos.push_back((int)(it - big.vars.begin()));
  }
  const auto& P = prime_table();
  for (int64_t e = 0; e < big.size(); ++e) {
    int64_t se = 0;
    for (size_t j = 0; j < pos.size(); ++j) se |= ((e >> pos[j]) & 1) << j;
    if (big.val[e] <= NEG_CUT) continue;
    if (small.val[se] <= NEG_CUT) { set_infeasible(big, e); continue; }
    big.val[e] += small.val[se];
    for (int p = 0; p < NP; ++p) {
      uint32_t& r = big.res[(size_t)p * big.size() + e];
      r = mulmod(r, small.res[(size_t)p * small.size() + se], P[p]);
    }
  }
}

// Tropical sum over variable position j.
static BaseTensor sum_out(const BaseTensor& t, int j) {
  std::vector<int32_t> nv = t.vars;
  nv.erase(nv.begin() + j);
  BaseTensor o = make_tensor(nv);
  const auto& P = prime_table();
  for (int64_t e = 0; e < o.size(); ++e) {
    const int64_t lo = e & ((1ll << j) - 1);
    const int64_t e0 = lo | ((e >> j) << (j + 1));
    const int64_t e1 = e0 | (1ll << j);
    const int32_t v0 = t.val[e0], v1 = t.val[e1];
    const bool f0 = v0 > NEG_CUT, f1 = v1 > NEG_CUT;
    if (!f0 && !f1) { set_infeasible(o, e); continue; }
    const int32_t best = (f0 && f1) ? std::max(v0, v1) : (f0 ? v0 : v1);
    o.val[e] = best;
    for (int p = 0; p < NP; ++p) {
      uint32_t r = 0;
      if (f0 && v0 == best) r = addmod(r, t.res[(size_t)p * t.size() + e0], P[p]);
      if (f1 && v1 == best) r = addmod(r, t.res[(size_t)p * t.size() + e1], P[p]);
      o.res[(size_t)p * o.size() + e] = r;
    }
  }
  return o;
}

void flatten(Network& net) {
  int64_t total = 0;
  for (const auto& T : net.tensors) total += T.size();
  net.flat_total = total;
  net.flat.assign((size_t)(1 + NP_FLAT) * total, 0);
  int64_t off = 0;
  for (const auto& T : net.tensors) {
    const int64_t n = T.size();
    for (int64_t e = 0; e < n; ++e) net.flat[off + e] = (uint32_t)T.val[e];
    for (int p = 0; p < NP_FLAT; ++p)
      for (int64_t e = 0; e < n; ++e)
        net.flat[(size_t)(p + 1) * total + off + e] = T.res[(size_t)p * n + e];
    off += n;
  }
}

void simplify(Network& net) {
  const auto& P = prime_table();
  std::vector<BaseTensor>& T = net.tensors;
  std::vector<char> alive(T.size(), 1);
  bool changed = true;
  while (changed) {
    changed = false;
    // holders of each variable
    std::vector<std::vector<int>> hold(net.n);
    for (size_t i = 0; i < T.size(); ++i)
      if (alive[i])
        for (int v : T[i].vars) hold[v].push_back((int)i);
    // 1) fold scalars
    for (size_t i = 0; i < T.size(); ++i) {
      if (!alive[i] || !T[i].vars.empty()) continue;
      if (T[i].val[0] <= NEG_CUT) net.infeasible = true;
      else {
        net.const_val += T[i].val[0];
        for (int p = 0; p < NP; ++p) net.const_res[p] = mulmod(net.const_res[p], T[i].res[p], P[p]);
      }
      alive[i] = 0;
      changed = true;
    }
    if (changed) continue;
    // 2) absorb a tensor into another holding all of its variables; 3) sum
    // out variables held by exactly one tensor.  Tensors touched in this
    // sweep wait for the next one (holders are rebuilt per sweep).
    std::vector<char> touched(T.size(), 0);
    for (size_t i = 0; i < T.size(); ++i) {
      if (!alive[i] || touched[i] || T[i].vars.empty()) continue;
      for (int cand : hold[T[i].vars[0]]) {
        if (cand == (int)i || !alive[cand] || touched[cand]) continue;
        const auto& cv = T[cand].vars;
        if (cv.size() < T[i].vars.size()) continue;
        if (cv.size() == T[i].vars.size() && cand > (int)i) continue;  // keep lower id
        bool subset = std::all_of(T[i].vars.begin(), T[i].vars.end(), [&](int v) {
          return std::find(cv.begin(), cv.end(), v) != cv.end();
        });
        if (!subset) continue;
        absorb(T[cand], T[i]);
        alive[i] = 0;
        touched[i] = touched[cand] = 1;
        changed = true;
        break;
      }
    }
    if (changed) continue;
    for (int v = 0; v < net.n; ++v) {
      if (hold[v].size() != 1) continue;
      const int i = hold[v][0];
      if (touched[i]) continue;
      const int j = (int)(std::find(T[i].vars.begin(), T[i].vars.end(), v) - T[i].vars.begin());
      net.peel.push_back(PeelRec{v, T[i].vars, T[i].val});
      T[i] = sum_out(T[i], j);
      touched[i] = 1;
      changed = true;
    }
  }
  std::vector<BaseTensor> keep;
  for (size_t i = 0; i < T.size(); ++i)
    if (alive[i]) keep.push_back(std::move(T[i]));
  T = std::move(keep);
}

}  // namespace bbtn
