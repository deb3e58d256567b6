#include "plan.h"
#include "kernels.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <iterator>
#include <map>

namespace bbtn {

// Runs of consecutive output bits mapping onto consecutive input bits.
GatherPlan make_gather_plan(int r_in, int r_out, const int32_t* src_bits) {
  BBTN_REQUIRE(r_in >= 0 && r_in <= 40 && r_out >= 0 && r_out <= r_in,
               "gather: bad ranks");
  GatherPlan g;
  g.r_in = r_in;
  g.r_out = r_out;
  uint64_t used = 0;
  for (int j = 0; j < r_out; ++j) {
    const int s = src_bits[j];
    BBTN_REQUIRE(s >= 0 && s < r_in, "gather: source bit out of range");
    BBTN_REQUIRE(!(used >> s & 1), "gather: source bit used twice");
    used |= 1ull << s;
    if (g.n_runs > 0) {
      GatherRun& last = g.runs[g.n_runs - 1];
      if (last.out_lo + last.len == j && last.in_lo + last.len == s) {
        ++last.len;
        continue;
      }
    }
    g.runs[g.n_runs++] = GatherRun{j, s, 1};
  }
  const uint64_t all = r_in >= 64 ? ~0ull : ((1ull << r_in) - 1);
  g.fixed_mask = all & ~used;
  return g;
}

namespace {

std::vector<int32_t> free_vars(const std::vector<int32_t>& vs, const std::vector<uint64_t>& fx) {
  std::vector<int32_t> o;
  for (int v : vs)
    if (!bit_get(fx, v)) o.push_back(v);
  return o;
}

std::vector<int32_t> isect(const std::vector<int32_t>& a, const std::vector<int32_t>& b) {
  std::vector<int32_t> o;
  std::set_intersection(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(o));
  return o;
}
std::vector<int32_t> minus(const std::vector<int32_t>& a, const std::vector<int32_t>& b) {
  std::vector<int32_t> o;
  std::set_difference(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(o));
  return o;
}
std::vector<int32_t> cat3(const std::vector<int32_t>& a, const std::vector<int32_t>& b,
                          const std::vector<int32_t>& c) {
  std::vector<int32_t> o = a;
  o.insert(o.end(), b.begin(), b.end());
  o.insert(o.end(), c.begin(), c.end());
  return o;
}

}  // namespace

GroupPlan build_plan(const Network& net, const Tree& tree,
                     const std::vector<uint64_t>& fixed, bool keep_all, int defer_log2) {
  static std::atomic<uint64_t> next_uid{1};
  GroupPlan g;
  g.uid = next_uid++;
  g.fixed = fixed;
  g.keep_all = keep_all;
  for (int v = 0; v < net.n; ++v)
    if (bit_get(fixed, v)) g.fixed_vars.push_back(v);
  enum { FOLDED, BASE, STEP };
  const int NN = (int)tree.nodes.size();
  std::vector<int> status(NN, FOLDED), rep(NN, -1), buf_of(NN, -1);
  std::vector<std::vector<int32_t>> layout(NN);  // stored layout of STEP outputs
  // subtrees without a fixed variable are the same in every branch
  std::vector<char> hasfix(NN, 0);
  for (int i = 0; i < tree.n_base; ++i)
    for (int v : tree.nodes[i].vars) hasfix[i] |= bit_get(fixed, v);
  for (int id : tree.dfs_post) hasfix[id] = hasfix[tree.nodes[id].left] | hasfix[tree.nodes[id].right];
  const bool sharing = !keep_all && !g.fixed_vars.empty();
  auto new_buf = [&](int64_t entries, int region) {
    g.buf_entries.push_back(entries);
    g.buf_region.push_back(region);
    return (int32_t)g.buf_entries.size() - 1;
  };
  // buffer lifetimes in step indices: [def, last use]
  std::vector<std::pair<int, int>> life;
  auto def = [&](int buf, int s) {
    if ((int)life.size() <= buf) life.resize(buf + 1, {-1, -1});
    life[buf] = {s, s};
  };
  auto use = [&](int buf, int s) { life[buf].second = std::max(life[buf].second, s); };

  for (int i = 0; i < tree.n_base; ++i) {
    if (free_vars(tree.nodes[i].vars, fixed).empty()) {
      status[i] = FOLDED;
      g.folded.push_back(i);
    } else {
      status[i] = BASE;
      rep[i] = i;
    }
  }
  // Deferred slicing.  A subtree whose tensors stay small when its fixed
  // variables are kept as free (batch) indices is contracted once per pass
  // with them kept, and every branch slices its root (T|_{s_S = x}, Eq. 3,
  // applied after the subtree's contraction instead of before; no fixed
  // variable is summed inside it, so the sliced root is the same).
  // fx[id]: fixed variables of the non-folded base tensors below id;
  // widest[id]: largest rank, with fx kept, of the tensors of its subtree.
  std::vector<std::vector<int32_t>> fx(NN);
  std::vector<int> widest(NN, 0);
  std::vector<char> deferred(NN, 0);
  // the node whose output is the branch result: the root, or, when the root
  // only joins subtrees whose variables are all fixed (folded), the node it
  // aliases
  int eff_root = tree.root;
  if (tree.root >= tree.n_base) {
    std::vector<char> all_folded(NN, 0);
    for (int i = 0; i < tree.n_base; ++i) all_folded[i] = status[i] == FOLDED;
    for (int id : tree.dfs_post)
      all_folded[id] = all_folded[tree.nodes[id].left] && all_folded[tree.nodes[id].right];
    while (eff_root >= tree.n_base) {
      const TNode& n = tree.nodes[eff_root];
      if (all_folded[n.left] == all_folded[n.right]) break;
      eff_root = all_folded[n.left] ? n.right : n.left;
    }
  }
  if (sharing && defer_log2 > 0) {
    for (int i = 0; i < tree.n_base; ++i)
      if (status[i] == BASE) {
        for (int v : tree.nodes[i].vars)
          if (bit_get(fixed, v)) fx[i].push_back(v);
        widest[i] = (int)tree.nodes[i].vars.size();
      }
    for (int id : tree.dfs_post) {
      const TNode& n = tree.nodes[id];
      std::set_union(fx[n.left].begin(), fx[n.left].end(), fx[n.right].begin(),
                     fx[n.right].end(), std::back_inserter(fx[id]));
      const int own = (int)free_vars(n.vars, fixed).size() + (int)fx[id].size();
      widest[id] = std::max({own, widest[n.left], widest[n.right]});
      deferred[id] = hasfix[id] && widest[id] <= defer_log2 && id != eff_root;
    }
  }
  auto with_fx = [&](std::vector<int32_t> v, int node) {
    std::vector<int32_t> o;
    std::set_union(v.begin(), v.end(), fx[node].begin(), fx[node].end(), std::back_inserter(o));
    return o;
  };
  for (int id : tree.dfs_post) {  // subtrees are contiguous in this order
    const TNode& n = tree.nodes[id];
    const int sl = status[n.left], sr = status[n.right];
    if (sl == FOLDED && sr == FOLDED) { status[id] = FOLDED; continue; }
    if (sl == FOLDED || sr == FOLDED) {
      const int child = sl == FOLDED ? n.right : n.left;
      status[id] = status[child];
      rep[id] = rep[child];
      if (free_vars(n.vars, fixed) != free_vars(tree.nodes[rep[id]].vars, fixed))
        throw Error(BBTN_E_INTERNAL, "plan: alias with different variables");
      continue;
    }
    status[id] = STEP;
    rep[id] = id;
    const int ra = rep[n.left], rb_ = rep[n.right];
    const bool dfr = deferred[id];
    const auto A = dfr ? with_fx(free_vars(tree.nodes[ra].vars, fixed), ra)
                       : free_vars(tree.nodes[ra].vars, fixed);
    const auto B = dfr ? with_fx(free_vars(tree.nodes[rb_].vars, fixed), rb_)
                       : free_vars(tree.nodes[rb_].vars, fixed);
    const auto C = dfr ? with_fx(free_vars(n.vars, fixed), id) : free_vars(n.vars, fixed);
    const auto AB = isect(A, B);
    auto batch = isect(AB, C);
    auto K = minus(AB, C);
    auto M = isect(minus(A, B), C);
    auto N = isect(minus(B, A), C);
    // Order within each index group: the product needs A as [K][M][batch]
    // and B as [N][K][batch], any order inside a group.  Following the
    // stored layouts makes an operand's permutation a regrouping of long
    // runs, or no permutation at all: M follows A's layout, N follows B's,
    // K and batch (shared by both) follow the larger operand's.
    {
      const auto& LA = status[ra] == BASE ? tree.nodes[ra].vars : layout[ra];
      const auto& LB = status[rb_] == BASE ? tree.nodes[rb_].vars : layout[rb_];
      auto by = [](std::vector<int32_t>& v, const std::vector<int32_t>& L) {
        auto pos = [&](int32_t x) { return std::find(L.begin(), L.end(), x) - L.begin(); };
        std::stable_sort(v.begin(), v.end(), [&](int32_t x, int32_t y) { return pos(x) < pos(y); });
      };
      const auto& LP = A.size() >= B.size() ? LA : LB;
      by(K, LP);
      by(batch, LP);
      by(M, LA);
      by(N, LB);
    }
    if (!minus(minus(A, B), C).empty() || !minus(minus(B, A), C).empty())
      throw Error(BBTN_E_INTERNAL, "plan: variable private to one operand");
    Step s;
    s.node = id;
    s.shared = sharing && (!hasfix[id] || dfr);
    s.rb = (int)batch.size();
    s.rm = (int)M.size();
    s.rn = (int)N.size();
    s.rk = (int)K.size();
    s.a_vars = cat3(K, M, batch);
    s.b_vars = cat3(N, K, batch);
    s.c_vars = cat3(N, M, batch);
    const int si = (int)g.steps.size();
    const int own_region = s.shared ? R_SUBTREE : R_BRANCH;
    auto make_op = [&](int r, const std::vector<int32_t>& want, int which) {
      Operand op;
      if (status[r] == BASE) {
        const auto& tv = tree.nodes[r].vars;  // physical order of the base tensor
        op.base = true;
        op.id = tree.nodes[r].base;
        op.r_in = (int)tv.size();
        for (int v : want)
          op.src_bits.push_back((int)(std::find(tv.begin(), tv.end(), v) - tv.begin()));
        if (!dfr)  // a deferred step reads base tensors whole
          for (int j = 0; j < (int)tv.size(); ++j)
            if (bit_get(fixed, tv[j])) op.fixed_pos.push_back({j, tv[j]});
        op.base_op = (int)g.base_ops.size();
        g.base_ops.push_back({si, which});
      } else {
        const auto& have = layout[r];
        op.base = false;
        op.id = buf_of[r];
        op.r_in = (int)have.size();
        // a branch step reading a shared subtree's root: that root lives in
        // the shared region and is gathered per branch (no branch stride)
        if (!s.shared && g.buf_region[op.id] != R_BRANCH) g.buf_region[op.id] = R_SHARED;
        op.direct = (have == want) && g.buf_region[op.id] != R_SHARED;
        for (int v : want)
          op.src_bits.push_back((int)(std::find(have.begin(), have.end(), v) - have.begin()));
        // the root of a deferred subtree holds fixed variables: sliced per
        // branch by the branch's states, like a base tensor
        if (!dfr)
          for (int j = 0; j < (int)have.size(); ++j)
            if (bit_get(fixed, have[j])) op.fixed_pos.push_back({j, have[j]});
        if (!op.fixed_pos.empty()) {
          op.direct = false;
          op.base_op = (int)g.base_ops.size();
          g.base_ops.push_back({si, which});
        }
      }
      if (!op.direct) {
        op.temp = new_buf(1ll << want.size(), own_region);
        def(op.temp, si);
      }
      if (!op.base) use(op.id, si);
      return op;
    };
    s.a = make_op(ra, s.a_vars, 0);
    s.b = make_op(rb_, s.b_vars, 1);
    s.out = new_buf(1ll << C.size(), own_region);
    def(s.out, si);
    buf_of[id] = s.out;
    layout[id] = s.c_vars;
    g.max_rank = std::max({g.max_rank, (int)s.a_vars.size(), (int)s.b_vars.size(),
                           (int)s.c_vars.size()});
    if (s.shared) g.shared_macs += s.macs();
    else { g.macs += s.macs(); g.n_branch_steps++; }
    g.steps.push_back(std::move(s));
  }
  if (tree.root >= 0 && status[tree.root] == STEP) {
    g.root_buf = buf_of[rep[tree.root]];  // the root may alias a step below it
    use(g.root_buf, (int)g.steps.size());  // read after the last step
  } else if (tree.root >= 0 && status[tree.root] == BASE) {
    throw Error(BBTN_E_INTERNAL, "plan: root is a base tensor with free variables");
  }
  // maximal shared subtrees: runs of consecutive shared steps ending at a
  // step whose output is read by a branch step
  for (int i = 0; i < (int)g.steps.size();) {
    if (!g.steps[i].shared) { ++i; continue; }
    int j = i;
    while (j < (int)g.steps.size() && g.steps[j].shared) {
      const bool root = g.buf_region[g.steps[j].out] == R_SHARED;
      ++j;
      if (root) break;
    }
    g.shared_ranges.push_back({i, j});
    i = j;
  }
  // offsets: first fit over lifetimes per region (or disjoint when keeping
  // everything); shared-region buffers never overlap
  const int nb = (int)g.buf_entries.size();
  g.buf_off.assign(nb, 0);
  if (keep_all) {
    int64_t off = 0;
    for (int i = 0; i < nb; ++i) { g.buf_off[i] = off; off += g.buf_entries[i]; }
    g.peak = off;
    return g;
  }
  for (int i = 0; i < nb; ++i)
    if (g.buf_region[i] == R_SHARED) { g.buf_off[i] = g.shared_total; g.shared_total += g.buf_entries[i]; }
  for (int region : {R_BRANCH, R_SUBTREE}) {
    std::vector<int> order;
    for (int i = 0; i < nb; ++i)
      if (g.buf_region[i] == region) order.push_back(i);
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return life[x].first < life[y].first; });
    std::vector<int> active;  // placed buffers still alive
    int64_t peak = 0;
    for (int i : order) {
      active.erase(std::remove_if(active.begin(), active.end(),
                                  [&](int j) { return life[j].second < life[i].first; }),
                   active.end());
      std::vector<std::pair<int64_t, int64_t>> busy;
      for (int j : active) busy.push_back({g.buf_off[j], g.buf_off[j] + g.buf_entries[j]});
      std::sort(busy.begin(), busy.end());
      int64_t off = 0;
      for (auto& bz : busy) {
        if (off + g.buf_entries[i] <= bz.first) break;
        off = std::max(off, bz.second);
      }
      g.buf_off[i] = off;
      peak = std::max(peak, off + g.buf_entries[i]);
      active.push_back(i);
    }
    (region == R_BRANCH ? g.peak : g.subtree_peak) = peak;
  }
  return g;
}

}  // namespace bbtn
