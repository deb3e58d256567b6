// Solve driver: network -> contraction tree -> branch-and-bound search ->
// batched contraction of every branch sub-network per prime pass -> tropical
// sum of the branch results -> CRT + certification -> one optimal
// configuration.  Several instances go through the same launches.
#include "solve.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <future>
#include <map>
#include <mutex>
#include <thread>

#include "crt.h"
#include "exec.h"
#include "persist.h"
#include "scorer.h"
#include "search.h"
#include "trace.h"

namespace bbtn {

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// tree ids, unique over the process (step programs are cached by them)
std::atomic<uint64_t> next_id{1};

// A network's structure: the variable lists of its simplified tensors,
// which do not depend on couplings or weights.
std::vector<std::vector<int32_t>> shape_of(const Network& net) {
  std::vector<std::vector<int32_t>> shape;
  shape.reserve(net.tensors.size() + 1);
  shape.push_back({net.n});
  for (const auto& T : net.tensors) shape.push_back(T.vars);
  return shape;
}

TreeRef tree_for(bbtn_ctx* ctx, const Network& net, const SearchOptions* probe) {
  const std::vector<std::vector<int32_t>> shape = shape_of(net);
  const bool refine = probe && ctx->opt.order_refine > 0;
  std::shared_ptr<std::promise<TreeRef>> mine;
  {
    std::unique_lock<std::mutex> lk(ctx->tree_mu);
    auto it = ctx->tree_cache.find(shape);
    if (it != ctx->tree_cache.end()) return TreeRef{it->second.tree, it->second.id};
    if (refine) {
      // a refined order is costly: one planning thread builds it, the
      // others with the same structure wait for it; other structures are
      // built in parallel
      auto bt = ctx->tree_building.find(shape);
      if (bt != ctx->tree_building.end()) {
        std::shared_future<TreeRef> f = bt->second;
        lk.unlock();
        return f.get();  // rethrows the builder's error
      }
      mine = std::make_shared<std::promise<TreeRef>>();
      ctx->tree_building.emplace(shape, mine->get_future().share());
    }
  }
  try {
    bool complete = true;
    auto tree = std::make_shared<const Tree>(
        refine ? choose_order(net, ctx->opt.order_refine, *probe, &complete)
               : (ctx->opt.order_refine < 0 ? minfill_tree(net) : greedy_tree(net)));
    std::lock_guard<std::mutex> lk(ctx->tree_mu);
    TreeRef r;
    auto it = ctx->tree_cache.find(shape);
    if (it != ctx->tree_cache.end()) {
      r = TreeRef{it->second.tree, it->second.id};
    } else if (!complete) {
      r = TreeRef{tree, next_id++};  // cut short by the time limit: not cached
    } else {
      if (ctx->tree_cache.size() >= 8) ctx->tree_cache.clear();
      r = TreeRef{tree, next_id++};
      ctx->tree_cache.emplace(shape, bbtn_ctx::TreeEntry{tree, r.id});
    }
    if (mine) {
      ctx->tree_building.erase(shape);
      mine->set_value(r);
    }
    return r;
  } catch (...) {
    if (mine) {
      std::lock_guard<std::mutex> lk(ctx->tree_mu);
      ctx->tree_building.erase(shape);
      mine->set_exception(std::current_exception());
    }
    throw;
  }
}

// The step program of fixed set `mask` on tree `t`, from the context's
// cache (instances with the same structure and fixed set share it).
std::shared_ptr<const GroupPlan> plan_for(bbtn_ctx* ctx, const Network& net, const TreeRef& t,
                                          const std::vector<uint64_t>& mask, bool keep_all) {
  auto key = std::make_tuple(t.id, keep_all, mask);
  {
    std::lock_guard<std::mutex> lk(ctx->tree_mu);
    auto it = ctx->plan_cache.find(key);
    if (it != ctx->plan_cache.end()) return it->second;
  }
  // subtrees whose tensors, with their fixed variables kept, stay within
  // T_target are contracted once per pass and sliced per branch (not in
  // keep-all plans, whose intermediates are traced)
  const int defer = keep_all ? 0 : std::max(0, ctx->opt.log2_target);
  auto plan = std::make_shared<const GroupPlan>(build_plan(net, *t.tree, mask, keep_all, defer));
  std::lock_guard<std::mutex> lk(ctx->tree_mu);
  auto it = ctx->plan_cache.find(key);
  if (it != ctx->plan_cache.end()) return it->second;
  if (ctx->plan_cache.size() >= 64) ctx->plan_cache.clear();
  ctx->plan_cache.emplace(std::move(key), plan);
  return plan;
}

// Leaves of the search in a flat order: (group, index in group).
struct LeafRef {
  int32_t group;
  int64_t idx;
};

// Per-branch results of one pass: value and k residues per leaf.
struct PassOut {
  std::vector<std::vector<int32_t>> val;                // [group][leaf]
  std::vector<std::vector<std::vector<uint32_t>>> res;  // [group][p][leaf]
};

int64_t leaves_per_chunk(bbtn_ctx* ctx, const GroupPlan& g, int k) {
  size_t freeb = 0, totalb = 0;
  if (hipMemGetInfo(&freeb, &totalb) != hipSuccess) freeb = (size_t)8 << 30;
  double budget = 0.45 * (double)(freeb + ctx->work.bytes);
  if (ctx->memcap->cap > 0)  // what the cap leaves, counting the workspace this replaces
    budget = std::min(budget, 0.9 * ((double)ctx->memcap->cap - (double)ctx->memcap->held.load() +
                                     (double)ctx->work.bytes));
  const double per = (double)(1 + k) * 4.0 * (double)std::max<int64_t>(g.peak, 1) * 1.05 +
                     (double)(1 + k) * 12.0 + 8.0 * (double)(g.base_ops.size() + 1);
  int64_t L = (int64_t)(budget / per);
  return std::max<int64_t>(1, std::min<int64_t>(L, 1 << 20));
}

// One instance's part of a pass: the selected leaves (ascending indices per
// group) of its groups.
struct PassItem {
  const Network* net;
  const std::vector<LeafGroup>* groups;
  const std::vector<std::shared_ptr<const GroupPlan>>* plans;
  const std::vector<std::vector<int64_t>>* sel;
  PassOut* out;
};

// A pass with primes pidx over several instances: every group whose
// operands fit in LDS, of every instance, in one persistent launch; the
// other groups step by step, batched over their branches (chunked by
// memory), or one branch at a time when batching is off.
void run_pass(bbtn_ctx* ctx, const std::vector<PassItem>& items, const std::vector<int>& pidx,
              bool batched) {
  const int k = (int)pidx.size();
  hipStream_t st = ctx->stream;
  std::vector<uint32_t> primes(k);
  for (int p = 0; p < k; ++p) primes[p] = prime_table()[pidx[p]];
  const Moduli mod = make_moduli(k, primes.data());
  std::vector<const Network*> nets;
  for (const PassItem& it : items) nets.push_back(it.net);
  BaseDev bd;
  std::vector<std::vector<int64_t>> offs;
  upload_bases(ctx, nets, pidx.data(), k, bd, offs, ctx->base);
  // the selected branches of every group, packed per group
  std::vector<std::vector<std::vector<uint8_t>>> asg(items.size());
  for (size_t ii = 0; ii < items.size(); ++ii) {
    const PassItem& it = items[ii];
    const auto& groups = *it.groups;
    const auto& sel = *it.sel;
    it.out->val.assign(groups.size(), {});
    it.out->res.assign(groups.size(), {});
    asg[ii].resize(groups.size());
    for (size_t gi = 0; gi < groups.size(); ++gi) {
      const LeafGroup& G = groups[gi];
      it.out->val[gi].assign(G.count, NEG);
      it.out->res[gi].assign(k, std::vector<uint32_t>(G.count, 0));
      const size_t S = G.vars.size();
      asg[ii][gi].resize(sel[gi].size() * S);
      for (size_t i = 0; i < sel[gi].size(); ++i)
        std::memcpy(&asg[ii][gi][i * S], &G.assign[sel[gi][i] * S], S);
    }
  }
  auto scatter = [&](size_t ii, size_t gi, size_t c0, int64_t L, const uint32_t* h) {
    PassOut& out = *items[ii].out;
    const auto& sel = *items[ii].sel;
    for (int64_t i = 0; i < L; ++i) {
      const int64_t leaf = sel[gi][c0 + i];
      out.val[gi][leaf] = (int32_t)h[i];
      for (int p = 0; p < k; ++p) out.res[gi][p][leaf] = h[(size_t)(p + 1) * L + i];
    }
  };
  std::vector<PersistJob> jobs;
  std::vector<std::pair<size_t, size_t>> job_src;
  std::vector<std::vector<uint32_t>> job_out;
  for (size_t ii = 0; ii < items.size(); ++ii)
    for (size_t gi = 0; gi < items[ii].groups->size(); ++gi) {
      const auto& sel = *items[ii].sel;
      if (!batched || sel[gi].empty() || !persist_fits(*(*items[ii].plans)[gi], k)) continue;
      job_src.push_back({ii, gi});
    }
  job_out.resize(job_src.size());
  for (size_t j = 0; j < job_src.size(); ++j) {
    const size_t ii = job_src[j].first, gi = job_src[j].second;
    jobs.push_back(PersistJob{(*items[ii].plans)[gi].get(), items[ii].net, offs[ii].data(),
                              asg[ii][gi].data(), (int64_t)(*items[ii].sel)[gi].size(),
                              &job_out[j]});
  }
  if (!jobs.empty()) {
    run_persistent(ctx, jobs, bd, mod, st);
    for (size_t j = 0; j < jobs.size(); ++j)
      scatter(job_src[j].first, job_src[j].second, 0, jobs[j].L, job_out[j].data());
  }
  for (size_t ii = 0; ii < items.size(); ++ii) {
    const PassItem& it = items[ii];
    BaseDev bdi;
    bdi.k = k;
    bdi.off = offs[ii];
    bdi.total = bd.total;
    bdi.t = bd.t;
    const auto& sel = *it.sel;
    for (size_t gi = 0; gi < it.groups->size(); ++gi) {
      if (sel[gi].empty()) continue;
      const GroupPlan& g = *(*it.plans)[gi];
      if (batched && persist_fits(g, k)) continue;
      const size_t S = (*it.groups)[gi].vars.size();
      const int64_t chunk = batched ? leaves_per_chunk(ctx, g, k) : 1;
      for (size_t c0 = 0; c0 < sel[gi].size(); c0 += chunk) {
        const int64_t L = std::min<int64_t>(chunk, (int64_t)(sel[gi].size() - c0));
        ctx->leafout.ensure((size_t)(1 + k) * L * 4);
        const DevTensor o{ctx->leafout.as<uint32_t>(), L};
        run_group(ctx, *it.net, g, bdi, mod, &asg[ii][gi][c0 * S], L, o, st,
                  /*reuse=*/sel[gi].size() > (size_t)chunk, /*shared_ready=*/c0 > 0,
                  /*L_group=*/(int64_t)sel[gi].size());
        std::vector<uint32_t> h((size_t)(1 + k) * L);
        BBTN_HIP(hipMemcpyAsync(h.data(), o.ptr, h.size() * 4, hipMemcpyDeviceToHost, st));
        BBTN_HIP(hipStreamSynchronize(st));
        ctx->prof.resolve();
        scatter(ii, gi, c0, L, h.data());
      }
    }
  }
}

// Configuration recovery ("Discussion": configurations as a semiring
// extension).  For each item: a values-only recontraction of its winning
// leaf that keeps every intermediate, an argmax traceback from the root, and
// the variables summed out while simplifying, in reverse order.
struct RecoverItem {
  const Network* net;
  const TreeRef* tree;
  const LeafGroup* G;
  int64_t leaf;
  std::vector<int8_t>* states;
};

// One traceback launch for the items `idx`, item idx[j] reading its
// workspace at ws[j].
void trace_items(bbtn_ctx* ctx, const std::vector<RecoverItem>& items,
                 const std::vector<std::shared_ptr<const GroupPlan>>& plans,
                 const std::vector<size_t>& idx,
                 const std::vector<const int32_t*>& ws) {
  hipStream_t st = ctx->stream;
  std::vector<TraceStep> ts;
  std::vector<int32_t> vars;
  std::vector<size_t> ts0(idx.size()), vars0(idx.size()), asg0(idx.size());
  size_t asg_bytes = 0;
  int32_t max_steps = 0, max_words = 0, max_vars = 0;
  std::vector<size_t> ts_n(idx.size()), vars_n(idx.size());
  // items with the same plan share one copy of its steps and variables
  std::map<const GroupPlan*, size_t> first_of;
  for (size_t j = 0; j < idx.size(); ++j) {
    const GroupPlan& g = *plans[idx[j]];
    const int32_t n = items[idx[j]].net->n;
    asg0[j] = asg_bytes;
    asg_bytes += (size_t)n;
    max_vars = std::max<int32_t>(max_vars, n);
    auto hit = first_of.find(&g);
    if (hit != first_of.end()) {
      ts0[j] = ts0[hit->second];
      vars0[j] = vars0[hit->second];
      ts_n[j] = ts_n[hit->second];
      vars_n[j] = vars_n[hit->second];
      continue;
    }
    first_of.emplace(&g, j);
    ts0[j] = ts.size();
    vars0[j] = vars.size();
    for (const Step& s : g.steps) {
      TraceStep t{};
      t.rb = s.rb; t.rm = s.rm; t.rn = s.rn; t.rk = s.rk;
      t.a_off = g.buf_off[s.a.direct ? s.a.id : s.a.temp];
      t.b_off = g.buf_off[s.b.direct ? s.b.id : s.b.temp];
      t.var_off = (int32_t)(vars.size() - vars0[j]);
      vars.insert(vars.end(), s.a_vars.begin(), s.a_vars.end());
      vars.insert(vars.end(), s.b_vars.begin(), s.b_vars.end());
      ts.push_back(t);
    }
    ts_n[j] = ts.size() - ts0[j];
    vars_n[j] = vars.size() - vars0[j];
    max_steps = std::max<int32_t>(max_steps, (int32_t)ts_n[j]);
    max_words = std::max<int32_t>(max_words, (int32_t)vars_n[j]);
  }
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t off_j = 0;
  const size_t off_t = off_j + al(idx.size() * sizeof(TraceJob));
  const size_t off_v = off_t + al(std::max<size_t>(ts.size(), 1) * sizeof(TraceStep));
  const size_t off_a = off_v + al(std::max<size_t>(vars.size(), 1) * 4);
  const size_t off_s = off_a + al(std::max<size_t>(asg_bytes, 1));
  const size_t total = off_s + al(idx.size() * 4);
  ctx->misc.ensure(total);
  char* base = ctx->misc.as<char>();
  std::vector<char> host(total, 0);
  std::vector<TraceJob> jobs(idx.size());
  for (size_t j = 0; j < idx.size(); ++j) {
    TraceJob& jb = jobs[j];
    jb.steps = (const TraceStep*)(base + off_t) + ts0[j];
    jb.vars = (const int32_t*)(base + off_v) + vars0[j];
    jb.ws = ws[j];
    jb.assign = (int8_t*)(base + off_a) + asg0[j];
    jb.status = (int32_t*)(base + off_s) + j;
    jb.n_steps = (int32_t)ts_n[j];
    jb.n_var_words = (int32_t)vars_n[j];
    jb.n_vars = items[idx[j]].net->n;
    std::memcpy(&host[off_a + asg0[j]], items[idx[j]].states->data(), (size_t)jb.n_vars);
  }
  std::memcpy(&host[off_j], jobs.data(), jobs.size() * sizeof(TraceJob));
  if (!ts.empty()) std::memcpy(&host[off_t], ts.data(), ts.size() * sizeof(TraceStep));
  if (!vars.empty()) std::memcpy(&host[off_v], vars.data(), vars.size() * 4);
  BBTN_HIP(hipMemcpyAsync(base, host.data(), total, hipMemcpyHostToDevice, st));
  launch_trace((const TraceJob*)(base + off_j), (int32_t)idx.size(), max_steps, max_words,
               max_vars, st);
  BBTN_HIP(hipMemcpyAsync(host.data() + off_a, base + off_a, total - off_a, hipMemcpyDeviceToHost,
                          st));
  BBTN_HIP(hipStreamSynchronize(st));
  for (size_t j = 0; j < idx.size(); ++j) {
    int32_t stat = 0;
    std::memcpy(&stat, &host[off_s + 4 * j], 4);
    if (stat) throw Error(BBTN_E_INTERNAL, "configuration traceback failed");
    std::memcpy(items[idx[j]].states->data(), &host[off_a + asg0[j]], (size_t)jobs[j].n_vars);
  }
}

void recover_configs(bbtn_ctx* ctx, const std::vector<RecoverItem>& items) {
  if (items.empty()) return;
  hipStream_t st = ctx->stream;
  const size_t n_items = items.size();
  std::vector<std::shared_ptr<const GroupPlan>> plans(n_items);
  std::vector<const Network*> nets(n_items);
  for (size_t i = 0; i < n_items; ++i) {
    const RecoverItem& it = items[i];
    const LeafGroup& G = *it.G;
    it.states->assign(it.net->n, -1);
    for (size_t j = 0; j < G.vars.size(); ++j)
      (*it.states)[G.vars[j]] = (int8_t)G.assign[it.leaf * G.vars.size() + j];
    plans[i] = plan_for(ctx, *it.net, *it.tree, G.mask, /*keep_all=*/true);
    nets[i] = it.net;
  }
  const int pidx0 = 0;
  BaseDev bd;
  std::vector<std::vector<int64_t>> offs;
  upload_bases(ctx, nets, &pidx0, 0, bd, offs, ctx->base);
  const Moduli mod = make_moduli(0, nullptr);
  const uint64_t macs0 = ctx->last_macs;
  std::vector<size_t> pers, rest;
  for (size_t i = 0; i < n_items; ++i) {
    if (plans[i]->steps.empty()) continue;
    if (ctx->opt.batched && persist_fits(*plans[i], 0)) pers.push_back(i);
    else rest.push_back(i);
  }
  if (!pers.empty()) {
    // one persistent launch; task j keeps its workspace at j * scratch
    std::vector<std::vector<uint32_t>> outs(pers.size());
    std::vector<PersistJob> jobs;
    for (size_t j = 0; j < pers.size(); ++j) {
      const RecoverItem& it = items[pers[j]];
      jobs.push_back(PersistJob{plans[pers[j]].get(), it.net, offs[pers[j]].data(),
                                &it.G->assign[it.leaf * it.G->vars.size()], 1, &outs[j]});
    }
    int64_t scratch = 0;
    run_persistent(ctx, jobs, bd, mod, st, /*per_task_scratch=*/true, &scratch);
    std::vector<const int32_t*> ws(pers.size());
    for (size_t j = 0; j < pers.size(); ++j) ws[j] = ctx->work.as<int32_t>() + (int64_t)j * scratch;
    trace_items(ctx, items, plans, pers, ws);
  }
  for (size_t i : rest) {
    // step by step on the workspace base, where the traceback then reads
    const RecoverItem& it = items[i];
    BaseDev bdi;
    bdi.k = 0;
    bdi.off = offs[i];
    bdi.total = bd.total;
    bdi.t = bd.t;
    ctx->leafout.ensure(64);
    const DevTensor o{ctx->leafout.as<uint32_t>(), 1};
    run_group(ctx, *it.net, *plans[i], bdi, mod, &it.G->assign[it.leaf * it.G->vars.size()], 1, o,
              st);
    trace_items(ctx, items, plans, {i}, {ctx->work.as<int32_t>()});
  }
  ctx->last_macs = macs0;  // bookkeeping counts the counting passes only
  for (const RecoverItem& it : items) {
    const Network& net = *it.net;
    std::vector<int8_t>& states = *it.states;
    // variables eliminated while simplifying, in reverse order
    for (size_t i = net.peel.size(); i-- > 0;) {
      const PeelRec& r = net.peel[i];
      int64_t b = 0;
      int pos = -1;
      for (size_t j = 0; j < r.tvars.size(); ++j) {
        if (r.tvars[j] == r.var) { pos = (int)j; continue; }
        b |= (int64_t)(states[r.tvars[j]] & 1) << j;
      }
      const int32_t v0 = r.tval[b], v1 = r.tval[b | (1ll << pos)];
      const bool f0 = v0 > NEG_CUT, f1 = v1 > NEG_CUT;
      states[r.var] = (f1 && (!f0 || v1 > v0)) ? 1 : 0;
    }
    for (int v = 0; v < net.n; ++v)
      if (states[v] < 0) states[v] = 0;  // variable in no tensor at all
  }
}

// The context that recovers configurations concurrently with the counting
// passes: created on first use with the same device and executor options,
// its own stream and workspaces, and a copy of the tile choices.
bbtn_ctx* aux_context(bbtn_ctx* ctx) {
  if (!ctx->aux) {
    bbtn_options o = ctx->opt;
    o.stream = nullptr;
    o.scorer_weights = nullptr;
    o.autotune_cache = nullptr;
    bbtn_ctx* a = nullptr;
    const bbtn_status s = bbtn_create(&o, &a);
    if (s != BBTN_OK) throw Error(s, "cannot create the configuration-recovery context");
    a->attach_memcap(ctx->memcap);  // one cap for both contexts
    ctx->aux = a;
  }
  ctx->aux->tune = ctx->tune;
  return ctx->aux;
}

// Run f(i) for i in [0, n) on up to `threads` host threads.
template <class F>
void parallel_for(size_t n, int threads, F&& f) {
  if (n == 0) return;
  const size_t T = std::min<size_t>(n, (size_t)std::max(1, threads));
  if (T == 1) {
    for (size_t i = 0; i < n; ++i) f(i);
    return;
  }
  std::atomic<size_t> next{0};
  std::vector<std::thread> pool;
  for (size_t t = 0; t < T; ++t)
    pool.emplace_back([&] {
      for (size_t i; (i = next.fetch_add(1)) < n;) f(i);
    });
  for (auto& th : pool) th.join();
}

// Pipeline state of one instance.
struct Work {
  TreeRef tree;
  std::vector<LeafGroup> groups;
  std::vector<std::shared_ptr<const GroupPlan>> plans;
  SearchStats stats;
  int64_t incumbent = INT64_MIN;
  bool active = true;
  double t_build = 0, t_search = 0;
  std::vector<std::vector<int64_t>> all_sel, opt_sel;
  PassOut pv, pc;
  int32_t best = NEG;
  LeafRef first{-1, -1};
  bool use_inc = false;
  std::vector<int> used;
  std::vector<uint32_t> residues;
  std::vector<uint32_t> count;
  int certified = 0;
  bool fused = false;
  std::vector<int8_t> states;
};

}  // namespace

void solve_instances(bbtn_ctx* ctx, std::vector<Instance>& insts) {
  const double t0 = now_s();
  const bbtn_options& opt = ctx->opt;
  ctx->last_macs = 0;
  ctx->clear_graphs();  // captured programs refer to the previous call's plans
  struct GraphScope {
    bbtn_ctx* c;
    ~GraphScope() { c->clear_graphs(); }
  } graph_scope{ctx};
  const double deadline = opt.time_limit_s > 0 ? t0 + opt.time_limit_s : 0;
  const size_t N = insts.size();
  std::vector<Work> W(N);
  auto fail = [&](size_t i, bbtn_status s, const std::string& msg) {
    insts[i].status = s;
    insts[i].err = msg;
    W[i].active = false;
  };
  for (Instance& in : insts)
    for (int i = 0; i < 8; ++i) in.res->seconds[i] = 0;
  const bool branch = opt.branching != 0 && opt.log2_target > 0;
  const bool values_only = opt.residues_per_pass == 0;
  const int k = values_only ? 0 : std::max(1, std::min(KUSER, opt.residues_per_pass));
  const int max_primes = std::max(k, std::min(BBTN_MAX_PRIMES, opt.max_primes));
  const auto& P = prime_table();
  // ---- planning: order, search and step programs, instances in parallel
  // (the learned scorer runs on the context's stream: one instance at a time)
  const bool scored = opt.branching == 2 && ctx->scorer_loaded;
  const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
  const int threads = scored ? 1 : (opt.host_threads > 0 ? opt.host_threads : hw);
  parallel_for(N, threads, [&](size_t i) {
    Instance& in = insts[i];
    Work& w = W[i];
    try {
      const double a = now_s();
      if (in.build) in.build(in);
      SearchOptions probe;
      probe.log2_target = opt.log2_target;
      probe.region_max = std::max(1, std::min(16, opt.region_max));
      probe.values_only = values_only;
      probe.deadline = deadline;
      w.tree = tree_for(ctx, in.net, branch ? &probe : nullptr);
      // spin-flip symmetry of a zero-field spin glass: a configuration and
      // its mirror image have the same energy and exactly one of them has a
      // given spin at +1, so that spin is fixed to +1 for the whole search
      // and the count doubled (the constant's count residues)
      int32_t flip = -1;
      if (opt.spin_flip && in.net.spin && in.net.zero_field && !in.net.infeasible) {
        flip = flip_variable(in.net, *w.tree.tree, branch ? opt.log2_target : 0);
        if (flip >= 0) {
          for (int p = 0; p < NP; ++p)
            in.net.const_res[p] = addmod(in.net.const_res[p], in.net.const_res[p], P[p]);
          if ((size_t)flip < in.ls_x.size() && in.ls_x[flip] == 0)
            for (auto& bit : in.ls_x) bit ^= 1;
        }
      }
      // value (with the folded constant, like node_bound) of the local-search
      // configuration: a lower bound on the optimum, used for global pruning
      w.incumbent = in.ls_x.empty() ? INT64_MIN : network_value(in.net, in.ls_x);
      const double b = now_s();
      if (!branch) {
        LeafGroup g;
        g.mask.assign((in.net.n + 63) / 64, 0);
        if (flip >= 0) {
          bit_set(g.mask, flip);
          g.vars = {flip};
          g.assign = {1};
        }
        g.count = 1;
        w.groups.push_back(g);
        w.stats.leaves = 1;
      } else {
        SearchOptions so;
        so.log2_target = opt.log2_target;
        so.region_max = std::max(1, std::min(16, opt.region_max));
        so.incumbent = w.incumbent;
        so.values_only = values_only;
        so.deadline = deadline;
        if (flip >= 0) so.prefix.push_back({flip, 1});
        if (scored) so.scorer = make_var_scorer(ctx, in.net, *w.tree.tree, opt.log2_target);
        bb_search(in.net, *w.tree.tree, so, w.groups, w.stats);
      }
      const double c = now_s();
      for (auto& G : w.groups) w.plans.push_back(plan_for(ctx, in.net, w.tree, G.mask, false));
      w.t_build = (b - a) + (now_s() - c);
      w.t_search = c - b;
      w.all_sel.resize(w.groups.size());
      for (size_t gi = 0; gi < w.groups.size(); ++gi)
        for (int64_t l = 0; l < w.groups[gi].count; ++l) w.all_sel[gi].push_back(l);
    } catch (const Error& e) {
      fail(i, e.status, e.what());
    } catch (const std::bad_alloc&) {
      fail(i, BBTN_E_OOM, "host allocation failed");
    } catch (const std::exception& e) {
      fail(i, BBTN_E_INTERNAL, e.what());
    }
  });
  const double t_planned = now_s();
  auto pass_items = [&](const std::vector<size_t>& idx, bool optimal_only, bool counting) {
    std::vector<PassItem> items;
    for (size_t i : idx)
      items.push_back(PassItem{&insts[i].net, &W[i].groups, &W[i].plans,
                               optimal_only ? &W[i].opt_sel : &W[i].all_sel,
                               counting ? &W[i].pc : &W[i].pv});
    return items;
  };
  std::vector<size_t> active;
  for (size_t i = 0; i < N; ++i)
    if (W[i].active) active.push_back(i);
  // ---- values pass over every leaf of every instance (the max-plus part of
  // the algebra): its exact values give each optimum, and a leaf below it
  // carries no count (global pruning with the exact incumbent), so the
  // counting passes touch only the leaves reaching the optimum
  run_pass(ctx, pass_items(active, false, false), {}, opt.batched != 0);
  const bool late = deadline > 0 && now_s() > deadline;
  std::vector<size_t> counting, recover;
  std::vector<RecoverItem> ritems;
  for (size_t i : active) {
    Work& w = W[i];
    if (late) { fail(i, BBTN_E_TIMEOUT, "time limit reached"); continue; }
    for (auto& gv : w.pv.val)
      for (int32_t v : gv)
        if (v > NEG_CUT && v > w.best) w.best = v;
    if (values_only) {
      // the optimum is the best leaf or, when the search pruned everything
      // that could not beat it, the incumbent itself
      w.use_inc = w.incumbent != INT64_MIN &&
                  (w.best <= NEG_CUT || w.incumbent > (int64_t)w.best + insts[i].net.const_val);
      if (w.best <= NEG_CUT && !w.use_inc) {
        fail(i, BBTN_E_INTERNAL, "no feasible configuration found");
        continue;
      }
      if (w.use_inc) {
        w.states.assign(insts[i].ls_x.begin(), insts[i].ls_x.end());
        continue;
      }
    } else if (w.best <= NEG_CUT) {
      fail(i, BBTN_E_INTERNAL, "no feasible configuration found");
      continue;
    }
    w.opt_sel.assign(w.groups.size(), {});
    uint64_t n_opt = 0;
    for (size_t gi = 0; gi < w.groups.size(); ++gi)
      for (int64_t l = 0; l < w.groups[gi].count; ++l)
        if (w.pv.val[gi][l] == w.best) {
          w.opt_sel[gi].push_back(l);
          ++n_opt;
          if (w.first.group < 0) w.first = LeafRef{(int32_t)gi, l};
        }
    if (!values_only) {
      w.stats.pruned += w.stats.leaves - n_opt;
      counting.push_back(i);
    }
    recover.push_back(i);
    ritems.push_back(RecoverItem{&insts[i].net, &W[i].tree, &w.groups[w.first.group], w.first.idx,
                                 &w.states});
  }
  const double t_values = now_s();
  // ---- one optimal configuration per instance, recovered on the second
  // context while this one runs the counting passes (no shared buffers)
  std::future<void> cfg_job;
  if (!ritems.empty()) {
    if (counting.empty()) {
      recover_configs(ctx, ritems);
    } else {
      bbtn_ctx* aux = aux_context(ctx);
      cfg_job = std::async(std::launch::async, [&ritems, aux] {
        BBTN_HIP(hipSetDevice(aux->opt.device));
        recover_configs(aux, ritems);
      });
    }
  }
  // ---- counting: k residues, plus, when k primes cannot certify by size
  // (a count never exceeds 2^n) and one more residue fits the entry, a
  // (k+1)-th prime in the same pass that checks the CRT value
  auto bits_of = [&](const std::vector<int>& ids) {
    double bits = 0;
    for (int id : ids) bits += std::log2((double)P[id]);
    return bits;
  };
  auto sum_into = [&](size_t i, const PassOut& o, const std::vector<int>& ids) {
    Work& w = W[i];
    for (size_t p = 0; p < ids.size(); ++p) {
      const uint32_t pr = P[ids[p]];
      uint32_t s = 0;
      for (size_t gi = 0; gi < w.groups.size(); ++gi)
        for (int64_t l : w.opt_sel[gi]) s = addmod(s, o.res[gi][p][l], pr);
      w.residues.push_back(mulmod(s, insts[i].net.const_res[ids[p]], pr));
    }
  };
  auto primes_of = [&](const std::vector<int>& ids, size_t n) {
    std::vector<uint32_t> pr;
    for (size_t j = 0; j < n; ++j) pr.push_back(P[ids[j]]);
    return pr;
  };
  // instances with the same prime list share a pass
  auto run_grouped = [&](const std::vector<size_t>& idx,
                         const std::vector<std::vector<int>>& lists, auto&& after) {
    std::vector<char> done(idx.size(), 0);
    for (size_t a = 0; a < idx.size(); ++a) {
      if (done[a]) continue;
      std::vector<size_t> same;
      for (size_t b = a; b < idx.size(); ++b)
        if (!done[b] && lists[b] == lists[a]) { same.push_back(idx[b]); done[b] = 1; }
      run_pass(ctx, pass_items(same, true, true), lists[a], opt.batched != 0);
      for (size_t i : same) after(i, lists[a]);
    }
  };
  {
    std::vector<std::vector<int>> lists;
    for (size_t i : counting) {
      Work& w = W[i];
      for (int p = 0; p < k; ++p) w.used.push_back(p);
      w.fused = bits_of(w.used) <= (double)insts[i].net.n + 1.0 && k < KMAX && max_primes > k;
      if (w.fused) w.used.push_back(k);
      lists.push_back(w.used);
    }
    run_grouped(counting, lists, [&](size_t i, const std::vector<int>& ids) {
      Work& w = W[i];
      for (size_t gi = 0; gi < w.groups.size(); ++gi)
        for (int64_t l : w.opt_sel[gi])
          if (w.pc.val[gi][l] != w.best)
            throw Error(BBTN_E_INTERNAL, "counting pass disagrees on a value");
      sum_into(i, w.pc, ids);
      if (w.fused) {
        // CRT over the first k primes, checked against the (k+1)-th
        const std::vector<uint32_t> first_k(w.residues.begin(), w.residues.begin() + k);
        w.count = crt_garner(first_k, primes_of(w.used, k));
        const bool agree = bigint_mod(w.count, P[w.used[k]]) == w.residues[k];
        w.count = crt_garner(w.residues, primes_of(w.used, w.used.size()));
        w.certified = agree ? 1 : 0;
      } else {
        w.count = crt_garner(w.residues, primes_of(w.used, w.used.size()));
      }
    });
  }
  const double t_counted = now_s();
  // ---- certification: by size, else one further prime must agree with the
  // CRT value; otherwise a pass of k more primes plus a check prime, until
  // max_primes
  for (;;) {
    std::vector<size_t> need;
    std::vector<std::vector<int>> one;
    for (size_t i : counting) {
      Work& w = W[i];
      if (w.certified) continue;
      if (bits_of(w.used) > (double)insts[i].net.n + 1.0) { w.certified = 1; continue; }
      const int nxt = (int)w.used.size();
      if (nxt >= max_primes) continue;
      need.push_back(i);
      one.push_back({nxt});
    }
    if (need.empty()) break;
    std::vector<size_t> more_idx;
    std::vector<std::vector<int>> more;
    run_grouped(need, one, [&](size_t i, const std::vector<int>& ids) {
      Work& w = W[i];
      const int nxt = ids[0];
      const uint32_t pq = P[nxt];
      uint32_t r = 0;
      for (size_t gi = 0; gi < w.groups.size(); ++gi)
        for (int64_t l : w.opt_sel[gi]) r = addmod(r, w.pc.res[gi][0][l], pq);
      r = mulmod(r, insts[i].net.const_res[nxt], pq);
      const bool agree = bigint_mod(w.count, pq) == r;
      w.used.push_back(nxt);
      w.residues.push_back(r);
      w.count = crt_garner(w.residues, primes_of(w.used, w.used.size()));
      if (agree) { w.certified = 1; return; }
      // k more primes, and one more in the same pass (when the entry has
      // room) that checks the CRT value of all the others: one pass instead
      // of a pass of k primes followed by a one-prime check pass
      std::vector<int> m;
      for (int p = 0; p < k + 1 && p < KMAX && (int)w.used.size() + p < max_primes; ++p)
        m.push_back((int)w.used.size() + p);
      if (!m.empty()) { more_idx.push_back(i); more.push_back(m); }
    });
    if (!more_idx.empty())
      run_grouped(more_idx, more, [&](size_t i, const std::vector<int>& ids) {
        Work& w = W[i];
        sum_into(i, w.pc, ids);
        for (int id : ids) w.used.push_back(id);
        if (ids.size() >= 2 && (int)ids.size() == std::min(k + 1, KMAX)) {
          const size_t nb = w.used.size() - 1;
          const std::vector<uint32_t> head(w.residues.begin(), w.residues.begin() + nb);
          const auto x = crt_garner(head, primes_of(w.used, nb));
          if (bigint_mod(x, P[w.used[nb]]) == w.residues[nb]) w.certified = 1;
        }
        w.count = crt_garner(w.residues, primes_of(w.used, w.used.size()));
      });
    bool progress = false;
    for (size_t i : need) progress |= W[i].certified || (int)W[i].used.size() < max_primes;
    if (!progress) break;
  }
  const double t_cert = now_s();
  // ---- configurations (wait for the recovery; rethrows its error)
  if (cfg_job.valid()) cfg_job.get();
  const double t_done = now_s();
  // ---- results
  for (size_t i = 0; i < N; ++i) {
    Instance& in = insts[i];
    Work& w = W[i];
    bbtn_result* res = in.res;
    res->seconds[1] = w.t_build;
    res->seconds[2] = w.t_search;
    res->leaves = w.stats.leaves;
    res->pruned = w.stats.pruned;
    res->nodes = w.stats.nodes;
    res->macs = ctx->last_macs;
    if (!w.active) continue;
    const Network& net = in.net;
    const int64_t value = w.use_inc ? w.incumbent : (int64_t)w.best + net.const_val;
    res->value = net.spin ? -value : value;
    res->seconds[3] = (t_values - t_planned) + (t_counted - t_values);
    res->seconds[7] = t_values - t_planned;
    res->seconds[4] = t_cert - t_counted;
    res->seconds[5] = t_done - t_cert;
    if (res->config)
      for (int v = 0; v < net.n; ++v)
        res->config[v] = net.spin ? (int8_t)(w.states[v] ? 1 : -1) : (int8_t)(w.states[v] ? 1 : 0);
    res->seconds[0] = now_s() - t0;
    if (values_only) {
      res->n_primes = 0;
      res->certified = 0;
      res->count_words = 0;
      if (res->count)
        for (int j = 0; j < res->count_capacity; ++j) res->count[j] = 0;
      continue;
    }
    res->n_primes = (int32_t)w.used.size();
    for (size_t j = 0; j < w.used.size(); ++j) {
      res->primes[j] = P[w.used[j]];
      res->residues[j] = w.residues[j];
    }
    res->certified = w.certified;
    res->count_words = (int32_t)w.count.size();
    if (res->count) {
      if (res->count_capacity < res->count_words) {
        fail(i, BBTN_E_BUFFER_TOO_SMALL, "count buffer too small");
        continue;
      }
      for (int j = 0; j < res->count_capacity; ++j)
        res->count[j] = j < (int)w.count.size() ? w.count[j] : 0;
    }
    if (!w.certified) fail(i, BBTN_E_COUNT_UNCERTIFIED, "count not certified within max_primes");
  }
  // the networks and pipeline state hold many small allocations; freeing
  // them on one thread costs as much as the rest of a large call's host
  // work, so they are freed on the planning threads
  parallel_for(N, (int)std::max(1u, std::thread::hardware_concurrency()), [&](size_t i) {
    insts[i].net = Network();
    insts[i].ls_x = std::vector<uint8_t>();
    W[i] = Work();
  });
}

int order_candidates(bbtn_ctx* ctx, const Network& net) {
  const auto shape = shape_of(net);
  {
    std::lock_guard<std::mutex> lk(ctx->tree_mu);
    auto it = ctx->order_cands.find(shape);
    if (it != ctx->order_cands.end()) return (int)it->second.size();
  }
  SearchOptions probe;
  probe.log2_target = ctx->opt.log2_target;
  probe.region_max = std::max(1, std::min(16, ctx->opt.region_max));
  probe.values_only = ctx->opt.residues_per_pass == 0;
  std::vector<Tree> ranked = rank_orders(net, std::max(1, ctx->opt.order_refine), probe);
  std::vector<std::shared_ptr<const Tree>> keep;
  for (Tree& t : ranked) keep.push_back(std::make_shared<const Tree>(std::move(t)));
  std::lock_guard<std::mutex> lk(ctx->tree_mu);
  if (ctx->order_cands.size() >= 8) ctx->order_cands.clear();
  return (int)ctx->order_cands.emplace(shape, std::move(keep)).first->second.size();
}

void order_use(bbtn_ctx* ctx, const Network& net, int which) {
  const auto shape = shape_of(net);
  std::lock_guard<std::mutex> lk(ctx->tree_mu);
  auto it = ctx->order_cands.find(shape);
  BBTN_REQUIRE(it != ctx->order_cands.end(), "no order candidates for this structure");
  BBTN_REQUIRE(which >= 0 && which < (int)it->second.size(), "order candidate out of range");
  ctx->tree_cache.erase(shape);
  if (ctx->tree_cache.size() >= 8) ctx->tree_cache.clear();
  ctx->tree_cache.emplace(shape, bbtn_ctx::TreeEntry{it->second[which], next_id++});
}

}  // namespace bbtn
