// C ABI of the library (include/bbtn.h) and the solve driver:
// build network -> contraction tree -> branch-and-bound search -> batched
// contraction of every branch sub-network per prime pass -> tropical sum of
// the branch results -> CRT + certification -> one optimal configuration.
#include <chrono>
#include <cmath>
#include <cstring>
#include <fstream>
#include <future>

#include "crt.h"
#include "ctx.h"
#include "exec.h"
#include "persist.h"
#include "scorer.h"
#include "search.h"
#include "trace.h"

using namespace bbtn;

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

template <class F>
bbtn_status guard(bbtn_ctx* ctx, F&& f) {
  try {
    f();
    if (ctx) ctx->err.clear();
    return BBTN_OK;
  } catch (const Error& e) {
    if (ctx) ctx->err = e.what();
    return e.status;
  } catch (const std::bad_alloc&) {
    if (ctx) ctx->err = "host allocation failed";
    return BBTN_E_OOM;
  } catch (const std::exception& e) {
    if (ctx) ctx->err = e.what();
    return BBTN_E_INTERNAL;
  }
}

// Kernel-level entry points run on the caller's stream; NULL is the null
// (default) stream, as everywhere in HIP.
hipStream_t pick_stream(bbtn_ctx*, void* s) { return (hipStream_t)s; }

// Leaves of the search in a flat order: (group, index in group).
struct LeafRef {
  int32_t group;
  int64_t idx;
};

// Per-branch results of one pass: value and k residues per leaf.
struct PassOut {
  std::vector<std::vector<int32_t>> val;             // [group][leaf]
  std::vector<std::vector<std::vector<uint32_t>>> res;  // [group][p][leaf]
};

int64_t leaves_per_chunk(bbtn_ctx* ctx, const GroupPlan& g, int k) {
  size_t freeb = 0, totalb = 0;
  if (hipMemGetInfo(&freeb, &totalb) != hipSuccess) freeb = (size_t)8 << 30;
  const double budget = 0.45 * (double)(freeb + ctx->work.bytes);
  const double per = (double)(1 + k) * 4.0 * (double)std::max<int64_t>(g.peak, 1) * 1.05 +
                     (double)(1 + k) * 12.0 + 8.0 * (double)(g.base_ops.size() + 1);
  int64_t L = (int64_t)(budget / per);
  return std::max<int64_t>(1, std::min<int64_t>(L, 1 << 20));
}

// Run pass with primes pidx[0..k) over the selected leaves of every group.
// sel[g] lists leaf indices (ascending) to run for group g.
void run_pass(bbtn_ctx* ctx, const Network& net, const std::vector<LeafGroup>& groups,
              std::vector<GroupPlan>& plans, const std::vector<std::vector<int64_t>>& sel,
              const std::vector<int>& pidx, PassOut& out, bool batched) {
  const int k = (int)pidx.size();
  hipStream_t st = ctx->stream;
  std::vector<uint32_t> primes(k);
  for (int p = 0; p < k; ++p) primes[p] = prime_table()[pidx[p]];
  const Moduli mod = make_moduli(k, primes.data());
  BaseDev bd;
  upload_base(ctx, net, pidx.data(), k, bd, ctx->base);
  out.val.assign(groups.size(), {});
  out.res.assign(groups.size(), {});
  // the selected branches of every group, packed per group
  std::vector<std::vector<uint8_t>> asg(groups.size());
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const LeafGroup& G = groups[gi];
    out.val[gi].assign(G.count, NEG);
    out.res[gi].assign(k, std::vector<uint32_t>(G.count, 0));
    const size_t S = G.vars.size();
    asg[gi].resize(sel[gi].size() * S);
    for (size_t i = 0; i < sel[gi].size(); ++i)
      std::memcpy(&asg[gi][i * S], &G.assign[sel[gi][i] * S], S);
  }
  auto scatter = [&](size_t gi, size_t c0, int64_t L, const uint32_t* h) {
    for (int64_t i = 0; i < L; ++i) {
      const int64_t leaf = sel[gi][c0 + i];
      out.val[gi][leaf] = (int32_t)h[i];
      for (int p = 0; p < k; ++p) out.res[gi][p][leaf] = h[(size_t)(p + 1) * L + i];
    }
  };
  // groups whose operands fit in LDS: one persistent launch for all of them
  std::vector<PersistJob> jobs;
  std::vector<size_t> job_group;
  std::vector<std::vector<uint32_t>> job_out(groups.size());
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    if (!batched || sel[gi].empty() || !persist_fits(plans[gi], k)) continue;
    jobs.push_back(PersistJob{&plans[gi], asg[gi].data(), (int64_t)sel[gi].size(), &job_out[gi]});
    job_group.push_back(gi);
  }
  if (!jobs.empty()) {
    run_persistent(ctx, net, jobs, bd, mod, st);
    for (size_t j = 0; j < jobs.size(); ++j)
      scatter(job_group[j], 0, jobs[j].L, job_out[job_group[j]].data());
  }
  // the rest: step by step, batched over the group's branches (chunked by
  // memory), or one branch at a time when batching is off
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    if (sel[gi].empty()) continue;
    if (batched && persist_fits(plans[gi], k)) continue;
    const GroupPlan& g = plans[gi];
    const size_t S = groups[gi].vars.size();
    const int64_t chunk = batched ? leaves_per_chunk(ctx, g, k) : 1;
    for (size_t c0 = 0; c0 < sel[gi].size(); c0 += chunk) {
      const int64_t L = std::min<int64_t>(chunk, (int64_t)(sel[gi].size() - c0));
      ctx->leafout.ensure((size_t)(1 + k) * L * 4);
      const DevTensor o{ctx->leafout.as<uint32_t>(), L};
      run_group(ctx, net, g, bd, mod, &asg[gi][c0 * S], L, o, st,
                /*reuse=*/sel[gi].size() > (size_t)chunk);
      std::vector<uint32_t> h((size_t)(1 + k) * L);
      BBTN_HIP(hipMemcpyAsync(h.data(), o.ptr, h.size() * 4, hipMemcpyDeviceToHost, st));
      BBTN_HIP(hipStreamSynchronize(st));
      ctx->prof.resolve();
      scatter(gi, c0, L, h.data());
    }
  }
}

// Recover an optimal configuration from the winning leaf.
void recover_config(bbtn_ctx* ctx, const Network& net, const Tree& tree, const LeafGroup& G,
                    int64_t leaf, std::vector<int8_t>& states) {
  hipStream_t st = ctx->stream;
  states.assign(net.n, -1);
  for (size_t j = 0; j < G.vars.size(); ++j) states[G.vars[j]] = (int8_t)G.assign[leaf * G.vars.size() + j];
  GroupPlan g = build_plan(net, tree, G.mask, /*keep_all=*/true);
  if (!g.steps.empty()) {
    const int pidx0 = 0;
    BaseDev bd;
    upload_base(ctx, net, &pidx0, 0, bd, ctx->base);
    const Moduli mod = make_moduli(0, nullptr);
    ctx->leafout.ensure(64);
    const DevTensor o{ctx->leafout.as<uint32_t>(), 1};
    const uint64_t macs0 = ctx->last_macs;
    if (ctx->opt.batched && persist_fits(g, 0)) {
      // one persistent launch (one workgroup: its scratch starts at the
      // workspace base, where the traceback reads)
      std::vector<uint32_t> tmp;
      std::vector<PersistJob> jobs{PersistJob{&g, &G.assign[leaf * G.vars.size()], 1, &tmp}};
      run_persistent(ctx, net, jobs, bd, mod, st);
    } else {
      run_group(ctx, net, g, bd, mod, &G.assign[leaf * G.vars.size()], 1, o, st);
    }
    ctx->last_macs = macs0;  // bookkeeping counts the counting passes only
    // traceback program
    std::vector<TraceStep> ts;
    std::vector<int32_t> vars;
    for (const Step& s : g.steps) {
      TraceStep t{};
      t.rb = s.rb; t.rm = s.rm; t.rn = s.rn; t.rk = s.rk;
      t.a_off = g.buf_off[s.a.direct ? s.a.id : s.a.temp];
      t.b_off = g.buf_off[s.b.direct ? s.b.id : s.b.temp];
      t.var_off = (int32_t)vars.size();
      vars.insert(vars.end(), s.a_vars.begin(), s.a_vars.end());
      vars.insert(vars.end(), s.b_vars.begin(), s.b_vars.end());
      ts.push_back(t);
    }
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t bytes_ts = ts.size() * sizeof(TraceStep);
    const size_t off_v = al(bytes_ts);
    const size_t off_a = off_v + al(std::max<size_t>(vars.size(), 1) * 4);
    const size_t off_s = off_a + al((size_t)net.n);
    ctx->misc.ensure(off_s + 256);
    char* base = ctx->misc.as<char>();
    TraceStep* dts = (TraceStep*)base;
    int32_t* dvars = (int32_t*)(base + off_v);
    int8_t* dasg = (int8_t*)(base + off_a);
    int32_t* dstat = (int32_t*)(base + off_s);
    BBTN_HIP(hipMemcpyAsync(dts, ts.data(), bytes_ts, hipMemcpyHostToDevice, st));
    BBTN_HIP(hipMemcpyAsync(dvars, vars.data(), vars.size() * 4, hipMemcpyHostToDevice, st));
    BBTN_HIP(hipMemcpyAsync(dasg, states.data(), net.n, hipMemcpyHostToDevice, st));
    const int32_t zero = 0;
    BBTN_HIP(hipMemcpyAsync(dstat, &zero, 4, hipMemcpyHostToDevice, st));
    launch_trace(dts, (int32_t)ts.size(), dvars, (int32_t)vars.size(), ctx->work.as<int32_t>(),
                 dasg, net.n, dstat, st);
    int32_t stat = 0;
    BBTN_HIP(hipMemcpyAsync(states.data(), dasg, net.n, hipMemcpyDeviceToHost, st));
    BBTN_HIP(hipMemcpyAsync(&stat, dstat, 4, hipMemcpyDeviceToHost, st));
    BBTN_HIP(hipStreamSynchronize(st));
    if (stat) throw Error(BBTN_E_INTERNAL, "configuration traceback failed");
  }
  // variables eliminated while simplifying, in reverse order
  for (size_t i = net.peel.size(); i-- > 0;) {
    const PeelRec& r = net.peel[i];
    int64_t base = 0;
    int pos = -1;
    for (size_t j = 0; j < r.tvars.size(); ++j) {
      if (r.tvars[j] == r.var) { pos = (int)j; continue; }
      base |= (int64_t)(states[r.tvars[j]] & 1) << j;
    }
    const int32_t v0 = r.tval[base], v1 = r.tval[base | (1ll << pos)];
    const bool f0 = v0 > NEG_CUT, f1 = v1 > NEG_CUT;
    states[r.var] = (f1 && (!f0 || v1 > v0)) ? 1 : 0;
  }
  for (int v = 0; v < net.n; ++v)
    if (states[v] < 0) states[v] = 0;  // variable in no tensor at all
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
    ctx->aux = a;
  }
  ctx->aux->tune = ctx->tune;
  return ctx->aux;
}

void solve_network(bbtn_ctx* ctx, Network& net, const std::vector<uint8_t>& ls_x,
                   bbtn_result* res) {
  const double t0 = now_s();
  const bbtn_options& opt = ctx->opt;
  ctx->last_macs = 0;
  ctx->clear_graphs();  // captured programs refer to the previous solve's plans
  struct GraphScope {
    bbtn_ctx* c;
    ~GraphScope() { c->clear_graphs(); }
  } graph_scope{ctx};
  for (int i = 0; i < 8; ++i) res->seconds[i] = 0;
  const double deadline = opt.time_limit_s > 0 ? t0 + opt.time_limit_s : 0;
  Tree tree;
  {
    std::vector<std::vector<int32_t>> shape;
    shape.reserve(net.tensors.size() + 1);
    shape.push_back({net.n});
    for (const auto& T : net.tensors) shape.push_back(T.vars);
    auto it = ctx->tree_cache.find(shape);
    if (it != ctx->tree_cache.end()) {
      tree = it->second;
    } else {
      tree = greedy_tree(net);
      if (ctx->tree_cache.size() >= 8) ctx->tree_cache.clear();
      ctx->tree_cache.emplace(std::move(shape), tree);
    }
  }
  // search
  const double t1 = now_s();
  std::vector<LeafGroup> groups;
  SearchStats stats;
  const bool branch = opt.branching != 0 && opt.log2_target > 0;
  const bool values_only = opt.residues_per_pass == 0;
  // value (with the folded constant, like node_bound) of the local-search
  // configuration: a lower bound on the optimum, used for global pruning
  const int64_t incumbent = ls_x.empty() ? INT64_MIN : network_value(net, ls_x);
  if (!branch) {
    LeafGroup g;
    g.mask.assign((net.n + 63) / 64, 0);
    g.count = 1;
    groups.push_back(g);
    stats.leaves = 1;
  } else {
    SearchOptions so;
    so.log2_target = opt.log2_target;
    so.region_max = std::max(1, std::min(16, opt.region_max));
    so.incumbent = incumbent;
    so.values_only = values_only;
    so.deadline = deadline;
    if (opt.branching == 2 && ctx->scorer_loaded) so.scorer = make_var_scorer(ctx, net, tree, opt.log2_target);
    bb_search(net, tree, so, groups, stats);
  }
  const double t2 = now_s();
  // plans
  std::vector<GroupPlan> plans;
  for (auto& G : groups) plans.push_back(build_plan(net, tree, G.mask, false));
  const double t3 = now_s();
  res->seconds[1] = (t1 - t0) + (t3 - t2);
  res->seconds[2] = t2 - t1;
  // Values-only pass over every leaf (the max-plus part of the algebra):
  // its exact values give the optimum, and a leaf whose value is below it
  // can contribute no count (global pruning with the exact incumbent), so
  // the counting passes below touch only the leaves reaching the optimum.
  const auto& P = prime_table();
  const int k = values_only ? 0 : std::max(1, std::min(KMAX, opt.residues_per_pass));
  const int max_primes = std::max(k, std::min(BBTN_MAX_PRIMES, opt.max_primes));
  std::vector<std::vector<int64_t>> sel(groups.size());
  for (size_t gi = 0; gi < groups.size(); ++gi)
    for (int64_t i = 0; i < groups[gi].count; ++i) sel[gi].push_back(i);
  PassOut pv;
  run_pass(ctx, net, groups, plans, sel, {}, pv, opt.batched != 0);
  if (deadline > 0 && now_s() > deadline) throw Error(BBTN_E_TIMEOUT, "time limit reached");
  int32_t best = NEG;
  for (auto& gv : pv.val)
    for (int32_t v : gv)
      if (v > NEG_CUT && v > best) best = v;
  if (values_only) {
    // the optimum is the best leaf or, when the search pruned everything
    // that could not beat it, the incumbent itself
    const bool use_inc = incumbent != INT64_MIN &&
                         (best <= NEG_CUT || incumbent > (int64_t)best + net.const_val);
    if (best <= NEG_CUT && !use_inc) throw Error(BBTN_E_INTERNAL, "no feasible configuration found");
    std::vector<int8_t> states;
    if (use_inc) {
      states.assign(ls_x.begin(), ls_x.end());
    } else {
      LeafRef first{-1, -1};
      for (size_t gi = 0; gi < groups.size() && first.group < 0; ++gi)
        for (int64_t i = 0; i < groups[gi].count; ++i)
          if (pv.val[gi][i] == best) { first = LeafRef{(int32_t)gi, i}; break; }
      recover_config(ctx, net, tree, groups[first.group], first.idx, states);
    }
    const double t6 = now_s();
    res->seconds[5] = t6 - t3;
    const int64_t value = use_inc ? incumbent : (int64_t)best + net.const_val;
    res->value = net.spin ? -value : value;
    res->n_primes = 0;
    res->certified = 0;
    res->count_words = 0;
    res->leaves = stats.leaves;
    res->pruned = stats.pruned;
    res->nodes = stats.nodes;
    res->macs = ctx->last_macs;
    if (res->config)
      for (int v = 0; v < net.n; ++v)
        res->config[v] = net.spin ? (int8_t)(states[v] ? 1 : -1) : (int8_t)(states[v] ? 1 : 0);
    if (res->count)
      for (int i = 0; i < res->count_capacity; ++i) res->count[i] = 0;
    res->seconds[0] = now_s() - t0;
    return;
  }
  if (best <= NEG_CUT) throw Error(BBTN_E_INTERNAL, "no feasible configuration found");
  std::vector<std::vector<int64_t>> opt_sel(groups.size());
  LeafRef first{-1, -1};
  uint64_t n_opt = 0;
  for (size_t gi = 0; gi < groups.size(); ++gi)
    for (int64_t i = 0; i < groups[gi].count; ++i)
      if (pv.val[gi][i] == best) {
        opt_sel[gi].push_back(i);
        ++n_opt;
        if (first.group < 0) first = LeafRef{(int32_t)gi, i};
      }
  stats.pruned += stats.leaves - n_opt;
  // one optimal configuration, recovered on the second context while this
  // one runs the counting passes (they share no device buffers)
  std::vector<int8_t> states;
  bbtn_ctx* aux = aux_context(ctx);
  std::future<void> cfg_job = std::async(std::launch::async, [&, aux] {
    BBTN_HIP(hipSetDevice(aux->opt.device));
    recover_config(aux, net, tree, groups[first.group], first.idx, states);
  });
  // certification: a count never exceeds 2^n (the number of configurations)
  auto bits_of = [&](const std::vector<int>& ids) {
    double bits = 0;
    for (int id : ids) bits += std::log2((double)P[id]);
    return bits;
  };
  const double need_bits = (double)net.n + 1.0;
  // first counting pass over the optimal leaves: k residues, plus, when k
  // primes cannot certify by size and one more residue fits the entry, a
  // (k+1)-th prime in the same pass that checks the CRT value
  std::vector<int> used;
  for (int p = 0; p < k; ++p) used.push_back(p);
  const bool fused_check = bits_of(used) <= need_bits && k < KMAX && max_primes > k;
  if (fused_check) used.push_back(k);
  PassOut po;
  run_pass(ctx, net, groups, plans, opt_sel, used, po, opt.batched != 0);
  for (size_t gi = 0; gi < groups.size(); ++gi)
    for (int64_t i : opt_sel[gi])
      if (po.val[gi][i] != best) throw Error(BBTN_E_INTERNAL, "counting pass disagrees on a value");
  std::vector<uint32_t> residues;  // aligned with `used`
  auto sum_pass = [&](const PassOut& o, const std::vector<int>& ids) {
    for (size_t p = 0; p < ids.size(); ++p) {
      const uint32_t pr = P[ids[p]];
      uint32_t s = 0;
      for (size_t gi = 0; gi < groups.size(); ++gi)
        for (int64_t i : opt_sel[gi]) s = addmod(s, o.res[gi][p][i], pr);
      residues.push_back(mulmod(s, net.const_res[ids[p]], pr));
    }
  };
  sum_pass(po, used);
  const double t4 = now_s();
  res->seconds[3] = t4 - t3;
  std::vector<uint32_t> pr_used;
  auto primes_of = [&](size_t count_of) {
    pr_used.clear();
    for (size_t i = 0; i < count_of; ++i) pr_used.push_back(P[used[i]]);
    return pr_used;
  };
  int certified = 0;
  std::vector<uint32_t> count;
  if (fused_check) {
    // CRT over the first k primes, checked against the (k+1)-th
    const std::vector<uint32_t> first_k(residues.begin(), residues.begin() + k);
    count = crt_garner(first_k, primes_of(k));
    const bool agree = bigint_mod(count, P[used[k]]) == residues[k];
    count = crt_garner(residues, primes_of(used.size()));
    certified = agree ? 1 : 0;
  } else {
    count = crt_garner(residues, primes_of(used.size()));
  }
  while (!certified) {
    if (bits_of(used) > need_bits) { certified = 1; break; }
    const int nxt = (int)used.size();
    if (nxt >= max_primes) break;
    // one extra prime over the optimal leaves only
    std::vector<int> one{nxt};
    PassOut pc;
    run_pass(ctx, net, groups, plans, opt_sel, one, pc, opt.batched != 0);
    const uint32_t pq = P[nxt];
    uint32_t r = 0;
    for (size_t gi = 0; gi < groups.size(); ++gi)
      for (int64_t i : opt_sel[gi]) r = addmod(r, pc.res[gi][0][i], pq);
    r = mulmod(r, net.const_res[nxt], pq);
    const bool agree = bigint_mod(count, pq) == r;
    used.push_back(nxt);
    residues.push_back(r);
    count = crt_garner(residues, primes_of(used.size()));
    if (agree) { certified = 1; break; }
    // not yet: add a full pass of k primes
    std::vector<int> more;
    for (int p = 0; p < k && (int)used.size() + p < max_primes; ++p) more.push_back((int)used.size() + p);
    if (more.empty()) break;
    PassOut pm;
    run_pass(ctx, net, groups, plans, opt_sel, more, pm, opt.batched != 0);
    sum_pass(pm, more);
    for (int id : more) used.push_back(id);
    count = crt_garner(residues, primes_of(used.size()));
  }
  const double t5 = now_s();
  res->seconds[4] = t5 - t4;
  // configuration (waits for the recovery; rethrows its error)
  cfg_job.get();
  const double t6 = now_s();
  res->seconds[5] = t6 - t5;
  // fill the result
  const int64_t value = (int64_t)best + net.const_val;
  res->value = net.spin ? -value : value;
  res->n_primes = (int32_t)used.size();
  for (size_t i = 0; i < used.size(); ++i) {
    res->primes[i] = P[used[i]];
    res->residues[i] = residues[i];
  }
  res->certified = certified;
  res->count_words = (int32_t)count.size();
  res->leaves = stats.leaves;
  res->pruned = stats.pruned;
  res->nodes = stats.nodes;
  res->macs = ctx->last_macs;
  if (res->config)
    for (int v = 0; v < net.n; ++v)
      res->config[v] = net.spin ? (int8_t)(states[v] ? 1 : -1) : (int8_t)(states[v] ? 1 : 0);
  res->seconds[0] = now_s() - t0;
  if (res->count) {
    if (res->count_capacity < res->count_words)
      throw Error(BBTN_E_BUFFER_TOO_SMALL, "count buffer too small");
    for (int i = 0; i < res->count_capacity; ++i) res->count[i] = i < (int)count.size() ? count[i] : 0;
  }
  if (!certified) throw Error(BBTN_E_COUNT_UNCERTIFIED, "count not certified within max_primes");
}

void check_graph(int32_t n, int32_t m, const int32_t* uv) {
  BBTN_REQUIRE(n >= 1 && n <= (1 << 22), "n out of range");
  BBTN_REQUIRE(m >= 0, "m out of range");
  BBTN_REQUIRE(m == 0 || uv != nullptr, "edge list is NULL");
}

}  // namespace

extern "C" {

void bbtn_default_options(bbtn_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->device = 0;
  o->residues_per_pass = 3;
  o->max_primes = 16;
  o->log2_target = 0;
  o->branching = 1;
  o->batched = 1;
  o->region_max = 8;
  o->local_search = 100;
  o->graphs = 1;
  o->scorer_weights = nullptr;
  o->autotune_cache = nullptr;
  o->time_limit_s = 0;
  o->stream = nullptr;
}

bbtn_status bbtn_create(const bbtn_options* opt, bbtn_ctx** out) {
  if (!out) return BBTN_E_INVALID_ARG;
  *out = nullptr;
  bbtn_ctx* ctx = new (std::nothrow) bbtn_ctx();
  if (!ctx) return BBTN_E_OOM;
  if (opt) ctx->opt = *opt; else bbtn_default_options(&ctx->opt);
  bbtn_status s = guard(ctx, [&] {
    BBTN_REQUIRE(ctx->opt.residues_per_pass >= 0 && ctx->opt.residues_per_pass <= KMAX,
                 "residues_per_pass must be in [0, 4]");
    int ndev = 0;
    BBTN_HIP(hipGetDeviceCount(&ndev));
    BBTN_REQUIRE(ctx->opt.device >= 0 && ctx->opt.device < ndev, "no such device");
    BBTN_HIP(hipSetDevice(ctx->opt.device));
    if (ctx->opt.stream) {
      ctx->stream = (hipStream_t)ctx->opt.stream;
    } else {
      BBTN_HIP(hipStreamCreateWithFlags(&ctx->own, hipStreamNonBlocking));
      ctx->stream = ctx->own;
    }
    (void)prime_table();
    if (ctx->opt.autotune_cache) load_tune_cache(ctx, ctx->opt.autotune_cache);
    if (ctx->opt.scorer_weights) load_scorer(ctx, ctx->opt.scorer_weights);
  });
  if (s != BBTN_OK) {
    bbtn_destroy(ctx);
    return s;
  }
  *out = ctx;
  return BBTN_OK;
}

void bbtn_destroy(bbtn_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->opt.device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  ctx->work.release();
  ctx->shared_ws.release();
  ctx->partial.release();
  ctx->base.release();
  ctx->fixbits.release();
  ctx->leafconst.release();
  ctx->leafout.release();
  ctx->misc.release();
  ctx->persist.release();
  ctx->clear_graphs();
  if (ctx->own) (void)hipStreamDestroy(ctx->own);
  bbtn_destroy(ctx->aux);
  delete ctx;
}

const char* bbtn_last_error(const bbtn_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

uint64_t bbtn_last_macs(const bbtn_ctx* ctx) { return ctx ? ctx->last_macs : 0; }

bbtn_status bbtn_profile(bbtn_ctx* ctx, int32_t enable) {
  if (!ctx) return BBTN_E_INVALID_ARG;
  return guard(ctx, [&] {
    BBTN_HIP(hipSetDevice(ctx->opt.device));
    ctx->prof.clear();
    ctx->prof.on = enable != 0;
  });
}

bbtn_status bbtn_get_kernel_stats(bbtn_ctx* ctx, int32_t kernel, bbtn_kernel_stats* out) {
  if (!ctx || !out) return BBTN_E_INVALID_ARG;
  return guard(ctx, [&] {
    BBTN_REQUIRE(kernel >= 0 && kernel < K_COUNT, "unknown kernel id");
    BBTN_HIP(hipSetDevice(ctx->opt.device));
    ctx->prof.resolve();
    const KStat& s = ctx->prof.stat[kernel];
    out->launches = s.launches;
    out->seconds = s.seconds;
    out->ops = s.ops;
    out->bytes = s.bytes;
  });
}

bbtn_status bbtn_solve_spinglass(bbtn_ctx* ctx, int32_t n, int32_t m, const int32_t* edge_uv,
                                 const int32_t* J, const int32_t* h, bbtn_result* res) {
  if (!ctx || !res) return BBTN_E_INVALID_ARG;
  return guard(ctx, [&] {
    check_graph(n, m, edge_uv);
    BBTN_REQUIRE(m == 0 || J != nullptr, "J is NULL");
    BBTN_HIP(hipSetDevice(ctx->opt.device));
    Network net = build_spinglass(n, m, edge_uv, J, h);
    std::vector<uint8_t> x;
    if (ctx->opt.local_search > 0)
      x = local_search_spinglass(n, m, edge_uv, J, h, ctx->opt.local_search, 12345);
    solve_network(ctx, net, x, res);
  });
}

bbtn_status bbtn_solve_mwis(bbtn_ctx* ctx, int32_t n, int32_t m, const int32_t* edge_uv,
                            const int32_t* w, bbtn_result* res) {
  if (!ctx || !res) return BBTN_E_INVALID_ARG;
  return guard(ctx, [&] {
    check_graph(n, m, edge_uv);
    BBTN_HIP(hipSetDevice(ctx->opt.device));
    Network net = build_mwis(n, m, edge_uv, w);
    std::vector<uint8_t> x;
    if (ctx->opt.local_search > 0)
      x = local_search_mwis(n, m, edge_uv, w, std::max(1, ctx->opt.local_search / 20), 12345);
    solve_network(ctx, net, x, res);
  });
}

bbtn_status bbtn_tgemm(bbtn_ctx* ctx, int32_t k, const uint32_t* primes, int64_t batch, int64_t M,
                       int64_t N, int64_t K, const void* A, const void* B, void* C, void* stream) {
  if (!ctx) return BBTN_E_INVALID_ARG;
  return guard(ctx, [&] {
    BBTN_REQUIRE(k >= 1 && k <= KMAX, "k must be in [1, 4]");
    BBTN_REQUIRE(primes != nullptr, "primes is NULL");
    BBTN_REQUIRE(batch >= 1 && M >= 1 && N >= 1 && K >= 1, "empty product");
    BBTN_REQUIRE(A && B && C, "NULL operand");
    BBTN_REQUIRE(batch * M * K < (1ll << 40) && batch * K * N < (1ll << 40) &&
                     batch * M * N < (1ll << 40), "operand too large");
    BBTN_HIP(hipSetDevice(ctx->opt.device));
    const Moduli mod = make_moduli(k, primes);
    const TuneVal tv = choose_tiles(ctx, k, batch, M, N, K);
    DevTensor part{};
    if (tv.splits > 1) {
      const int64_t ent = (int64_t)tv.splits * batch * M * N;
      ctx->partial.ensure((size_t)(1 + k) * ent * 4);
      part = DevTensor{ctx->partial.as<uint32_t>(), ent};
    }
    GemmShape sh{batch, M, N, K, M * K, K * N, M * N};
    hipStream_t st = pick_stream(ctx, stream);
    const int ph = ctx->prof.begin(st);
    launch_tgemm(k, mod, sh, DevTensor{(uint32_t*)A, batch * M * K},
                 DevTensor{(uint32_t*)B, batch * K * N}, DevTensor{(uint32_t*)C, batch * M * N},
                 tv.cfg, tv.splits, part, st);
    ctx->prof.end(ph, st, K_TGEMM, (double)batch * M * N * K * (2 + 2 * k),
                  (double)(1 + k) * 4 * (double)batch * (double)(M * K + K * N + M * N));
  });
}

bbtn_status bbtn_gather(bbtn_ctx* ctx, int32_t k, int32_t r_in, int32_t r_out,
                        const int32_t* src_bits, int64_t L, int64_t in_stride,
                        const uint64_t* fixed_bits, const void* in, int64_t in_entries, void* out,
                        void* stream) {
  if (!ctx) return BBTN_E_INVALID_ARG;
  return guard(ctx, [&] {
    BBTN_REQUIRE(k >= 0 && k <= KMAX, "k must be in [0, 4]");
    BBTN_REQUIRE(L >= 1 && in && out, "bad gather arguments");
    BBTN_REQUIRE(r_out == 0 || src_bits != nullptr, "src_bits is NULL");
    BBTN_REQUIRE(r_in <= 36, "r_in too large");
    const int64_t sz = 1ll << r_in;
    BBTN_REQUIRE(in_stride == 0 || in_stride == sz, "in_stride must be 0 or 2^r_in");
    BBTN_REQUIRE(in_entries >= (in_stride == 0 ? sz : L * sz), "input buffer too small");
    BBTN_HIP(hipSetDevice(ctx->opt.device));
    const GatherPlan gp = make_gather_plan(r_in, r_out, src_bits);
    launch_gather(k, gp, L, in_stride, fixed_bits, DevTensor{(uint32_t*)in, in_entries},
                  DevTensor{(uint32_t*)out, L << r_out}, pick_stream(ctx, stream));
  });
}

bbtn_status bbtn_reduce(bbtn_ctx* ctx, int32_t k, const uint32_t* primes, int64_t outer,
                        int64_t S, int64_t seg_stride, int64_t elem_stride, const void* in,
                        int64_t in_entries, void* out, void* stream) {
  if (!ctx) return BBTN_E_INVALID_ARG;
  return guard(ctx, [&] {
    BBTN_REQUIRE(k >= 1 && k <= KMAX, "k must be in [1, 4]");
    BBTN_REQUIRE(primes && in && out, "NULL argument");
    BBTN_REQUIRE(outer >= 1 && S >= 1 && seg_stride >= 0 && elem_stride >= 0, "bad sizes");
    BBTN_REQUIRE((S - 1) * seg_stride + (outer - 1) * elem_stride < in_entries,
                 "input buffer too small");
    BBTN_HIP(hipSetDevice(ctx->opt.device));
    const Moduli mod = make_moduli(k, primes);
    launch_reduce(k, mod, outer, S, seg_stride, elem_stride, DevTensor{(uint32_t*)in, in_entries},
                  DevTensor{(uint32_t*)out, outer}, pick_stream(ctx, stream));
  });
}

bbtn_status bbtn_bound(bbtn_ctx* ctx, int64_t n_branch, int32_t tensors_per_branch,
                       const int32_t* values, const int64_t* tensor_off, const int32_t* tensor_len,
                       const int64_t* offset, int64_t incumbent, int64_t* bound,
                       int32_t* keep_idx, int32_t* n_keep, void* stream) {
  if (!ctx) return BBTN_E_INVALID_ARG;
  return guard(ctx, [&] {
    BBTN_REQUIRE(n_branch >= 0 && tensors_per_branch >= 0, "bad sizes");
    BBTN_REQUIRE(n_keep && (n_branch == 0 || (values && tensor_off && tensor_len && offset &&
                                              bound && keep_idx)), "NULL argument");
    BBTN_HIP(hipSetDevice(ctx->opt.device));
    ctx->misc.ensure((size_t)std::max<int64_t>(n_branch, 1) * 4);
    launch_bound(n_branch, tensors_per_branch, values, tensor_off, tensor_len, offset, incumbent,
                 bound, ctx->misc.as<int32_t>(), keep_idx, n_keep, pick_stream(ctx, stream));
  });
}

}  // extern "C"

// ------------------------------------------------------------------ scorer
#include <random>

#include "mlp.h"

extern "C" {

bbtn_status bbtn_mlp_forward(bbtn_ctx* ctx, int64_t rows, const uint16_t* X, const uint16_t* W,
                             const float* bias, float* y, float* h1, float* h2, void* stream) {
  if (!ctx) return BBTN_E_INVALID_ARG;
  return guard(ctx, [&] {
    BBTN_REQUIRE(rows >= 0 && (rows == 0 || (X && W && bias && y)), "bad arguments");
    BBTN_REQUIRE((h1 == nullptr) == (h2 == nullptr), "h1 and h2 go together");
    BBTN_HIP(hipSetDevice(ctx->opt.device));
    launch_mlp_forward(rows, X, W, bias, y, h1, h2, pick_stream(ctx, stream));
  });
}

bbtn_status bbtn_mlp_backward(bbtn_ctx* ctx, int64_t rows, const uint16_t* X, const uint16_t* W,
                              const float* y, const float* t, const float* h1, const float* h2,
                              float* grad, void* stream) {
  if (!ctx) return BBTN_E_INVALID_ARG;
  return guard(ctx, [&] {
    BBTN_REQUIRE(rows >= 1 && X && W && y && t && h1 && h2 && grad, "bad arguments");
    BBTN_HIP(hipSetDevice(ctx->opt.device));
    ctx->partial.ensure((size_t)mlp_partial_floats(rows) * 4);
    launch_mlp_backward(rows, X, W, y, t, h1, h2, ctx->partial.as<float>(), grad,
                        pick_stream(ctx, stream));
  });
}

bbtn_status bbtn_mlp_adam(bbtn_ctx* ctx, float* master, uint16_t* wbf, float* bias, float* m,
                          float* v, const float* grad, float lr, float beta1, float beta2,
                          float eps, int32_t step, void* stream) {
  if (!ctx) return BBTN_E_INVALID_ARG;
  return guard(ctx, [&] {
    BBTN_REQUIRE(master && wbf && bias && m && v && grad && step >= 1, "bad arguments");
    BBTN_HIP(hipSetDevice(ctx->opt.device));
    launch_mlp_adam(master, wbf, bias, m, v, grad, lr, beta1, beta2, eps, step,
                    pick_stream(ctx, stream));
  });
}

bbtn_status bbtn_scorer_load(bbtn_ctx* ctx, const char* path) {
  if (!ctx || !path) return BBTN_E_INVALID_ARG;
  return guard(ctx, [&] {
    BBTN_HIP(hipSetDevice(ctx->opt.device));
    load_scorer(ctx, path);
  });
}

bbtn_status bbtn_plan_leaves(bbtn_ctx* ctx, int32_t kind, int32_t n, int32_t m,
                             const int32_t* edge_uv, const int32_t* weights, const int32_t* h,
                             int32_t log2_target, int32_t region_max, int32_t local_search,
                             int32_t values_only, int8_t* leaves, int64_t capacity,
                             int64_t* n_leaves, int64_t* incumbent) {
  if (!n_leaves || !incumbent) return BBTN_E_INVALID_ARG;
  return guard(ctx, [&] {  // host-only: ctx may be NULL
    check_graph(n, m, edge_uv);
    BBTN_REQUIRE(kind == 0 || kind == 1, "kind must be 0 (spin glass) or 1 (MWIS)");
    BBTN_REQUIRE(log2_target > 0 && region_max >= 1 && local_search >= 0, "bad options");
    if (kind == 0) BBTN_REQUIRE(weights != nullptr, "J is NULL");
    Network net = kind == 0 ? build_spinglass(n, m, edge_uv, weights, h)
                            : build_mwis(n, m, edge_uv, weights);
    Tree tree = greedy_tree(net);
    std::vector<uint8_t> x;
    if (local_search > 0)
      x = kind == 0 ? local_search_spinglass(n, m, edge_uv, weights, h, local_search, 12345)
                    : local_search_mwis(n, m, edge_uv, weights, std::max(1, local_search / 20), 12345);
    SearchOptions so;
    so.log2_target = log2_target;
    so.region_max = std::min(16, region_max);
    so.incumbent = x.empty() ? INT64_MIN : network_value(net, x);
    so.values_only = values_only != 0;
    std::vector<LeafGroup> groups;
    SearchStats stats;
    bb_search(net, tree, so, groups, stats);
    int64_t total = 0;
    for (const auto& g : groups) total += g.count;
    *n_leaves = total;
    *incumbent = so.incumbent == INT64_MIN ? INT64_MIN
                 : (net.spin ? -so.incumbent : so.incumbent);
    if (!leaves) return;
    if (capacity < total) throw Error(BBTN_E_BUFFER_TOO_SMALL, "leaf buffer too small");
    int64_t row = 0;
    for (const auto& g : groups)
      for (int64_t l = 0; l < g.count; ++l, ++row) {
        int8_t* out = leaves + row * n;
        std::memset(out, -1, (size_t)n);
        for (size_t j = 0; j < g.vars.size(); ++j)
          out[g.vars[j]] = (int8_t)g.assign[(size_t)l * g.vars.size() + j];
      }
  });
}

bbtn_status bbtn_scorer_collect(bbtn_ctx* ctx, int32_t kind, int32_t n, int32_t m,
                                const int32_t* edge_uv, const int32_t* weights, const int32_t* h,
                                int32_t log2_target, int32_t max_nodes, int32_t cand_per_node,
                                float* X, float* y, int64_t capacity, int64_t* rows) {
  if (!rows) return BBTN_E_INVALID_ARG;
  return guard(ctx, [&] {  // host-only: ctx may be NULL
    check_graph(n, m, edge_uv);
    BBTN_REQUIRE(kind == 0 || kind == 1, "kind must be 0 (spin glass) or 1 (MWIS)");
    BBTN_REQUIRE(log2_target > 0 && max_nodes >= 1 && cand_per_node >= 1, "bad sizes");
    Network net = kind == 0 ? build_spinglass(n, m, edge_uv, weights, h)
                            : build_mwis(n, m, edge_uv, weights);
    Tree tree = greedy_tree(net);
    std::vector<uint8_t> x = kind == 0 ? local_search_spinglass(n, m, edge_uv, weights, h, 200, 12345)
                                       : local_search_mwis(n, m, edge_uv, weights, 10, 12345);
    std::vector<float> fx, fy;
    const int rmax = ctx ? std::max(1, std::min(16, ctx->opt.region_max)) : 8;
    collect_training(net, tree, log2_target, rmax,
                     network_value(net, x), max_nodes, cand_per_node, fx, fy);
    *rows = (int64_t)fy.size();
    if (X && y) {
      BBTN_REQUIRE(capacity >= (int64_t)fy.size(), "capacity too small");
      std::memcpy(X, fx.data(), fx.size() * 4);
      std::memcpy(y, fy.data(), fy.size() * 4);
    }
  });
}

bbtn_status bbtn_scorer_train(bbtn_ctx* ctx, const float* X, const float* y, int64_t rows,
                              int32_t epochs, int32_t batch, float lr, uint64_t seed,
                              float* loss_out, const char* save_path) {
  if (!ctx) return BBTN_E_INVALID_ARG;
  return guard(ctx, [&] {
    BBTN_REQUIRE(X && y && rows >= 1 && epochs >= 1 && batch >= 1 && lr > 0, "bad arguments");
    BBTN_HIP(hipSetDevice(ctx->opt.device));
    hipStream_t st = ctx->stream;
    ScorerModel mdl;
    // standardisation
    for (int q = 0; q < N_FEAT; ++q) {
      double s = 0, s2 = 0;
      for (int64_t r = 0; r < rows; ++r) { s += X[r * N_FEAT + q]; s2 += (double)X[r * N_FEAT + q] * X[r * N_FEAT + q]; }
      const double mu = s / rows, var = std::max(0.0, s2 / rows - mu * mu);
      mdl.fmean[q] = (float)mu;
      mdl.fstd[q] = var > 1e-12 ? (float)std::sqrt(var) : 1.f;
    }
    {
      double s = 0, s2 = 0;
      for (int64_t r = 0; r < rows; ++r) { s += y[r]; s2 += (double)y[r] * y[r]; }
      const double mu = s / rows, var = std::max(0.0, s2 / rows - mu * mu);
      mdl.ymean = (float)mu;
      mdl.ystd = var > 1e-12 ? (float)std::sqrt(var) : 1.f;
    }
    // shuffled, standardised data (bf16 inputs, f32 targets)
    std::mt19937_64 rng(seed);
    std::vector<int64_t> perm(rows);
    for (int64_t r = 0; r < rows; ++r) perm[r] = r;
    std::shuffle(perm.begin(), perm.end(), rng);
    std::vector<uint16_t> xb((size_t)rows * N_FEAT);
    std::vector<float> yt(rows);
    for (int64_t i = 0; i < rows; ++i) {
      const int64_t r = perm[i];
      for (int q = 0; q < N_FEAT; ++q) {
        float v = (X[r * N_FEAT + q] - mdl.fmean[q]) / mdl.fstd[q];
        uint32_t u;
        std::memcpy(&u, &v, 4);
        xb[i * N_FEAT + q] = (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
      }
      yt[i] = (y[r] - mdl.ymean) / mdl.ystd;
    }
    // parameters: uniform +-1/sqrt(fan_in) weights, zero biases
    std::vector<float> master(MLP_NPARAM, 0.f);
    std::uniform_real_distribution<float> U(-1.f, 1.f);
    for (int i = 0; i < MLP_H * MLP_IN; ++i) master[MLP_W1 + i] = U(rng) / std::sqrt((float)MLP_IN);
    for (int i = 0; i < MLP_H * MLP_H; ++i) master[MLP_W2 + i] = U(rng) / std::sqrt((float)MLP_H);
    for (int i = 0; i < MLP_H; ++i) master[MLP_W3 + i] = U(rng) / std::sqrt((float)MLP_H);
    const int64_t B = std::min<int64_t>(batch, rows);
    // device buffers
    DevBuf dbuf;
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    size_t off = 0;
    const size_t o_x = off; off += al(xb.size() * 2);
    const size_t o_y = off; off += al(yt.size() * 4);
    const size_t o_p = off; off += al((size_t)rows * 4);
    const size_t o_h1 = off; off += al((size_t)rows * MLP_H * 4);
    const size_t o_h2 = off; off += al((size_t)rows * MLP_H * 4);
    const size_t o_ms = off; off += al(MLP_NPARAM * 4);
    const size_t o_m = off; off += al(MLP_NPARAM * 4);
    const size_t o_v = off; off += al(MLP_NPARAM * 4);
    const size_t o_g = off; off += al(MLP_NPART * 4);
    const size_t o_w = off; off += al(MLP_NW * 2);
    const size_t o_b = off; off += al(MLP_NB * 4);
    dbuf.ensure(off);
    char* d = dbuf.as<char>();
    std::vector<uint16_t> wb(MLP_NW);
    for (int i = 0; i < MLP_NW; ++i) {
      uint32_t u;
      std::memcpy(&u, &master[i], 4);
      wb[i] = (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
    }
    std::vector<float> zeros(MLP_NPARAM, 0.f);
    BBTN_HIP(hipMemcpyAsync(d + o_x, xb.data(), xb.size() * 2, hipMemcpyHostToDevice, st));
    BBTN_HIP(hipMemcpyAsync(d + o_y, yt.data(), yt.size() * 4, hipMemcpyHostToDevice, st));
    BBTN_HIP(hipMemcpyAsync(d + o_ms, master.data(), MLP_NPARAM * 4, hipMemcpyHostToDevice, st));
    BBTN_HIP(hipMemcpyAsync(d + o_m, zeros.data(), MLP_NPARAM * 4, hipMemcpyHostToDevice, st));
    BBTN_HIP(hipMemcpyAsync(d + o_v, zeros.data(), MLP_NPARAM * 4, hipMemcpyHostToDevice, st));
    BBTN_HIP(hipMemcpyAsync(d + o_w, wb.data(), MLP_NW * 2, hipMemcpyHostToDevice, st));
    BBTN_HIP(hipMemcpyAsync(d + o_b, master.data() + MLP_NW, MLP_NB * 4, hipMemcpyHostToDevice, st));
    ctx->partial.ensure((size_t)mlp_partial_floats(B) * 4);
    const uint16_t* dX = (const uint16_t*)(d + o_x);
    const float* dY = (const float*)(d + o_y);
    float* dP = (float*)(d + o_p);
    float* dH1 = (float*)(d + o_h1);
    float* dH2 = (float*)(d + o_h2);
    int step = 0;
    std::vector<float> pred(rows);
    for (int e = 0; e < epochs; ++e) {
      for (int64_t r0 = 0; r0 < rows; r0 += B) {
        const int64_t nb = std::min<int64_t>(B, rows - r0);
        launch_mlp_forward(nb, dX + r0 * N_FEAT, (const uint16_t*)(d + o_w),
                           (const float*)(d + o_b), dP + r0, dH1 + r0 * MLP_H, dH2 + r0 * MLP_H, st);
        launch_mlp_backward(nb, dX + r0 * N_FEAT, (const uint16_t*)(d + o_w), dP + r0, dY + r0,
                            dH1 + r0 * MLP_H, dH2 + r0 * MLP_H, ctx->partial.as<float>(),
                            (float*)(d + o_g), st);
        launch_mlp_adam((float*)(d + o_ms), (uint16_t*)(d + o_w), (float*)(d + o_b),
                        (float*)(d + o_m), (float*)(d + o_v), (const float*)(d + o_g), lr, 0.9f,
                        0.999f, 1e-8f, ++step, st);
      }
      if (loss_out) {
        launch_mlp_forward(rows, dX, (const uint16_t*)(d + o_w), (const float*)(d + o_b), dP,
                           nullptr, nullptr, st);
        BBTN_HIP(hipMemcpyAsync(pred.data(), dP, rows * 4, hipMemcpyDeviceToHost, st));
        BBTN_HIP(hipStreamSynchronize(st));
        double l = 0;
        for (int64_t r = 0; r < rows; ++r) l += (double)(pred[r] - yt[r]) * (pred[r] - yt[r]);
        loss_out[e] = (float)(l / rows);
      }
    }
    mdl.params.resize(MLP_NPARAM);
    BBTN_HIP(hipMemcpyAsync(mdl.params.data(), d + o_ms, MLP_NPARAM * 4, hipMemcpyDeviceToHost, st));
    BBTN_HIP(hipStreamSynchronize(st));
    dbuf.release();
    if (save_path) {
      if (!write_model(save_path, mdl)) throw Error(BBTN_E_INVALID_ARG, "cannot write scorer weights");
      load_scorer(ctx, save_path);
    }
  });
}

}  // extern "C"
