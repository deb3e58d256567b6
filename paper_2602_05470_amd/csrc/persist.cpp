#include "persist.h"

#include <algorithm>
#include <array>
#include <cstring>
#include <thread>
#include <atomic>
#include <map>
#include <string>

#include "persist_dev.h"

namespace bbtn {

int persist_max_rank(int k) {
  // two operand buffers of (1 + k) planes within 64 KiB of LDS
  int r = 0;
  while (persist_lds_bytes(k, 1ll << (r + 1), 0, 64, 0) <= (64u << 10)) ++r;
  return r;
}

bool persist_fits(const GroupPlan& g, int k) {
  if (g.steps.empty()) return true;
  // the per-task fixed-bit table lives in LDS: at most 4096 slots
  size_t n_slots = 0;
  for (const Step& s : g.steps) n_slots += !s.a.fixed_pos.empty() + !s.b.fixed_pos.empty();
  if (n_slots > 4096) return false;
  int mx = 0;
  for (const Step& s : g.steps) mx = std::max({mx, (int)s.a_vars.size(), (int)s.b_vars.size()});
  return mx <= std::min(persist_max_rank(k), P_MAX_RANK);
}

namespace {
size_t align_up(size_t x) { return (x + 255) / 256 * 256; }

// Offsets in the workgroup's LDS arena for the outputs of a branch program
// that hold at most `limit` entries: first fit over their lifetimes (from
// the producing step to the last step reading them; the root lives to the
// end).  Sets *entries to the arena size.
std::map<int32_t, int64_t> lds_arena(const GroupPlan& g, const std::vector<const Step*>& prog,
                                     int64_t limit, int64_t* entries) {
  std::map<int32_t, std::pair<int, int>> life;  // buffer -> (def, last use)
  for (int i = 0; i < (int)prog.size(); ++i) {
    const Step& s = *prog[i];
    for (const Operand* op : {&s.a, &s.b})
      if (!op->base) {
        auto it = life.find(op->id);
        if (it != life.end()) it->second.second = i;
      }
    if (g.buf_region[s.out] == R_BRANCH && g.buf_entries[s.out] <= limit)
      life[s.out] = {i, i};
  }
  if (g.root_buf >= 0) {
    auto it = life.find(g.root_buf);
    if (it != life.end()) it->second.second = (int)prog.size();
  }
  std::vector<int32_t> order;
  for (auto& kv : life) order.push_back(kv.first);
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t x, int32_t y) { return life[x].first < life[y].first; });
  std::map<int32_t, int64_t> off;
  std::vector<int32_t> active;
  int64_t peak = 0;
  for (int32_t b : order) {
    active.erase(std::remove_if(active.begin(), active.end(),
                                [&](int32_t j) { return life[j].second < life[b].first; }),
                 active.end());
    std::vector<std::pair<int64_t, int64_t>> busy;
    for (int32_t j : active) busy.push_back({off[j], off[j] + g.buf_entries[j]});
    std::sort(busy.begin(), busy.end());
    int64_t o = 0;
    for (auto& bz : busy) {
      if (o + g.buf_entries[b] <= bz.first) break;
      o = std::max(o, bz.second);
    }
    off[b] = o;
    peak = std::max(peak, o + g.buf_entries[b]);
    active.push_back(b);
  }
  *entries = peak;
  return off;
}
// LDS a workgroup may allocate (bytes)
size_t lds_per_workgroup() {
  static size_t bytes = [] {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return (size_t)64 << 10;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        n <= 0)
      return (size_t)64 << 10;
    return std::min<size_t>((size_t)n, (size_t)160 << 10);
  }();
  return bytes;
}
int device_cus() {
  static int cus = [] {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 256;
    return n > 0 ? n : 256;
  }();
  return cus;
}
}  // namespace

void run_persistent(bbtn_ctx* ctx, const std::vector<PersistJob>& jobs, const BaseDev& bd,
                    const Moduli& mod, hipStream_t st, bool per_task_scratch,
                    int64_t* scratch_entries) {
  const int k = bd.k;
  const int W = 1 + k;
  std::vector<PStep> steps;
  std::vector<PFix> fixes;
  std::vector<PSlot> slots;
  std::vector<PTask> shared_tasks, tasks;
  std::vector<uint8_t> assign;
  int64_t n_out = 0, scratch = 1, max_rank = 0, shared_total = 0;
  int32_t max_slots = 0;
  std::vector<int64_t> out_base(jobs.size());
  // programs already emitted, by content: instances with the same
  // contraction tree and fixed set share one copy
  struct ProgRef {
    int32_t step_off, n_steps, slot_off, n_slots;
    int64_t arena = 0;      // LDS arena entries the program uses
    int64_t root_lds = -1;  // arena offset of the root scalar, or -1
  };
  // branch outputs of at most lds_limit entries live in an LDS arena of the
  // workgroup: smaller for more residues, so that the arena does not lower
  // the workgroups per CU the operand staging admits
  const int64_t lds_limit = k == 0 ? 256 : 128;
  int64_t max_arena = 0;
  // LDS left for the arena: what a workgroup may allocate, less the operand
  // staging, the partials of the widest workgroup and the fixed-bit table of
  // the launch's largest program
  int rank_all = 0;
  size_t slot_bound = 0;
  for (const PersistJob& j : jobs) {
    rank_all = std::max(rank_all, (int)j.plan->max_rank);
    size_t n = 0;
    for (const Step& st_ : j.plan->steps) n += !st_.a.fixed_pos.empty() + !st_.b.fixed_pos.empty();
    slot_bound = std::max(slot_bound, n);
  }
  const size_t fixed_lds =
      persist_lds_bytes(k, 1ll << std::min(rank_all, P_MAX_RANK), 0, 1024, (int)slot_bound);
  const int64_t arena_budget =
      fixed_lds < lds_per_workgroup() ? (int64_t)((lds_per_workgroup() - fixed_lds) / (4 * W)) : 0;
  std::map<std::string, ProgRef> seen;
  // programs already emitted per plan: a job with the same plan and the
  // same base-tensor layout (offsets relative to its first tensor) reuses
  // them without emitting again
  struct Emitted {
    std::vector<int64_t> rel;  // base offsets relative to the first tensor
    std::vector<ProgRef> shared;
    ProgRef branch;
  };
  std::map<const GroupPlan*, Emitted> emitted;
  int64_t n_branch_tasks = 0;
  for (size_t ji = 0; ji < jobs.size(); ++ji) {
    const GroupPlan& g = *jobs[ji].plan;
    const int64_t shared_base = shared_total;
    shared_total += g.shared_total;
    scratch = std::max<int64_t>(scratch, std::max(g.peak, g.subtree_peak));
    const Network& net = *jobs[ji].net;
    const int64_t base0 = net.tensors.empty() ? 0 : jobs[ji].base_off[0];
    std::vector<int64_t> rel(net.tensors.size());
    for (size_t t = 0; t < rel.size(); ++t) rel[t] = jobs[ji].base_off[t] - base0;
    auto hit = emitted.find(&g);
    const bool reuse = hit != emitted.end() && hit->second.rel == rel;
    std::vector<int> pos_of;
    if (!reuse) {
      pos_of.assign(net.n, -1);
      for (size_t j = 0; j < g.fixed_vars.size(); ++j) pos_of[g.fixed_vars[j]] = (int)j;
    }
    // a program: steps, their fixed-bit slots and fixes (offsets relative to
    // the program), deduplicated by content
    auto emit_program = [&](const std::vector<const Step*>& prog,
                            const std::map<int32_t, int64_t>& in_lds) {
      auto lds_off = [&](int32_t buf) {
        auto it = in_lds.find(buf);
        return it == in_lds.end() ? (int64_t)-1 : it->second;
      };
      std::vector<PStep> ps_v;
      std::vector<PSlot> sl_v;
      std::vector<PFix> fx_v;
      for (const Step* sp : prog) {
        const Step& s = *sp;
        PStep ps{};
        ps.rb = s.rb; ps.rm = s.rm; ps.rn = s.rn; ps.rk = s.rk;
        const bool out_shared = g.buf_region[s.out] == R_SHARED;
        ps.c_kind = out_shared ? PK_SHARED : PK_SCRATCH;
        ps.c_off = g.buf_off[s.out];
        if (lds_off(s.out) >= 0) {
          ps.c_kind = PK_LDS;
          ps.c_off = lds_off(s.out);
        }
        const Operand* ops[2] = {&s.a, &s.b};
        POperand* pops[2] = {&ps.a, &ps.b};
        for (int w = 0; w < 2; ++w) {
          const Operand& op = *ops[w];
          POperand& po = *pops[w];
          const int rank = (int)op.src_bits.size();
          max_rank = std::max<int64_t>(max_rank, rank);
          if (rank > P_MAX_RANK) throw Error(BBTN_E_INTERNAL, "persistent: operand rank too large");
          if (op.base) {
            po.kind = PK_BASE;
            po.src_off = jobs[ji].base_off[op.id] - base0;
          } else if (g.buf_region[op.id] == R_SHARED) {
            po.kind = PK_SHARED;
            po.src_off = g.buf_off[op.id];
          } else if (lds_off(op.id) >= 0) {
            po.kind = PK_LDS;
            po.src_off = lds_off(op.id);
          } else {
            po.kind = PK_SCRATCH;
            po.src_off = g.buf_off[op.id];
          }
          po.rank = rank;
          for (int j = 0; j < rank; ++j)
            po.bitpos[j / 4] |= (uint32_t)op.src_bits[j] << (8 * (j % 4));
          // programs that keep everything materialise gathered operands
          po.mat_off = (op.temp >= 0 && g.keep_all) ? g.buf_off[op.temp] : -1;
          po.slot = -1;
          if (!op.fixed_pos.empty()) {  // sliced per branch: a fixed-bit slot
            po.slot = (int32_t)sl_v.size();
            sl_v.push_back(PSlot{(int32_t)fx_v.size(), (int32_t)op.fixed_pos.size()});
            for (auto& fp : op.fixed_pos) fx_v.push_back(PFix{fp.first, pos_of[fp.second]});
          }
        }
        ps_v.push_back(ps);
      }
      std::string key((const char*)ps_v.data(), ps_v.size() * sizeof(PStep));
      key.append((const char*)sl_v.data(), sl_v.size() * sizeof(PSlot));
      key.append((const char*)fx_v.data(), fx_v.size() * sizeof(PFix));
      auto it = seen.find(key);
      if (it != seen.end()) return it->second;
      ProgRef pr{(int32_t)steps.size(), (int32_t)ps_v.size(), (int32_t)slots.size(),
                 (int32_t)sl_v.size()};
      const int32_t fix0 = (int32_t)fixes.size();
      for (PSlot q : sl_v) slots.push_back(PSlot{q.fix_off + fix0, q.n_fix});
      fixes.insert(fixes.end(), fx_v.begin(), fx_v.end());
      steps.insert(steps.end(), ps_v.begin(), ps_v.end());
      max_slots = std::max(max_slots, pr.n_slots);
      seen.emplace(std::move(key), pr);
      return pr;
    };
    // shared subtrees: one task each, run before any branch
    std::vector<ProgRef> shared_refs;
    ProgRef branch_ref;
    if (reuse) {
      shared_refs = hit->second.shared;
      branch_ref = hit->second.branch;
    } else {
      for (auto& rg : g.shared_ranges) {
        std::vector<const Step*> prog;
        for (int i = rg.first; i < rg.second; ++i) prog.push_back(&g.steps[i]);
        shared_refs.push_back(emit_program(prog, {}));
      }
      std::vector<const Step*> prog;
      for (const Step& s : g.steps)
        if (!s.shared) prog.push_back(&s);
      int64_t arena = 0;
      std::map<int32_t, int64_t> in_lds;
      // the largest size limit (halving) whose arena fits the budget
      for (int64_t lim = g.keep_all ? 0 : lds_limit; lim > 0; lim /= 2) {
        in_lds = lds_arena(g, prog, lim, &arena);
        if (arena <= arena_budget) break;
        in_lds.clear();
        arena = 0;
      }
      branch_ref = emit_program(prog, in_lds);
      branch_ref.arena = arena;
      branch_ref.root_lds = -1;
      if (g.root_buf >= 0 && in_lds.count(g.root_buf)) branch_ref.root_lds = in_lds.at(g.root_buf);
      if (hit == emitted.end()) emitted.emplace(&g, Emitted{rel, shared_refs, branch_ref});
    }
    for (const ProgRef& pr : shared_refs) {
      PTask t{};
      t.step_off = pr.step_off;
      t.n_steps = pr.n_steps;
      t.slot_off = pr.slot_off;
      t.n_slots = pr.n_slots;
      t.first = (int64_t)shared_tasks.size();
      t.assign_off = 0;
      t.assign_stride = 0;
      t.out_idx = -1;
      t.root_off = -1;
      t.base_off = base0;
      t.shared_off = shared_base;
      shared_tasks.push_back(t);
    }
    // the branches: one run of L tasks
    const size_t S = g.fixed_vars.size();
    out_base[ji] = n_out;
    if (jobs[ji].L > 0) {
      PTask t{};
      t.step_off = branch_ref.step_off;
      t.n_steps = branch_ref.n_steps;
      t.slot_off = branch_ref.slot_off;
      t.n_slots = branch_ref.n_slots;
      t.first = n_branch_tasks;
      t.assign_off = (int64_t)assign.size();
      t.assign_stride = (int64_t)S;
      t.out_idx = n_out;
      t.root_off = g.root_buf >= 0 ? g.buf_off[g.root_buf] : -1;
      t.root_kind = PK_SCRATCH;
      if (branch_ref.root_lds >= 0) {
        t.root_kind = PK_LDS;
        t.root_off = branch_ref.root_lds;
      }
      t.base_off = base0;
      t.shared_off = shared_base;
      tasks.push_back(t);
      max_arena = std::max(max_arena, branch_ref.arena);
    }
    assign.insert(assign.end(), jobs[ji].assign, jobs[ji].assign + jobs[ji].L * S);
    n_out += jobs[ji].L;
    n_branch_tasks += jobs[ji].L;
  }
  if (tasks.empty()) return;
  // folded constants per branch, gathered into (1 + k) planes of n_out
  std::vector<int> pidx(k);
  for (int p = 0; p < k; ++p) {
    const auto& P = prime_table();
    pidx[p] = (int)(std::find(P.begin(), P.end(), mod.p[p]) - P.begin());
  }
  std::vector<uint32_t> lconst((size_t)W * n_out);
  {
    // jobs write disjoint slices: a few host threads when there are many
    std::atomic<size_t> next{0};
    auto work = [&] {
      std::vector<uint32_t> lc;
      for (size_t ji; (ji = next.fetch_add(1)) < jobs.size();) {
        leaf_constants(*jobs[ji].net, *jobs[ji].plan, pidx.data(), k, jobs[ji].assign,
                       jobs[ji].L, lc);
        for (int p = 0; p < W; ++p)
          std::memcpy(&lconst[(size_t)p * n_out + out_base[ji]], &lc[(size_t)p * jobs[ji].L],
                      jobs[ji].L * 4);
      }
    };
    const size_t T = std::min<size_t>(8, (n_branch_tasks >> 14) + 1);
    std::vector<std::thread> pool;
    for (size_t t = 1; t < T; ++t) pool.emplace_back(work);
    work();
    for (auto& th : pool) th.join();
  }
  // one device buffer for the program and per-branch data
  size_t off = 0;
  const size_t o_steps = off; off = align_up(off + steps.size() * sizeof(PStep));
  const size_t o_fixes = off; off = align_up(off + std::max<size_t>(fixes.size(), 1) * sizeof(PFix));
  const size_t o_slots = off; off = align_up(off + std::max<size_t>(slots.size(), 1) * sizeof(PSlot));
  const size_t o_stasks = off; off = align_up(off + std::max<size_t>(shared_tasks.size(), 1) * sizeof(PTask));
  const size_t o_tasks = off; off = align_up(off + tasks.size() * sizeof(PTask));
  const size_t o_assign = off; off = align_up(off + std::max<size_t>(assign.size(), 1));
  const size_t o_lconst = off; off = align_up(off + lconst.size() * 4);
  const size_t o_out = off; off = align_up(off + lconst.size() * 4);
  const size_t o_queue = off; off = align_up(off + 16);
  const size_t o_shared = off; off = align_up(off + (size_t)W * std::max<int64_t>(shared_total, 1) * 4);
  // staged in pinned memory (written only after the previous launch's
  // results were read back, which synchronised the stream)
  BBTN_HIP(hipStreamSynchronize(st));
  ctx->pin_persist.ensure(o_out);
  uint8_t* host = ctx->pin_persist.as<uint8_t>();
  std::memset(host, 0, o_out);
  std::memcpy(&host[o_steps], steps.data(), steps.size() * sizeof(PStep));
  if (!fixes.empty()) std::memcpy(&host[o_fixes], fixes.data(), fixes.size() * sizeof(PFix));
  if (!slots.empty()) std::memcpy(&host[o_slots], slots.data(), slots.size() * sizeof(PSlot));
  if (!shared_tasks.empty()) std::memcpy(&host[o_stasks], shared_tasks.data(), shared_tasks.size() * sizeof(PTask));
  std::memcpy(&host[o_tasks], tasks.data(), tasks.size() * sizeof(PTask));
  if (!assign.empty()) std::memcpy(&host[o_assign], assign.data(), assign.size());
  std::memcpy(&host[o_lconst], lconst.data(), lconst.size() * 4);
  ctx->persist.ensure(off);
  uint8_t* dev = ctx->persist.as<uint8_t>();
  BBTN_HIP(hipMemcpyAsync(dev, host, o_out, hipMemcpyHostToDevice, st));
  // launch shape per launch: one-wave workgroups when tasks are plentiful,
  // wider ones when they are few; as many per CU as LDS and the wave limit
  // allow, never more than tasks
  const int64_t lds_entries = 1ll << max_rank;
  struct Shape {
    int threads;
    int64_t blocks;
  };
  auto shape_for = [&](int64_t n_tasks) {
    const int64_t cus = device_cus();
    auto per_cu = [&](int threads) {
      const size_t lds = persist_lds_bytes(k, lds_entries, max_arena, threads, max_slots);
      const int by_lds = (int)((160u << 10) / std::max<size_t>(lds, 1));
      const int by_waves = 32 / (threads / 64);
      return std::max(1, std::min({32, by_lds, by_waves}));
    };
    int threads = n_tasks >= 2 * cus ? 64 : (n_tasks >= cus / 4 ? 256 : 1024);
    // one-wave workgroups whose LDS admits fewer than 8 per CU leave the CU
    // waiting on memory: give each task four waves instead
    if (threads == 64 && per_cu(64) < 8) threads = 256;
    return Shape{threads, std::min<int64_t>(cus * per_cu(threads), n_tasks)};
  };
  const Shape sh_shared = shape_for((int64_t)shared_tasks.size());
  const Shape sh_branch = shape_for(n_branch_tasks);
  int64_t most = std::max<int64_t>(shared_tasks.empty() ? 0 : sh_shared.blocks, sh_branch.blocks);
  if (per_task_scratch) {
    BBTN_REQUIRE(shared_tasks.empty(), "per-task scratch takes programs without shared steps");
    most = n_branch_tasks;
  }
  ctx->work.ensure((size_t)most * W * scratch * 4);
  if (scratch_entries) *scratch_entries = scratch;
  PersistArgs a{};
  a.steps = (const PStep*)(dev + o_steps);
  a.fixes = (const PFix*)(dev + o_fixes);
  a.slots = (const PSlot*)(dev + o_slots);
  a.max_slots = max_slots;
  a.assign = dev + o_assign;
  a.base = bd.t.ptr;
  a.base_total = bd.total;
  a.lconst = (const uint32_t*)(dev + o_lconst);
  a.out = (uint32_t*)(dev + o_out);
  a.n_out = n_out;
  a.scratch = ctx->work.as<uint32_t>();
  a.scratch_entries = scratch;
  a.shared = (uint32_t*)(dev + o_shared);
  a.shared_entries = std::max<int64_t>(shared_total, 1);
  a.lds_entries = lds_entries;
  a.arena_entries = max_arena;
  a.per_task_scratch = per_task_scratch ? 1 : 0;
  a.mod = mod;
  // algorithmic work of the launch: semiring operations and operand bytes
  // (entries of A, B and C of every step), summed once per plan
  double ops = 0, bytes = 0;
  std::map<const GroupPlan*, std::pair<double, double>> entries;  // (shared, per branch)
  for (auto& j : jobs) {
    ops += ((double)j.L * j.plan->macs + j.plan->shared_macs) * (2 + 2 * k);
    auto it = entries.find(j.plan);
    if (it == entries.end()) {
      double sh = 0, br = 0;
      for (const Step& s : j.plan->steps)
        (s.shared ? sh : br) += std::ldexp(1.0, (int)s.a_vars.size()) +
                                std::ldexp(1.0, (int)s.b_vars.size()) +
                                std::ldexp(1.0, (int)s.c_vars.size());
      it = entries.emplace(j.plan, std::make_pair(sh, br)).first;
    }
    bytes += (it->second.first + (double)j.L * it->second.second) * W * 4;
  }
  const int ph = ctx->prof.begin(st, K_PERSIST);
  if (!shared_tasks.empty()) {
    // shared subtrees first, then the branches (stream order separates them)
    a.tasks = (const PTask*)(dev + o_stasks);
    a.n_runs = (int64_t)shared_tasks.size();
    a.n_tasks = (int64_t)shared_tasks.size();
    a.queue = (unsigned long long*)(dev + o_queue);
    launch_persist(k, a, (int)sh_shared.blocks, sh_shared.threads, st);
  }
  a.tasks = (const PTask*)(dev + o_tasks);
  a.n_runs = (int64_t)tasks.size();
  a.n_tasks = n_branch_tasks;
  a.queue = (unsigned long long*)(dev + o_queue + 8);
  launch_persist(k, a, (int)sh_branch.blocks, sh_branch.threads, st);
  ctx->prof.end(ph, st, K_PERSIST, ops, bytes);
  std::vector<uint32_t> outh(lconst.size());
  BBTN_HIP(hipMemcpyAsync(outh.data(), dev + o_out, outh.size() * 4, hipMemcpyDeviceToHost, st));
  BBTN_HIP(hipStreamSynchronize(st));
  ctx->prof.resolve();
  for (size_t ji = 0; ji < jobs.size(); ++ji) {
    auto& o = *jobs[ji].out;
    const int64_t L = jobs[ji].L;
    o.assign((size_t)W * L, 0);
    for (int p = 0; p < W; ++p)
      std::memcpy(&o[(size_t)p * L], &outh[(size_t)p * n_out + out_base[ji]], L * 4);
  }
  uint64_t macs = 0;
  for (auto& j : jobs) macs += (uint64_t)(j.L * j.plan->macs + j.plan->shared_macs);
  ctx->last_macs += macs;
}

SmallForest plan_small_forest(const GroupPlan& g, const std::vector<int64_t>& base_off, int k,
                              int64_t L) {
  SmallForest f;
  const int W = 1 + k;
  const int n = (int)g.steps.size();
  f.in.assign(n, 0);
  f.root_off.assign(g.buf_entries.size(), -1);
  if (n == 0) return f;
  // in place: a keep-all program of one branch, values only (its buffers
  // are disjoint, W = 1)
  f.in_place = g.keep_all;
  if (g.keep_all && (L != 1 || k != 0)) return f;
  // operand staging within the default 64 KiB of LDS
  int rmax = 0;
  while (rmax < P_MAX_RANK &&
         persist_lds_bytes(k, 1ll << (rmax + 1), 0, f.threads, 0) <= (64u << 10))
    ++rmax;
  std::vector<int> prod(g.buf_entries.size(), -1), cons(g.buf_entries.size(), -1);
  for (int i = 0; i < n; ++i) {
    prod[g.steps[i].out] = i;
    for (const Operand* op : {&g.steps[i].a, &g.steps[i].b})
      if (!op->base) cons[op->id] = i;
  }
  for (int i = 0; i < n; ++i) {
    const Step& s = g.steps[i];
    bool ok = (s.shared || L == 1) && s.a.fixed_pos.empty() && s.b.fixed_pos.empty();
    ok = ok && std::max({(int)s.a_vars.size(), (int)s.b_vars.size(), (int)s.c_vars.size(),
                         s.a.r_in, s.b.r_in}) <= rmax;
    for (const Operand* op : {&s.a, &s.b})
      if (!op->base) ok = ok && prod[op->id] >= 0 && f.in[prod[op->id]];
    f.in[i] = ok;
  }
  // tasks: a root (output read outside the forest, or the program's result)
  // opens one; every other forest step joins its consumer's
  std::vector<int> task_of(n, -1);
  int n_tasks = 0;
  for (int i = n - 1; i >= 0; --i) {
    if (!f.in[i]) continue;
    const int out = g.steps[i].out;
    const int c = cons[out];
    const bool root = c < 0 || !f.in[c] || out == g.root_buf;
    task_of[i] = root ? n_tasks++ : task_of[c];
    if (root && !f.in_place) {
      f.root_off[out] = f.root_entries;
      f.root_entries += g.buf_entries[out];
    }
  }
  if (n_tasks == 0) return f;
  std::vector<std::vector<int>> members(n_tasks);
  for (int i = 0; i < n; ++i)
    if (f.in[i]) members[task_of[i]].push_back(i);
  std::vector<int> order(n_tasks);
  for (int t = 0; t < n_tasks; ++t) order[t] = t;
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return members[x].size() > members[y].size(); });
  std::vector<int64_t> scr_off(g.buf_entries.size(), -1);
  for (int t : order) {
    const std::vector<int>& m = members[t];
    // scratch offsets of the task's intermediates: first fit over their
    // lifetimes (local step index of the producer to that of the consumer)
    std::map<int, int> local;
    for (int j = 0; j < (int)m.size(); ++j) local[m[j]] = j;
    int64_t peak = 0;
    std::vector<std::array<int64_t, 3>> busy;  // off, end, last use
    for (int j = 0; j < (int)m.size() && !f.in_place; ++j) {
      const Step& s = g.steps[m[j]];
      if (f.root_off[s.out] >= 0) continue;
      const int last = local.at(cons[s.out]);
      busy.erase(std::remove_if(busy.begin(), busy.end(),
                                [&](const std::array<int64_t, 3>& b) { return b[2] < j; }),
                 busy.end());
      std::sort(busy.begin(), busy.end());
      const int64_t e = g.buf_entries[s.out];
      int64_t o = 0;
      for (auto& b : busy) {
        if (o + e <= b[0]) break;
        o = std::max(o, b[1]);
      }
      scr_off[s.out] = o;
      busy.push_back({o, o + e, (int64_t)last});
      peak = std::max(peak, o + e);
    }
    f.scratch_entries = std::max(f.scratch_entries, peak);
    PTask tk{};
    tk.step_off = (int32_t)f.steps.size();
    tk.n_steps = (int32_t)m.size();
    tk.first = (int64_t)f.tasks.size();
    tk.out_idx = -1;
    tk.root_off = -1;
    for (int i : m) {
      const Step& s = g.steps[i];
      PStep ps{};
      ps.rb = s.rb; ps.rm = s.rm; ps.rn = s.rn; ps.rk = s.rk;
      if (f.in_place) {
        ps.c_kind = PK_SCRATCH;  // the workspace (W = 1, one branch)
        ps.c_off = g.buf_off[s.out];
      } else if (f.root_off[s.out] >= 0) {
        ps.c_kind = PK_SHARED;
        ps.c_off = (int64_t)W * f.root_off[s.out];
        ps.c_stride = (int32_t)g.buf_entries[s.out];
      } else {
        ps.c_kind = PK_SCRATCH;
        ps.c_off = scr_off[s.out];
      }
      const Operand* ops[2] = {&s.a, &s.b};
      POperand* pops[2] = {&ps.a, &ps.b};
      for (int w = 0; w < 2; ++w) {
        const Operand& op = *ops[w];
        POperand& po = *pops[w];
        const int rank = (int)op.src_bits.size();
        f.max_rank = std::max(f.max_rank, rank);
        if (op.base) {
          po.kind = PK_BASE;
          po.src_off = base_off[op.id];
        } else {
          po.kind = PK_SCRATCH;
          po.src_off = f.in_place ? g.buf_off[op.id] : scr_off[op.id];
          if (po.src_off < 0) throw Error(BBTN_E_INTERNAL, "small forest: operand outside its task");
        }
        po.rank = rank;
        for (int j = 0; j < rank; ++j) po.bitpos[j / 4] |= (uint32_t)op.src_bits[j] << (8 * (j % 4));
        // in place, gathered operands are materialised where the traceback
        // reads them
        po.mat_off = (f.in_place && op.temp >= 0) ? g.buf_off[op.temp] : -1;
        po.slot = -1;
      }
      f.steps.push_back(ps);
      f.ops += s.macs() * (2 + 2 * k);
      f.bytes += (std::ldexp(1.0, (int)s.a_vars.size()) + std::ldexp(1.0, (int)s.b_vars.size()) +
                  std::ldexp(1.0, (int)s.c_vars.size())) * W * 4;
    }
    f.tasks.push_back(tk);
  }
  return f;
}

namespace {
int64_t forest_blocks(const SmallForest& f, int k) {
  const size_t lds = persist_lds_bytes(k, 1ll << f.max_rank, 0, f.threads, 0);
  const int per_cu = std::max(1, std::min<int>((int)((160u << 10) / std::max<size_t>(lds, 1)),
                                               32 / (f.threads / 64)));
  return std::min<int64_t>((int64_t)device_cus() * per_cu, (int64_t)f.tasks.size());
}
size_t forest_scratch_off(const SmallForest& f, int k) {
  return align_up((size_t)(1 + k) * f.root_entries * 4);
}
}  // namespace

size_t small_forest_prog_off(const SmallForest& f, int k) {
  return forest_scratch_off(f, k) +
         align_up((size_t)forest_blocks(f, k) * (1 + k) * std::max<int64_t>(f.scratch_entries, 1) * 4);
}

std::vector<uint8_t> small_forest_image(const SmallForest& f) {
  const size_t o_tasks = align_up(f.steps.size() * sizeof(PStep));
  const size_t o_queue = o_tasks + align_up(f.tasks.size() * sizeof(PTask));
  std::vector<uint8_t> img(o_queue + 16, 0);
  std::memcpy(img.data(), f.steps.data(), f.steps.size() * sizeof(PStep));
  std::memcpy(img.data() + o_tasks, f.tasks.data(), f.tasks.size() * sizeof(PTask));
  return img;
}

size_t small_forest_bytes(const SmallForest& f, int k) {
  return small_forest_prog_off(f, k) + small_forest_image(f).size();
}

void launch_small_forest(const SmallForest& f, int k, const Moduli& mod, const BaseDev& bd,
                         uint8_t* dev, hipStream_t st, uint32_t* workspace) {
  if (f.tasks.empty()) return;
  const size_t o_prog = small_forest_prog_off(f, k);
  const size_t o_tasks = align_up(f.steps.size() * sizeof(PStep));
  const size_t o_queue = o_tasks + align_up(f.tasks.size() * sizeof(PTask));
  PersistArgs a{};
  a.steps = (const PStep*)(dev + o_prog);
  a.fixes = nullptr;  // no fixed-bit slots: never read
  a.slots = nullptr;
  a.max_slots = 0;
  a.tasks = (const PTask*)(dev + o_prog + o_tasks);
  a.n_runs = (int64_t)f.tasks.size();
  a.n_tasks = (int64_t)f.tasks.size();
  a.assign = nullptr;
  a.base = bd.t.ptr;
  a.base_total = bd.total;
  a.lconst = nullptr;  // no branch results: never read
  a.out = nullptr;
  a.n_out = 0;
  a.scratch = (uint32_t*)(dev + forest_scratch_off(f, k));
  a.scratch_entries = std::max<int64_t>(f.scratch_entries, 1);
  a.shared = (uint32_t*)dev;  // the root region (per-tensor plane strides)
  a.shared_entries = std::max<int64_t>(f.root_entries, 1);
  a.lds_entries = 1ll << f.max_rank;
  a.arena_entries = 0;
  a.per_task_scratch = 0;
  if (f.in_place) {
    // every task addresses the workspace itself: per-task scratch at a
    // stride of zero entries (one plane, W = 1)
    BBTN_REQUIRE(workspace != nullptr && k == 0, "in-place forest needs the values workspace");
    a.scratch = workspace;
    a.scratch_entries = 0;
    a.per_task_scratch = 1;
  }
  a.queue = (unsigned long long*)(dev + o_prog + o_queue);
  a.mod = mod;
  launch_persist(k, a, (int)forest_blocks(f, k), f.threads, st);
}

}  // namespace bbtn
