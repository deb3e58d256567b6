#include "persist.h"

#include <cstring>

#include "persist_dev.h"

namespace bbtn {

int persist_max_rank(int k) {
  // two operand buffers of (1 + k) planes within 64 KiB of LDS, so that two
  // workgroups share a CU
  int r = 0;
  while (persist_lds_bytes(k, 1ll << (r + 1)) <= (64u << 10)) ++r;
  return r;
}

bool persist_fits(const GroupPlan& g, int k) {
  if (g.steps.empty()) return true;
  int mx = 0;
  for (const Step& s : g.steps) mx = std::max({mx, (int)s.a_vars.size(), (int)s.b_vars.size()});
  for (const Step& s : g.steps) {
    const Operand* ops[2] = {&s.a, &s.b};
    for (const Operand* op : ops)
      if ((int)op->src_bits.size() > P_MAX_RUNS && make_gather_plan(op->r_in, (int)op->src_bits.size(), op->src_bits.data()).n_runs > P_MAX_RUNS)
        return false;
  }
  return mx <= persist_max_rank(k);
}

namespace {
size_t align_up(size_t x) { return (x + 255) / 256 * 256; }
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

void run_persistent(bbtn_ctx* ctx, const Network& net, const std::vector<PersistJob>& jobs,
                    const BaseDev& bd, const Moduli& mod, hipStream_t st) {
  const int k = bd.k;
  const int W = 1 + k;
  std::vector<PStep> steps;
  std::vector<PGroup> groups;
  std::vector<PFix> fixes;
  std::vector<PTask> tasks;
  std::vector<uint8_t> assign;
  int64_t n_out = 0, scratch = 1, max_rank = 0;
  std::vector<int64_t> out_base(jobs.size());
  for (size_t ji = 0; ji < jobs.size(); ++ji) {
    const GroupPlan& g = *jobs[ji].plan;
    PGroup pg{};
    pg.step_off = (int32_t)steps.size();
    pg.n_steps = (int32_t)g.steps.size();
    pg.root_off = g.root_buf >= 0 ? g.buf_off[g.root_buf] : -1;
    scratch = std::max<int64_t>(scratch, g.peak);
    std::vector<int> pos_of(net.n, -1);
    for (size_t j = 0; j < g.fixed_vars.size(); ++j) pos_of[g.fixed_vars[j]] = (int)j;
    for (const Step& s : g.steps) {
      PStep ps{};
      ps.rb = s.rb; ps.rm = s.rm; ps.rn = s.rn; ps.rk = s.rk;
      ps.c_off = g.buf_off[s.out];
      const Operand* ops[2] = {&s.a, &s.b};
      POperand* pops[2] = {&ps.a, &ps.b};
      for (int w = 0; w < 2; ++w) {
        const Operand& op = *ops[w];
        POperand& po = *pops[w];
        const int rank = (int)op.src_bits.size();
        max_rank = std::max<int64_t>(max_rank, rank);
        const GatherPlan gpn = make_gather_plan(op.r_in, rank, op.src_bits.data());
        if (gpn.n_runs > P_MAX_RUNS) throw Error(BBTN_E_INTERNAL, "persistent: too many runs");
        po.base = op.base ? 1 : 0;
        po.rank = rank;
        po.src_off = op.base ? bd.off[op.id] : g.buf_off[op.id];
        po.n_runs = gpn.n_runs;
        for (int r = 0; r < gpn.n_runs; ++r) po.runs[r] = gpn.runs[r];
        // programs that keep everything materialise gathered operands
        po.mat_off = (op.temp >= 0 && g.keep_all) ? g.buf_off[op.temp] : -1;
        po.fix_off = (int32_t)fixes.size();
        po.n_fix = 0;
        if (op.base)
          for (auto& fp : op.fixed_pos) {
            fixes.push_back(PFix{fp.first, pos_of[fp.second]});
            po.n_fix++;
          }
      }
      steps.push_back(ps);
    }
    groups.push_back(pg);
    const size_t S = g.fixed_vars.size();
    out_base[ji] = n_out;
    for (int64_t l = 0; l < jobs[ji].L; ++l) {
      PTask t{};
      t.group = (int32_t)ji;
      t.assign_off = (int64_t)assign.size() + (int64_t)(l * S);
      t.out_idx = n_out + l;
      tasks.push_back(t);
    }
    assign.insert(assign.end(), jobs[ji].assign, jobs[ji].assign + jobs[ji].L * S);
    n_out += jobs[ji].L;
  }
  if (tasks.empty()) return;
  // folded constants per branch, gathered into (1 + k) planes of n_out
  std::vector<int> pidx(k);
  for (int p = 0; p < k; ++p) {
    const auto& P = prime_table();
    pidx[p] = (int)(std::find(P.begin(), P.end(), mod.p[p]) - P.begin());
  }
  std::vector<uint32_t> lconst((size_t)W * n_out);
  for (size_t ji = 0; ji < jobs.size(); ++ji) {
    std::vector<uint32_t> lc;
    leaf_constants(net, *jobs[ji].plan, pidx.data(), k, jobs[ji].assign, jobs[ji].L, lc);
    for (int p = 0; p < W; ++p)
      std::memcpy(&lconst[(size_t)p * n_out + out_base[ji]], &lc[(size_t)p * jobs[ji].L],
                  jobs[ji].L * 4);
  }
  // one device buffer for the program and per-branch data
  size_t off = 0;
  const size_t o_steps = off; off = align_up(off + steps.size() * sizeof(PStep));
  const size_t o_groups = off; off = align_up(off + groups.size() * sizeof(PGroup));
  const size_t o_fixes = off; off = align_up(off + std::max<size_t>(fixes.size(), 1) * sizeof(PFix));
  const size_t o_tasks = off; off = align_up(off + tasks.size() * sizeof(PTask));
  const size_t o_assign = off; off = align_up(off + std::max<size_t>(assign.size(), 1));
  const size_t o_lconst = off; off = align_up(off + lconst.size() * 4);
  const size_t o_out = off; off = align_up(off + lconst.size() * 4);
  const size_t o_queue = off; off = align_up(off + 8);
  std::vector<uint8_t> host(o_out, 0);
  std::memcpy(&host[o_steps], steps.data(), steps.size() * sizeof(PStep));
  std::memcpy(&host[o_groups], groups.data(), groups.size() * sizeof(PGroup));
  if (!fixes.empty()) std::memcpy(&host[o_fixes], fixes.data(), fixes.size() * sizeof(PFix));
  std::memcpy(&host[o_tasks], tasks.data(), tasks.size() * sizeof(PTask));
  if (!assign.empty()) std::memcpy(&host[o_assign], assign.data(), assign.size());
  std::memcpy(&host[o_lconst], lconst.data(), lconst.size() * 4);
  ctx->persist.ensure(off);
  uint8_t* dev = ctx->persist.as<uint8_t>();
  BBTN_HIP(hipMemcpyAsync(dev, host.data(), host.size(), hipMemcpyHostToDevice, st));
  // launch shape: up to 2 workgroups per CU (LDS-limited), never more than tasks
  const int64_t lds_entries = 1ll << max_rank;
  const size_t lds = persist_lds_bytes(k, lds_entries);
  const int per_cu = std::max(1, std::min(2, (int)((160u << 10) / std::max<size_t>(lds, 1))));
  const int n_blocks = (int)std::min<int64_t>((int64_t)device_cus() * per_cu, (int64_t)tasks.size());
  ctx->work.ensure((size_t)n_blocks * W * scratch * 4);
  PersistArgs a{};
  a.steps = (const PStep*)(dev + o_steps);
  a.groups = (const PGroup*)(dev + o_groups);
  a.fixes = (const PFix*)(dev + o_fixes);
  a.tasks = (const PTask*)(dev + o_tasks);
  a.n_tasks = (int64_t)tasks.size();
  a.assign = dev + o_assign;
  a.base = bd.t.ptr;
  a.base_total = bd.total;
  a.lconst = (const uint32_t*)(dev + o_lconst);
  a.out = (uint32_t*)(dev + o_out);
  a.n_out = n_out;
  a.scratch = ctx->work.as<uint32_t>();
  a.scratch_entries = scratch;
  a.lds_entries = lds_entries;
  a.queue = (unsigned long long*)(dev + o_queue);
  a.mod = mod;
  double ops = 0, bytes = 0;
  for (auto& j : jobs) {
    ops += (double)j.L * j.plan->macs * (2 + 2 * k);
    double e = 0;
    for (const Step& s : j.plan->steps)
      e += std::ldexp(1.0, (int)s.a_vars.size()) + std::ldexp(1.0, (int)s.b_vars.size()) +
           std::ldexp(1.0, (int)s.c_vars.size());
    bytes += (double)j.L * e * W * 4;
  }
  const int ph = ctx->prof.begin(st);
  launch_persist(k, a, n_blocks, st);
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
  for (auto& j : jobs) macs += (uint64_t)(j.L * j.plan->macs);
  ctx->last_macs += macs;
}

}  // namespace bbtn
