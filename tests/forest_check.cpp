// Host-only check of the small-step forests (built by tests/test_forest_cpu.py
// with g++, no device code): for every leaf group of an instance, the
// forest planned for the step program (and, in place, for the keep-all
// program of configuration recovery) is run on the host with the
// executor's addressing rules (operand kinds, offsets, plane strides,
// per-bit source tables, materialised operands), values only, and every
// buffer it produces is compared with a per-buffer contraction of the same
// steps.  Every offset is bounds-checked against its region.
//
// Input file: kind n m log2_target order_refine values_only, then m lines
// "u v w" (spin glass: w = J) and, for kind 1, n vertex weights.
#include <algorithm>
#include <cstdlib>
#include <cstdio>
#include <map>
#include <random>
#include <vector>

#include "network.h"
#include "persist.h"
#include "plan.h"
#include "scorer.h"
#include "search.h"
#include "tree.h"

namespace bbtn {
FeatureCtx::FeatureCtx(const Network&, const Tree&, int) {}
void FeatureCtx::features(int, const std::vector<uint64_t>&, const std::vector<int16_t>&,
                          const std::vector<double>&, int64_t, float*) const {}
// device-side pieces the planner links against (never called here)
void launch_persist(int, const PersistArgs&, int, int, hipStream_t) {}
void leaf_constants(const Network&, const GroupPlan&, const int*, int, const uint8_t*, int64_t,
                    std::vector<uint32_t>&) {}
// LDS bytes of an executor workgroup (the executor's own formula)
size_t persist_lds_bytes(int k, int64_t lds_entries, int64_t arena_entries, int threads,
                         int slots) {
  return (size_t)(2 * lds_entries + arena_entries) * (1 + k) * 4 +
         (size_t)threads * 4 * (1 + k) + (size_t)slots * 4;
}
}  // namespace bbtn

using namespace bbtn;
static const int32_t NEGV = -(1 << 30);
static int failures = 0;
#define CHECK(c, ...)                       \
  do {                                      \
    if (!(c)) {                             \
      if (failures++ < 10) {                \
        std::printf("FAIL: " __VA_ARGS__);  \
        std::printf("\n");                  \
      }                                     \
    }                                       \
  } while (0)

// C[b,m,n] = max_q A[b,m,q] + B[b,q,n] in the product layouts
static std::vector<int32_t> product(int rb, int rm, int rn, int rk, const std::vector<int32_t>& A,
                                    const std::vector<int32_t>& B) {
  std::vector<int32_t> C(size_t(1) << (rb + rm + rn), NEGV);
  for (int b = 0; b < (1 << rb); ++b)
    for (int m = 0; m < (1 << rm); ++m)
      for (int n = 0; n < (1 << rn); ++n) {
        int32_t v = INT32_MIN;
        for (int q = 0; q < (1 << rk); ++q)
          v = std::max(v, A[q | (m << rk) | (b << (rk + rm))] + B[n | (q << rn) | (b << (rn + rk))]);
        C[n | (m << rn) | (b << (rn + rm))] = v > -(1 << 29) ? v : NEGV;
      }
  return C;
}

static std::vector<int32_t> gather(const int32_t* src, int64_t src_n, const std::vector<int32_t>& bits) {
  std::vector<int32_t> o(size_t(1) << bits.size());
  for (int64_t e = 0; e < (int64_t)o.size(); ++e) {
    int64_t s = 0;
    for (size_t j = 0; j < bits.size(); ++j) s |= ((e >> j) & 1) << bits[j];
    CHECK(s < src_n, "source index %lld out of %lld", (long long)s, (long long)src_n);
    o[e] = s < src_n ? src[s] : 0;
  }
  return o;
}

static void check_forest(const Network& net, const GroupPlan& g, int k, int64_t L,
                         const std::vector<int64_t>& off, const std::vector<int32_t>& base) {
  const SmallForest f = plan_small_forest(g, off, k, L);
  if (f.tasks.empty()) return;
  if (getenv("FOREST_VERBOSE")) std::printf("forest k=%d L=%lld in_place=%d tasks %zu steps %zu\n", k, (long long)L, (int)f.in_place, f.tasks.size(), f.steps.size());
  const int W = 1 + k;
  const int64_t total = (int64_t)base.size();
  // per-buffer truth for the forest steps (and their gathered operands)
  std::map<int, std::vector<int32_t>> truth, temps;
  for (size_t si = 0; si < g.steps.size(); ++si) {
    if (!f.in[si]) continue;
    const Step& s = g.steps[si];
    std::vector<int32_t> op[2];
    const Operand* ops[2] = {&s.a, &s.b};
    for (int w = 0; w < 2; ++w) {
      const Operand& o = *ops[w];
      CHECK(o.fixed_pos.empty(), "forest step reads sliced operand");
      if (o.base) op[w] = gather(base.data() + off[o.id], total - off[o.id], o.src_bits);
      else op[w] = gather(truth.at(o.id).data(), (int64_t)truth.at(o.id).size(), o.src_bits);
      if (o.temp >= 0) temps[o.temp] = op[w];
    }
    truth[s.out] = product(s.rb, s.rm, s.rn, s.rk, op[0], op[1]);
  }
  // the forest program with the executor's addressing
  const int64_t scr_n = f.in_place ? g.peak : std::max<int64_t>(f.scratch_entries, 1);
  std::vector<int32_t> root((size_t)W * std::max<int64_t>(f.root_entries, 1), 12345);
  std::vector<int32_t> ws;  // in place: the program's workspace (W = 1)
  if (f.in_place) ws.assign((size_t)g.peak, 777);
  for (const PTask& tk : f.tasks) {
    std::vector<int32_t> scr_own((size_t)W * scr_n, 777);
    std::vector<int32_t>& scr = f.in_place ? ws : scr_own;
    for (int j = 0; j < tk.n_steps; ++j) {
      const PStep& ps = f.steps[tk.step_off + j];
      std::vector<int32_t> op[2];
      const POperand* pops[2] = {&ps.a, &ps.b};
      for (int w = 0; w < 2; ++w) {
        const POperand& po = *pops[w];
        CHECK(po.rank <= f.max_rank, "operand rank over the staging size");
        std::vector<int32_t> bits(po.rank);
        for (int q = 0; q < po.rank; ++q) bits[q] = (po.bitpos[q / 4] >> (8 * (q % 4))) & 255;
        if (po.kind == PK_BASE) {
          op[w] = gather(base.data() + po.src_off, total - po.src_off, bits);
        } else if (po.kind == PK_SCRATCH) {
          CHECK(po.src_off >= 0 && po.src_off < scr_n, "scratch operand offset");
          op[w] = gather(scr.data() + po.src_off, scr_n - po.src_off, bits);
        } else {
          CHECK(false, "operand kind %d", po.kind);
        }
        if (po.mat_off >= 0) {
          CHECK(po.mat_off + (int64_t)op[w].size() <= scr_n, "materialised operand out of range");
          std::copy(op[w].begin(), op[w].end(), scr.begin() + po.mat_off);
        }
      }
      const auto C = product(ps.rb, ps.rm, ps.rn, ps.rk, op[0], op[1]);
      if (ps.c_kind == PK_SHARED) {
        CHECK(ps.c_stride == (int64_t)C.size(), "root plane stride");
        CHECK(ps.c_off + (int64_t)W * (int64_t)C.size() <= (int64_t)root.size(), "root out of range");
        if (ps.c_off + (int64_t)C.size() <= (int64_t)root.size())
          std::copy(C.begin(), C.end(), root.begin() + ps.c_off);
      } else {
        CHECK(ps.c_kind == PK_SCRATCH, "output kind %d", ps.c_kind);
        CHECK(ps.c_off >= 0 && ps.c_off + (int64_t)C.size() <= scr_n, "output out of range");
        if (ps.c_off + (int64_t)C.size() <= scr_n) std::copy(C.begin(), C.end(), scr.begin() + ps.c_off);
      }
    }
  }
  if (f.in_place) {
    // every forest output and every materialised operand at its own buffer
    for (auto& kv : truth)
      for (size_t e = 0; e < kv.second.size(); ++e)
        CHECK(ws[g.buf_off[kv.first] + e] == kv.second[e], "in-place buffer %d entry %zu", kv.first, e);
    for (auto& kv : temps)
      for (size_t e = 0; e < kv.second.size(); ++e)
        CHECK(ws[g.buf_off[kv.first] + e] == kv.second[e], "materialised operand %d entry %zu", kv.first, e);
  } else {
    for (size_t id = 0; id < f.root_off.size(); ++id) {
      if (f.root_off[id] < 0) continue;
      const auto& T = truth.at((int)id);
      for (size_t e = 0; e < T.size(); ++e)
        CHECK(root[(size_t)W * f.root_off[id] + e] == T[e], "root %zu entry %zu", id, e);
    }
  }
}

int main(int argc, char** argv) {
  if (argc != 2) return 2;
  FILE* fp = std::fopen(argv[1], "r");
  if (!fp) return 2;
  int kind, n, m, lt, refine, vonly;
  if (std::fscanf(fp, "%d %d %d %d %d %d", &kind, &n, &m, &lt, &refine, &vonly) != 6) return 2;
  std::vector<int32_t> uv(2 * (size_t)m), w(m), vw(n, 1);
  for (int i = 0; i < m; ++i)
    if (std::fscanf(fp, "%d %d %d", &uv[2 * i], &uv[2 * i + 1], &w[i]) != 3) return 2;
  if (kind == 1)
    for (int i = 0; i < n; ++i)
      if (std::fscanf(fp, "%d", &vw[i]) != 1) return 2;
  std::fclose(fp);
  Network net = kind == 0 ? build_spinglass(n, m, uv.data(), w.data(), nullptr)
                          : build_mwis(n, m, uv.data(), vw.data());
  SearchOptions so;
  so.log2_target = lt;
  so.region_max = 8;
  const Tree t = choose_order(net, refine, so);
  std::vector<LeafGroup> groups;
  SearchStats st;
  bb_search(net, t, so, groups, st);
  std::vector<int64_t> off(net.tensors.size());
  int64_t total = 0;
  for (size_t i = 0; i < net.tensors.size(); ++i) { off[i] = total; total += net.tensors[i].size(); }
  std::mt19937 rng(7);
  std::vector<int32_t> base(std::max<int64_t>(total, 1));
  for (auto& x : base) x = (int32_t)(rng() % 9) - 4;
  int forests = 0;
  for (const auto& G : groups) {
    const GroupPlan g = build_plan(net, t, G.mask, false, lt);
    for (int k : {0, 3})
      for (int64_t L : {(int64_t)G.count, (int64_t)1}) {
        check_forest(net, g, k, L, off, base);
        ++forests;
      }
    const GroupPlan ka = build_plan(net, t, G.mask, true, 0);
    check_forest(net, ka, 0, 1, off, base);
    ++forests;
  }
  if (failures) { std::printf("failures %d\n", failures); return 1; }
  std::printf("ok groups %zu forests %d\n", groups.size(), forests);
  return 0;
}
