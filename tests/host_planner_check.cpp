// Host-only driver for the planner under AddressSanitizer and
// UndefinedBehaviorSanitizer (built by tests/test_host_sanitized.py with g++,
// no device code): reads an instance, chooses the contraction order (greedy
// or refined), runs the branch-and-bound search and builds the step program
// of every leaf group, with and without deferred slicing and keep-all.
//
// Input file: kind n m log2_target order_refine values_only, then m lines
// "u v w" (spin glass: w = J) and, for kind 1, n vertex weights.
#include <cstdio>
#include <vector>

#include "network.h"
#include "plan.h"
#include "scorer.h"
#include "search.h"
#include "tree.h"

namespace bbtn {
// the learned scorer's features are not used by the plain planner
FeatureCtx::FeatureCtx(const Network&, const Tree&, int) {}
void FeatureCtx::features(int, const std::vector<uint64_t>&, const std::vector<int16_t>&,
                          const std::vector<double>&, int64_t, float*) const {}
}  // namespace bbtn

int main(int argc, char** argv) {
  using namespace bbtn;
  if (argc != 2) return 2;
  FILE* f = std::fopen(argv[1], "r");
  if (!f) return 2;
  int kind, n, m, lt, refine, vonly;
  if (std::fscanf(f, "%d %d %d %d %d %d", &kind, &n, &m, &lt, &refine, &vonly) != 6) return 2;
  std::vector<int32_t> uv(2 * (size_t)m), w(m), vw(n, 1);
  for (int i = 0; i < m; ++i)
    if (std::fscanf(f, "%d %d %d", &uv[2 * i], &uv[2 * i + 1], &w[i]) != 3) return 2;
  if (kind == 1)
    for (int i = 0; i < n; ++i)
      if (std::fscanf(f, "%d", &vw[i]) != 1) return 2;
  std::fclose(f);
  Network net = kind == 0 ? build_spinglass(n, m, uv.data(), w.data(), nullptr)
                          : build_mwis(n, m, uv.data(), vw.data());
  SearchOptions so;
  so.log2_target = lt;
  so.region_max = 8;
  so.values_only = vonly != 0;
  const Tree t = choose_order(net, refine, so);
  std::vector<LeafGroup> groups;
  SearchStats st;
  bb_search(net, t, so, groups, st);
  int64_t leaves = 0, steps = 0;
  for (const auto& g : groups) {
    leaves += g.count;
    steps += (int64_t)build_plan(net, t, g.mask, false, lt).steps.size();
    steps += (int64_t)build_plan(net, t, g.mask, false, 0).steps.size();
    steps += (int64_t)build_plan(net, t, g.mask, true, 0).steps.size();
  }
  std::printf("ok groups %zu leaves %lld steps %lld\n", groups.size(), (long long)leaves,
              (long long)steps);
  return 0;
}
