// Per-kernel timing with HIP events recorded on the launch stream around
// every launch of the instrumented kernels (enabled per context).
#pragma once
#include <vector>
#include "common.h"

struct bbtn_ctx;

namespace bbtn {

enum KernelId { K_TGEMM = 0, K_PERSIST = 1, K_GATHER = 2, K_REDUCE = 3, K_COUNT = 4 };

struct KStat {
  uint64_t launches = 0;
  double seconds = 0;
  double ops = 0;    // algorithmic semiring operations
  double bytes = 0;  // algorithmic bytes (operands in + results out)
};

struct Prof {
  bool on = false;
  KStat stat[K_COUNT];
  struct Pending {
    int id;
    hipEvent_t a, b;
    double ops, bytes;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  hipEvent_t get();
  // bracket a launch: begin() before, end() after
  int begin(hipStream_t st);
  void end(int h, hipStream_t st, int id, double ops, double bytes);
  void resolve();  // after a stream synchronisation
  void clear();
  ~Prof();
};

Prof& prof_of(bbtn_ctx* ctx);

}  // namespace bbtn
