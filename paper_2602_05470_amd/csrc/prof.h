// Per-kernel timing with HIP events recorded on the launch stream around
// every launch of the instrumented kernels (enabled per context).
#pragma once
#include <vector>
#include "common.h"

struct bbtn_ctx;

namespace bbtn {

enum KernelId { K_TGEMM = 0, K_PERSIST = 1, K_GATHER = 2, K_REDUCE = 3, K_THIN = 4, K_COUNT = 5 };

struct KStat {
  uint64_t launches = 0;
  double seconds = 0;
  double ops = 0;    // algorithmic semiring operations
  double bytes = 0;  // algorithmic bytes (operands in + results out)
};

struct Prof {
  bool on = false;
  uint32_t mask = ~0u;  // kernel ids timed while on (bit i: kernel i)
  KStat stat[K_COUNT];
  struct Pending {
    int id;
    hipEvent_t a, b;
    double ops, bytes;
    bool ext;  // events taken by the kernel launches themselves
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  hipEvent_t get();
  // bracket a launch of kernel `id`: begin() before, end() after (a
  // kernel outside the mask is not timed: begin returns -1).  Products and
  // gathers hand their events to the kernel launches (launch_kernel in
  // kernels.h); the executor pass records them on the stream around its
  // dispatches.
  int begin(hipStream_t st, int id);
  void end(int h, hipStream_t st, int id, double ops, double bytes);
  void resolve();  // after a stream synchronisation
  void clear();
  ~Prof();
};

Prof& prof_of(bbtn_ctx* ctx);

}  // namespace bbtn
