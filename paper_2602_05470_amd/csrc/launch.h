// Kernel launches that take the profiler's timing events (see TimedLaunch
// in kernels.h).  Included by the kernel sources only.
#pragma once
#include <hip/hip_ext.h>
#include "kernels.h"

namespace bbtn {

// Launch `kernel`; `last` marks the final kernel of the operation being
// timed (it takes the stop event).
template <class F, class... Args>
inline void launch_kernel(F kernel, dim3 grid, dim3 block, uint32_t shm, hipStream_t st,
                          bool last, Args... args) {
  TimedLaunch& t = timed_launch();
  hipEvent_t a = t.start, b = last ? t.stop : nullptr;
  if (a || b) {
    t.start = nullptr;
    if (last) t.stop = nullptr;
    hipExtLaunchKernelGGL(kernel, grid, block, shm, st, a, b, 0u, args...);
  } else {
    hipLaunchKernelGGL(kernel, grid, block, shm, st, args...);
  }
}

}  // namespace bbtn
