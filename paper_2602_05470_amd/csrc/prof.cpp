#include "prof.h"

#include "ctx.h"
#include "kernels.h"

namespace bbtn {

hipEvent_t Prof::get() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e;
  BBTN_HIP(hipEventCreate(&e));
  return e;
}

TimedLaunch& timed_launch() {
  static thread_local TimedLaunch slot;
  return slot;
}

int Prof::begin(hipStream_t st, int id) {
  if (!on || id < 0 || id >= K_COUNT || !(mask >> id & 1)) return -1;
  Pending p{};
  p.a = get();
  p.b = get();
  p.ext = id != K_PERSIST;
  if (p.ext) {
    timed_launch() = TimedLaunch{p.a, p.b};
  } else {
    BBTN_HIP(hipEventRecord(p.a, st));
  }
  pending.push_back(p);
  return (int)pending.size() - 1;
}

void Prof::end(int h, hipStream_t st, int id, double ops, double bytes) {
  if (h < 0) return;
  Pending& p = pending[h];
  p.id = id;
  p.ops = ops;
  p.bytes = bytes;
  if (p.ext) {
    // a launch path that did not take the events (none should): record
    // what is left on the stream, so the pair stays valid
    TimedLaunch& t = timed_launch();
    if (t.start) BBTN_HIP(hipEventRecord(t.start, st));
    if (t.stop) BBTN_HIP(hipEventRecord(t.stop, st));
    t = TimedLaunch{};
  } else {
    BBTN_HIP(hipEventRecord(p.b, st));
  }
}

void Prof::resolve() {
  for (auto& p : pending) {
    float ms = 0;
    // a pair left unrecorded by a launch that failed is counted as 0 s
    if (hipEventSynchronize(p.b) != hipSuccess || hipEventElapsedTime(&ms, p.a, p.b) != hipSuccess) {
      ms = 0;
      (void)hipGetLastError();
    }
    KStat& s = stat[p.id];
    s.launches++;
    s.seconds += ms * 1e-3;
    s.ops += p.ops;
    s.bytes += p.bytes;
    pool.push_back(p.a);
    pool.push_back(p.b);
  }
  pending.clear();
}

void Prof::clear() {
  resolve();
  for (auto& s : stat) s = KStat{};
}

Prof::~Prof() {
  for (auto& p : pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
  for (auto e : pool) (void)hipEventDestroy(e);
}

Prof& prof_of(bbtn_ctx* ctx) { return ctx->prof; }

}  // namespace bbtn
