// The opaque context behind bbtn_ctx: device, stream, workspace, caches.
#pragma once
#include <atomic>
#include <future>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include "common.h"
#include "prof.h"
#include "plan.h"
#include "tree.h"

namespace bbtn {

// Device bytes held by a context and its recovery context, against the
// option device_mem_cap (0: no cap).
struct MemCap {
  size_t cap = 0;
  std::atomic<size_t> held{0};
};

// Growable device allocation (contents are not preserved on growth).
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  MemCap* mc = nullptr;  // the owning context's account, or none
  void ensure(size_t b) {
    if (b <= bytes) return;
    size_t want = std::max<size_t>(b, 1 << 20);
    if (mc && mc->cap > 0 && mc->held.load() - bytes + want > mc->cap)
      throw Error(BBTN_E_OOM, "device_mem_cap of " + std::to_string(mc->cap) +
                                  " bytes reached (" + std::to_string(want) +
                                  " more bytes wanted)");
    release();
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      throw Error(BBTN_E_OOM, "device allocation of " + std::to_string(want) + " bytes failed");
    }
    bytes = want;
    if (mc) mc->held += want;
  }
  void release() {
    if (p) (void)hipFree(p);
    if (mc) mc->held -= bytes;
    p = nullptr;
    bytes = 0;
  }
  template <class T>
  T* as() const { return (T*)p; }
};

// Growable pinned host staging buffer for host-to-device uploads (contents
// are not preserved on growth).  The caller keeps it untouched until the
// copies queued from it have completed.
struct PinBuf {
  void* p = nullptr;
  size_t bytes = 0;
  void ensure(size_t b) {
    if (b <= bytes) return;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
    size_t want = std::max<size_t>(b + b / 4, 1 << 20);
    if (hipHostMalloc(&p, want, hipHostMallocDefault) != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      throw Error(BBTN_E_OOM, "pinned host allocation of " + std::to_string(want) + " bytes failed");
    }
    bytes = want;
  }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <class T>
  T* as() const { return (T*)p; }
};

// Captured step programs: keyed by the program, its batch, residues, every
// device pointer the launches bake in, the base tensors' offsets (a hash:
// instances of one structure share a program but not their offsets) and
// whether the shared steps are skipped (chunks after a pass's first).
using GraphKey = std::tuple<const void*, int64_t, int, void*, void*, void*, void*, void*, void*,
                            uint32_t, void*, void*, uint64_t, bool>;

// Autotuner key: residues, log2 of (batch, M, N, K) buckets.
using TuneKey = std::tuple<int, int, int, int, int>;
struct TuneVal {
  int cfg;
  int splits;
};

// A contraction tree from a context's cache, with its cache id.
struct TreeRef {
  std::shared_ptr<const Tree> tree;
  uint64_t id = 0;
};

}  // namespace bbtn

struct bbtn_ctx {
  bbtn_options opt;
  std::string err;
  hipStream_t own = nullptr;
  hipStream_t stream = nullptr;
  bbtn::DevBuf work;      // step-program workspace
  bbtn::DevBuf shared_ws; // shared subtrees of the step-program workspace
  bbtn::DevBuf partial;   // split-K partials
  bbtn::DevBuf base;      // base tensors of the current pass
  bbtn::DevBuf fixbits;   // per-branch fixed bits of base operands
  bbtn::DevBuf leafconst; // per-branch folded constants
  bbtn::DevBuf leafout;   // per-branch results
  bbtn::DevBuf misc;      // small scratch (merge outputs, traceback)
  bbtn::DevBuf persist;   // persistent executor programs and scratch
  bbtn::DevBuf forest;    // small-step forests: root region, scratch, program
  // account of the device bytes above, shared with the recovery context
  std::shared_ptr<bbtn::MemCap> memcap = std::make_shared<bbtn::MemCap>();
  void attach_memcap(std::shared_ptr<bbtn::MemCap> m) {
    memcap = std::move(m);
    for (bbtn::DevBuf* b : {&work, &shared_ws, &partial, &base, &fixbits, &leafconst, &leafout,
                            &misc, &persist, &forest, &scorer_dev})
      b->mc = memcap.get();
  }
  bbtn::PinBuf pin_base;    // staging of the base tensors of a pass
  bbtn::PinBuf pin_persist; // staging of a persistent launch's program
  uint64_t last_macs = 0;
  std::map<bbtn::TuneKey, bbtn::TuneVal> tune;
  bool tune_loaded = false;
  // learned scorer: [fmean 32][fstd 32][ymean][ystd][params] (host) and the
  // device copy [bf16 weights][f32 biases][rows x 32 bf16 inputs][rows f32 out]
  std::vector<float> scorer_model;
  bool scorer_loaded = false;
  bbtn::DevBuf scorer_dev;
  bbtn::Prof prof;         // kernel timing (off unless enabled)
  std::map<bbtn::GraphKey, hipGraphExec_t> graphs;
  // contraction trees by network structure (the variable lists of the
  // simplified tensors, which do not depend on couplings or weights)
  struct TreeEntry {
    std::shared_ptr<const bbtn::Tree> tree;
    uint64_t id;  // unique over the process
  };
  std::map<std::vector<std::vector<int32_t>>, TreeEntry> tree_cache;
  // ranked candidate orders by structure (order_candidates / order_use)
  std::map<std::vector<std::vector<int32_t>>, std::vector<std::shared_ptr<const bbtn::Tree>>>
      order_cands;
  // step programs by (tree id, keep-all, fixed set): they depend on the
  // network's structure and the fixed variables only
  std::map<std::tuple<uint64_t, bool, std::vector<uint64_t>>,
           std::shared_ptr<const bbtn::GroupPlan>>
      plan_cache;
  std::mutex tree_mu;  // planning threads share both caches
  // refined orders being built, by structure (waited on by other threads)
  std::map<std::vector<std::vector<int32_t>>, std::shared_future<bbtn::TreeRef>> tree_building;
  // second context (own stream and workspaces) that recovers the optimal
  // configuration while this one runs the counting passes
  bbtn_ctx* aux = nullptr;
  void clear_graphs() {
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    graphs.clear();
  }
};
