// Host-side launchers of the HIP kernels.  All launches are asynchronous on
// the given stream; shapes are validated by the callers.
#pragma once
#include "common.h"

namespace bbtn {

// Events of the launch being timed.  Before a timed product, gather or
// executor pass the profiler leaves a start and a stop event here; the first
// kernel launched takes the start event and the last one the stop event
// (hipExtLaunchKernel), so the interval is that of the kernels' own
// dispatches, not of markers queued between other kernels.
struct TimedLaunch {
  hipEvent_t start = nullptr, stop = nullptr;
};
TimedLaunch& timed_launch();  // this host thread's slot (launch_kernel in launch.h)

// Tile shape of the counting tropical GEMM: TM x TN outputs per workgroup,
// RM x RN per thread, TK-deep LDS stages.
struct TileCfg {
  int tm, tn, rm, rn, tk;
};
constexpr int N_TILE_CFGS = 13;
extern const TileCfg kTileCfgs[N_TILE_CFGS];

struct GemmShape {
  int64_t batch, M, N, K;
  // element strides between consecutive batch entries of A, B, C (0 =
  // operand shared by every batch entry); rows are contiguous.
  int64_t sAb, sBb, sCb;
};

// C[b,m,n] = (+)_q A[b,m,q] (.) B[b,q,n].  With splits > 1 the K range is cut
// into `splits` chunks whose partial results go to `partial` (a tensor buffer
// of splits * batch * M * N entries) and are merged into C afterwards.
void launch_tgemm(int k, const Moduli& mod, const GemmShape& s, DevTensor A,
                  DevTensor B, DevTensor C, int cfg, int splits,
                  DevTensor partial, hipStream_t st);

// True when launch_tgemm runs the product with the thin kernel (one thread
// per output, no LDS): unsplit, power-of-two sizes, K <= 32 and M or N
// below 32.
bool tgemm_is_thin(const GemmShape& s, int splits);

// Values-only product (k = 0) with two values per 32-bit word, for operands
// whose finite values all satisfy |v| < 2^12 (the caller guarantees it):
// half the VALU instructions per multiply-accumulate.  Same layouts, split-K
// and partial buffer as launch_tgemm with k = 0.
void launch_tgemm_values16(const GemmShape& s, DevTensor A, DevTensor B, DevTensor C,
                           int splits, DevTensor partial, hipStream_t st);
constexpr int64_t kValues16Bound = 1 << 12;  // |v| below this for the packed path

// Operand read through a bit permutation instead of a gathered copy: entry
// e of the operand's product layout ([K][M][batch] for A, [N][K][batch] for
// B) is source entry l * stride + perm(e) of branch l = batch index >> rb,
// where perm moves bit j of e to bit bits[j] (a bijection of the operand's
// bits; OR-linear over disjoint bit sets, so perm(m0 + i) = perm(m0) |
// perm(i) for tile-aligned m0).  `fast` = 1 when lanes should walk the
// row index (m for A, n for B) to read consecutive source words, 0 when they
// should walk k.
struct FusedOp {
  const uint32_t* src;
  int64_t stride;      // entries between branches (0: one tensor for all)
  int32_t rb;          // batch bits of the operand per branch
  int32_t fast;
  int8_t bits[40];     // source bit of layout bit j
};

// The packed values product (k = 0, |v| < kValues16Bound) with one or both
// operands read through FusedOp instead of A / B (whose pointers are then
// unused for that operand); power-of-two M, N, K, unsplit.
void launch_tgemm_values16_fused(const GemmShape& s, const FusedOp* fa, DevTensor A,
                                 const FusedOp* fb, DevTensor B, DevTensor C, hipStream_t st);

// Entries of the split-K partial buffer launch_tgemm needs for `splits`
// chunks of K with tile config `cfg` and outer = batch * M * N outputs (0 when
// the product runs unsplit).
int64_t tgemm_partial_entries(int cfg, int splits, int64_t K, int64_t outer);

// Device scratch of the allocation-free product: a static device array of
// kNoAllocScratchWords words per device.  noalloc_scratch_init(d), called
// once per device with d current, looks up the array's address on d;
// noalloc_scratch(d) returns it (nullptr before set-up).
constexpr int64_t kNoAllocScratchWords = 1ll << 24;
void noalloc_scratch_init(int device);
uint32_t* noalloc_scratch(int device);

// Values-only variant (k = 0): the max-plus product used for bounds and
// configuration recovery.
void launch_tgemm_values(const GemmShape& s, const int32_t* A, const int32_t* B,
                         int32_t* C, hipStream_t st);

// Bit-permutation / slicing gather (see bbtn_gather in bbtn.h).
struct GatherRun {
  int32_t out_lo, in_lo, len;
};
constexpr int MAX_RUNS = 40;
struct GatherPlan {
  int32_t r_out = 0, r_in = 0;
  int32_t n_runs = 0;
  GatherRun runs[MAX_RUNS];
  uint64_t fixed_mask = 0;  // input bits not covered by runs
};
GatherPlan make_gather_plan(int r_in, int r_out, const int32_t* src_bits);
void launch_gather(int k, const GatherPlan& g, int64_t L, int64_t in_stride,
                   const uint64_t* fixed_bits, DevTensor in, DevTensor out,
                   hipStream_t st);

// Segmented tropical sum: out[o] = (+)_{s<S} in[s*seg_stride + o*elem_stride].
void launch_reduce(int k, const Moduli& mod, int64_t outer, int64_t S,
                   int64_t seg_stride, int64_t elem_stride, DevTensor in,
                   DevTensor out, hipStream_t st);

// out[l] = a[l] (.) b[l] for l < L.
void launch_otimes(int k, const Moduli& mod, int64_t L, DevTensor a, DevTensor b,
                   DevTensor out, hipStream_t st);

// Branch bounds + stream compaction (see bbtn_bound in bbtn.h).  `flags`
// is device scratch of n_branch int32.
void launch_bound(int64_t n_branch, int32_t T, const int32_t* values,
                  const int64_t* off, const int32_t* len, const int64_t* offset,
                  int64_t incumbent, int64_t* bound, int32_t* flags,
                  int32_t* keep_idx, int32_t* n_keep, hipStream_t st);

}  // namespace bbtn
