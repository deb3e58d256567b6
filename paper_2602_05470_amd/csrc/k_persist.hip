// Persistent work-queue executor for branch sub-networks whose tensors fit
// in LDS.  One launch contracts every queued branch of every group: a
// workgroup pops a task (a branch and its group's step program) from a device
// counter, and runs the program's steps in order.  Per step it
//   1. stages both operands into LDS in the layout the step needs, reading
//      base tensors sliced by the branch's fixed states (T|_{s_S = x},
//      Eq. 3) or earlier intermediates from the workgroup's global scratch
//      through the step's bit-permutation runs;
//   2. forms C = A (.) B summed over the step's contracted variables (Eq. 2
//      pairwise, counting tropical algebra), with the K range split over
//      several threads when the output is small, and writes C to scratch.
// The root scalar (.) the branch's folded constant is the branch's result.
// A program built to keep every intermediate also writes each staged operand
// to scratch (configuration recovery reads them afterwards).
// Counts use the same lazy 64-bit accumulation as the tiled product.
#include "persist_dev.h"

namespace bbtn {

namespace {

__device__ __forceinline__ uint64_t pfold(uint64_t x, uint32_t c) {
  return (uint64_t)(uint32_t)(x >> 32) * c + (uint32_t)x;
}
__device__ __forceinline__ uint32_t pmod(uint64_t x, uint32_t p, uint32_t c) {
  x = pfold(x, c);
  x = pfold(x, c);
  x = pfold(x, c);
  x = pfold(x, c);
  x = x >= p ? x - p : x;
  x = x >= p ? x - p : x;
  return (uint32_t)x;
}

template <int KR>
__device__ __forceinline__ void combine(int32_t& v, uint32_t* r, int32_t v2, const uint32_t* r2,
                                        const Moduli& m) {
  if (v2 > v) {
    v = v2;
#pragma unroll
    for (int p = 0; p < KR; ++p) r[p] = r2[p];
  } else if (v2 == v) {
#pragma unroll
    for (int p = 0; p < KR; ++p) {
      const uint32_t s = r[p] + r2[p];
      r[p] = s >= m.p[p] ? s - m.p[p] : s;
    }
  }
}

constexpr int NTHR = 256;

template <int KR>
__global__ void __launch_bounds__(NTHR)
persist_kernel(const PersistArgs a) {
  constexpr int W = 1 + KR;
  extern __shared__ uint32_t lds[];
  const int64_t cap = a.lds_entries;  // entries per operand buffer
  uint32_t* la = lds;                 // W planes of cap entries
  uint32_t* lb = lds + W * cap;
  int32_t* pv = (int32_t*)(lb + W * cap);  // NTHR partial values
  uint32_t* pr = (uint32_t*)(pv + NTHR);   // KR x NTHR partial residues
  __shared__ int64_t s_task;
  uint32_t* scr = a.scratch + (int64_t)blockIdx.x * W * a.scratch_entries;
  const int tid = threadIdx.x;

  for (;;) {
    if (tid == 0) s_task = atomicAdd(a.queue, 1ull);
    __syncthreads();
    const int64_t task = s_task;
    __syncthreads();
    if (task >= a.n_tasks) break;
    const PTask tk = a.tasks[task];
    const uint8_t* asg = a.assign + tk.assign_off;

    for (int32_t si = 0; si < tk.n_steps; ++si) {
      const PStep st = a.steps[tk.step_off + si];
      // ---- stage operands
#pragma unroll
      for (int w = 0; w < 2; ++w) {
        const POperand& op = w == 0 ? st.a : st.b;
        uint32_t* dst = w == 0 ? la : lb;
        uint64_t fixed = 0;
        for (int f = 0; f < op.n_fix; ++f) {
          const PFix fx = a.fixes[op.fix_off + f];
          fixed |= (uint64_t)(asg[fx.idx] & 1) << fx.pos;
        }
        const uint32_t* src = op.kind == PK_BASE     ? a.base + op.src_off
                              : op.kind == PK_SHARED ? a.shared + op.src_off
                                                     : scr + op.src_off;
        const int64_t sstride = op.kind == PK_BASE     ? a.base_total
                                : op.kind == PK_SHARED ? a.shared_entries
                                                       : a.scratch_entries;
        const int64_t n = 1ll << op.rank;
        for (int64_t e = tid; e < n; e += NTHR) {
          uint64_t s = fixed;
          for (int r = 0; r < op.n_runs; ++r) {
            const GatherRun run = op.runs[r];
            s |= (((uint64_t)e >> run.out_lo) & ((1ull << run.len) - 1)) << run.in_lo;
          }
#pragma unroll
          for (int p = 0; p < W; ++p) {
            const uint32_t x = src[p * sstride + s];
            dst[p * cap + e] = x;
            if (op.mat_off >= 0) scr[p * a.scratch_entries + op.mat_off + e] = x;
          }
        }
      }
      __syncthreads();
      // ---- product
      const int rn = st.rn, rm = st.rm, rk = st.rk;
      const int64_t nC = 1ll << (st.rb + rm + rn);
      const int64_t K = 1ll << rk;
      // threads per output: split K when outputs are few
      int tpo = 1;
      while (tpo * 2 <= NTHR / nC && tpo * 2 <= K) tpo *= 2;
      const int64_t kper = K / tpo;
      const int64_t per_round = NTHR / tpo;
      for (int64_t o0 = 0; o0 < nC; o0 += per_round) {
        const int64_t o = o0 + tid / tpo;
        const int j = tid % tpo;
        int32_t V = INT32_MIN;
        uint32_t res[KR > 0 ? KR : 1];
        if (o < nC) {
          const int64_t n = o & ((1ll << rn) - 1);
          const int64_t m = (o >> rn) & ((1ll << rm) - 1);
          const int64_t b = o >> (rn + rm);
          const int64_t abase = (m << rk) | (b << (rk + rm));
          const int64_t bbase = n | (b << (rn + rk));
          const int64_t q0 = j * kper, q1 = q0 + kper;
          const int32_t* Av = (const int32_t*)la;
          const int32_t* Bv = (const int32_t*)lb;
          for (int64_t q = q0; q < q1; ++q) V = max(V, Av[abase + q] + Bv[bbase + (q << rn)]);
          if constexpr (KR > 0) {
            uint64_t acc[KR];
#pragma unroll
            for (int p = 0; p < KR; ++p) acc[p] = 0;
            if (V > NEG_CUT) {
              int cnt = 0;
              for (int64_t q = q0; q < q1; ++q) {
                const int64_t ia = abase + q, ib = bbase + (q << rn);
                if (Av[ia] + Bv[ib] == V) {
#pragma unroll
                  for (int p = 0; p < KR; ++p)
                    acc[p] += (uint64_t)la[(p + 1) * cap + ia] * lb[(p + 1) * cap + ib];
                  if (++cnt == 3) {
                    cnt = 0;
#pragma unroll
                    for (int p = 0; p < KR; ++p) acc[p] = pfold(acc[p], a.mod.c[p]);
                  }
                }
              }
            }
#pragma unroll
            for (int p = 0; p < KR; ++p) res[p] = pmod(acc[p], a.mod.p[p], a.mod.c[p]);
          }
        }
        if (tpo > 1) {
          pv[tid] = V;
#pragma unroll
          for (int p = 0; p < KR; ++p) pr[p * NTHR + tid] = res[p];
          __syncthreads();
          if (j == 0 && o < nC) {
            for (int t = 1; t < tpo; ++t) {
              uint32_t r2[KR > 0 ? KR : 1];
#pragma unroll
              for (int p = 0; p < KR; ++p) r2[p] = pr[p * NTHR + tid + t];
              combine<KR>(V, res, pv[tid + t], r2, a.mod);
            }
          }
          __syncthreads();
        }
        if (j == 0 && o < nC) {
          const bool fin = V > NEG_CUT;
          const bool sh = st.c_kind == PK_SHARED;
          uint32_t* c = (sh ? a.shared : scr) + st.c_off;
          const int64_t cs = sh ? a.shared_entries : a.scratch_entries;
          c[o] = (uint32_t)(fin ? V : NEG);
#pragma unroll
          for (int p = 0; p < KR; ++p) c[(p + 1) * cs + o] = fin ? res[p] : 0u;
        }
      }
      __syncthreads();
    }
    // ---- branch result = root (.) folded constant
    if (tid == 0 && tk.out_idx >= 0) {
      const int64_t l = tk.out_idx;
      const int32_t cv = (int32_t)a.lconst[l];
      int32_t rv = 0;
      const uint32_t* root = scr + tk.root_off;
      if (tk.root_off >= 0) rv = (int32_t)root[0];
      const bool fin = cv > NEG_CUT && rv > NEG_CUT;
      a.out[l] = (uint32_t)(fin ? cv + rv : NEG);
#pragma unroll
      for (int p = 0; p < KR; ++p) {
        const uint32_t rr = tk.root_off >= 0 ? root[(p + 1) * a.scratch_entries] : 1u;
        const uint64_t x = (uint64_t)rr * a.lconst[(p + 1) * a.n_out + l];
        a.out[(p + 1) * a.n_out + l] = fin ? pmod(x, a.mod.p[p], a.mod.c[p]) : 0u;
      }
    }
    __syncthreads();
  }
}

__global__ void zero_kernel(unsigned long long* q) { *q = 0; }

}  // namespace

size_t persist_lds_bytes(int k, int64_t lds_entries) {
  return (size_t)2 * (1 + k) * lds_entries * 4 + (size_t)NTHR * 4 * (1 + k);
}

void launch_persist(int k, const PersistArgs& a, int n_blocks, hipStream_t st) {
  const size_t lds = persist_lds_bytes(k, a.lds_entries);
  hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(1), 0, st, a.queue);
  BBTN_HIP(hipGetLastError());
  switch (k) {
#define BBTN_PK(K)                                                                 \
  case K:                                                                          \
    BBTN_HIP(hipFuncSetAttribute((const void*)persist_kernel<K>,                    \
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)); \
    hipLaunchKernelGGL(persist_kernel<K>, dim3(n_blocks), dim3(NTHR), lds, st, a); \
    break;
    BBTN_PK(0)
    BBTN_PK(1)
    BBTN_PK(2)
    BBTN_PK(3)
    BBTN_PK(4)
#undef BBTN_PK
    default:
      throw Error(BBTN_E_INVALID_ARG, "k must be in [0, 4]");
  }
  BBTN_HIP(hipGetLastError());
}

}  // namespace bbtn
