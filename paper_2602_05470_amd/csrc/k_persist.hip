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
#include <atomic>
#include <type_traits>

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

__device__ __forceinline__ int32_t max3i(int32_t a, int32_t b, int32_t c) {
  return max(max(a, b), c);
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

// Step programs are read-only during a launch: reading them through the
// constant address space lets uniform descriptor reads become scalar loads.
template <class T>
using kptr = const __attribute__((address_space(4))) T*;
template <class T>
__device__ __forceinline__ kptr<T> kconst(const T* p) {
  return (kptr<T>)p;
}

// Pointers typed by address space (global = 1, LDS = 3): staging and
// output code written once for both sources must not be merged into one
// body over a pointer that may be either (which would need flat accesses).
template <class T>
using gptr = __attribute__((address_space(1))) T*;
template <class T>
using lptr = __attribute__((address_space(3))) T*;

template <int N>
struct Log2 {
  static constexpr int value = N <= 1 ? 0 : 1 + Log2<N / 2>::value;
};
template <>
struct Log2<1> {
  static constexpr int value = 0;
};

// One workgroup per task: one wavefront when tasks are many, 256 or 1024
// threads when they are few (the steps of a task are then wide enough to use
// them).  The task index is made uniform and every descriptor is read at a
// uniform address, so descriptors stay in scalar registers.
template <int KR, int NTHR>
__global__ void __launch_bounds__(NTHR)
persist_kernel(const PersistArgs a) {
  constexpr int W = 1 + KR;
  constexpr int LT = Log2<NTHR>::value;
  extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
  const int cap = (int)a.lds_entries;  // entries per operand buffer
  const int ae = (int)a.arena_entries;  // entries per arena plane
  // plane strides as locals: the lambdas below capture by reference, and a
  // reference to the kernel argument would move it to private memory
  const int64_t scr_stride = a.scratch_entries, sh_stride = a.shared_entries;
  uint32_t* la = lds;                  // W planes of cap entries
  uint32_t* lb = lds + W * cap;
  uint32_t* arena = lb + W * cap;      // W planes of ae entries: small intermediates
  int32_t* pv = (int32_t*)(arena + W * ae);  // NTHR partial values
  uint32_t* pr = (uint32_t*)(pv + NTHR);   // KR x NTHR partial residues
  uint32_t* fixtab = pr + KR * NTHR;       // the task's fixed bits per slot
  uint32_t* const scr_block = a.scratch + (int64_t)blockIdx.x * W * a.scratch_entries;
  const int tid = threadIdx.x;

  __shared__ uint32_t s_task;
  for (;;) {
    uint32_t got = 0;
    if (tid == 0) got = (uint32_t)atomicAdd(a.queue, 1ull);
    if constexpr (NTHR == 64) {
      got = __shfl(got, 0);
    } else {
      if (tid == 0) s_task = got;
      __syncthreads();
      got = s_task;
      __syncthreads();
    }
    const int64_t task = (int64_t)__builtin_amdgcn_readfirstlane(got);
    if (task >= a.n_tasks) break;
    uint32_t* const scr =
        a.per_task_scratch ? a.scratch + task * W * a.scratch_entries : scr_block;
    // the run holding the task (uniform binary search over the runs)
    int64_t lo = 0, hi = a.n_runs - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (kconst(a.tasks + mid)->first <= task) lo = mid;
      else hi = mid - 1;
    }
    const kptr<PTask> tk = kconst(a.tasks + lo);
    const int64_t ti = task - tk->first;
    const uint8_t* asg = a.assign + tk->assign_off + ti * tk->assign_stride;
    const int32_t n_steps = tk->n_steps;
    kptr<PStep> sp = kconst(a.steps + tk->step_off);
    const uint32_t* const base = a.base + tk->base_off;
    uint32_t* const shared = a.shared + tk->shared_off;
    // the fixed bits of every base operand of the program, from the task's
    // states (once per task instead of once per step)
    const int32_t n_slots = tk->n_slots;
    if (n_slots > 0) {
      const kptr<PSlot> sl = kconst(a.slots + tk->slot_off);
      const kptr<PFix> fxs = kconst(a.fixes);
      for (int j = tid; j < n_slots; j += NTHR) {
        const int32_t fo = sl[j].fix_off, nf = sl[j].n_fix;
        uint32_t f = 0;
        for (int i = 0; i < nf; ++i)
          f |= (uint32_t)(asg[fxs[fo + i].idx] & 1) << fxs[fo + i].pos;
        fixtab[j] = f;
      }
      __syncthreads();
    }

    for (int32_t si = 0; si < n_steps; ++si, ++sp) {
      // ---- stage operands
#pragma unroll
      for (int w = 0; w < 2; ++w) {
        const kptr<POperand> op = w == 0 ? &sp->a : &sp->b;
        uint32_t* dst = w == 0 ? la : lb;
        const int slot = op->slot;
        const uint32_t fixed = slot >= 0 ? fixtab[slot] : 0u;
        const int kind = op->kind;
        const uint32_t* src = kind == PK_BASE     ? base + op->src_off
                              : kind == PK_SHARED ? shared + op->src_off
                                                  : scr + op->src_off;
        const int64_t sstride = kind == PK_BASE ? a.base_total
                                : kind == PK_SHARED
                                    ? (op->stride > 0 ? (int64_t)op->stride : a.shared_entries)
                                    : a.scratch_entries;
        uint32_t pw[P_MAX_RANK / 4];
#pragma unroll
        for (int i = 0; i < P_MAX_RANK / 4; ++i) pw[i] = op->bitpos[i];
        // source bit of layout bit j (j a constant after unrolling)
        auto pos = [&](int j) { return (pw[j >> 2] >> (8 * (j & 3))) & 255u; };
        const int n = 1 << op->rank;
        const int64_t mat = op->mat_off;
        const bool from_lds = kind == PK_LDS;
        // The layout-to-source index map only moves bits, so it is OR-linear
        // over disjoint bit sets: entry e = e0 | u * NTHR | tid maps to
        // map(e0) | map(u * NTHR) | map(tid).  The thread part is formed
        // once per operand, the batch parts are uniform.  SB entries per
        // thread are in flight (every load of a batch is issued before the
        // first is used), SB sized to the operand: n and NTHR are powers of
        // two and SB divides n / NTHR when n >= NTHR, so the batches cover
        // the operand exactly; a smaller operand has one batch, whose lanes
        // past the end load its last entry and store nothing.
        const uint32_t el = (uint32_t)min(tid, n - 1);
        uint32_t lo_bits = 0;
#pragma unroll
        for (int j = 0; j < LT; ++j) lo_bits |= ((el >> j) & 1u) << pos(j);
        // `sp_` and `ss_` are the source and its plane stride: the arena
        // (LDS) or a global buffer, each inlined with its own address space
        auto stage = [&](auto sb_tag, auto sp_, int64_t ss_) __attribute__((always_inline)) {
          constexpr int SB = decltype(sb_tag)::value;
          constexpr int LB = Log2<SB>::value;
          uint32_t hu[SB];
#pragma unroll
          for (int u = 0; u < SB; ++u) {
            uint32_t h = lo_bits;
#pragma unroll
            for (int b = 0; b < LB; ++b)
              if ((u >> b) & 1) h |= 1u << pos(LT + b);
            hu[u] = h;
          }
          for (int e0 = 0; e0 < n; e0 += NTHR * SB) {
            uint32_t he = fixed;
#pragma unroll
            for (int j = LT + LB; j < P_MAX_RANK; ++j) he |= (((uint32_t)e0 >> j) & 1u) << pos(j);
            uint32_t v[SB][W];
#pragma unroll
            for (int u = 0; u < SB; ++u) {
              const uint32_t s = he | hu[u];
#pragma unroll
              for (int p = 0; p < W; ++p) v[u][p] = (sp_ + p * ss_)[s];
            }
#pragma unroll
            for (int u = 0; u < SB; ++u) {
              const int e = e0 + u * NTHR + tid;
              if (SB > 1 || e < n) {  // SB > 1 only when n >= 2 * NTHR
#pragma unroll
                for (int p = 0; p < W; ++p) {
                  dst[p * cap + e] = v[u][p];
                  if (mat >= 0) ((gptr<uint32_t>)scr)[p * scr_stride + mat + e] = v[u][p];
                }
              }
            }
          }
        };
        const int per = (n + NTHR - 1) / NTHR;  // entries per thread (uniform)
        if (from_lds) {
          const lptr<const uint32_t> ls = (lptr<const uint32_t>)(arena + op->src_off);
          if (per >= 4) stage(std::integral_constant<int, 4>{}, ls, (int64_t)ae);
          else if (per >= 2) stage(std::integral_constant<int, 2>{}, ls, (int64_t)ae);
          else stage(std::integral_constant<int, 1>{}, ls, (int64_t)ae);
        } else {
          const gptr<const uint32_t> gs = (gptr<const uint32_t>)src;
          if (per >= 8 && KR < 3) stage(std::integral_constant<int, 8>{}, gs, sstride);
          else if (per >= 4) stage(std::integral_constant<int, 4>{}, gs, sstride);
          else if (per >= 2) stage(std::integral_constant<int, 2>{}, gs, sstride);
          else stage(std::integral_constant<int, 1>{}, gs, sstride);
        }
      }
      __syncthreads();
      // ---- product
      const int rn = sp->rn, rm = sp->rm, rk = sp->rk;
      const int nC = 1 << (sp->rb + rm + rn);
      const int K = 1 << rk;
      const int c_kind = sp->c_kind;
      const int64_t c_off = sp->c_off;
      const int64_t c_sh = sp->c_stride > 0 ? (int64_t)sp->c_stride : sh_stride;
      // write output entry o (tropical zero when not finite) to the arena,
      // the shared region or the workgroup's scratch (uniform choice)
      auto put = [&](int o, int32_t v, const uint32_t (&r)[KR > 0 ? KR : 1])
                     __attribute__((always_inline)) {
        const bool fin = v > NEG_CUT;
        if (c_kind == PK_LDS) {
          const lptr<uint32_t> cl = (lptr<uint32_t>)(arena + c_off);
          cl[o] = (uint32_t)(fin ? v : NEG);
#pragma unroll
          for (int p = 0; p < KR; ++p) cl[(p + 1) * ae + o] = fin ? r[p] : 0u;
        } else {
          const bool sh = c_kind == PK_SHARED;
          const gptr<uint32_t> c = (gptr<uint32_t>)((sh ? shared : scr) + c_off);
          const int64_t cs = sh ? c_sh : scr_stride;
          c[o] = (uint32_t)(fin ? v : NEG);
#pragma unroll
          for (int p = 0; p < KR; ++p) c[(p + 1) * cs + o] = fin ? r[p] : 0u;
        }
      };
      // values pass, wide steps over row pairs: two m by four consecutive n
      // per thread, so that four K steps cost two 16-byte reads of A and
      // four of B for 32 MACs
      const bool vec8 = KR == 0 && rn >= 2 && rm >= 1 && K >= 4 && (nC >> 3) >= NTHR;
      if constexpr (KR == 0) {
        if (vec8) {
          const int nI = nC >> 3;
          const int gb = rn - 2;  // bits of the four-wide n group
          for (int it = tid; it < nI; it += NTHR) {
            const int g = it & ((1 << gb) - 1);
            const int mb = it >> gb;
            const int m = (mb & ((1 << (rm - 1)) - 1)) << 1;
            const int b = mb >> (rm - 1);
            const int o = (g << 2) | (m << rn) | (b << (rn + rm));
            const int32_t* A0 = (const int32_t*)la + ((m << rk) | (b << (rk + rm)));
            const int32_t* A1 = A0 + K;  // row m + 1
            const int32_t* Bv = (const int32_t*)lb + ((g << 2) | (b << (rn + rk)));
            int32_t V[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) V[i] = INT32_MIN;
            for (int q = 0; q < K; q += 4) {
              const int4 a0 = *(const int4*)(A0 + q);
              const int4 a1 = *(const int4*)(A1 + q);
              const int4 b0 = *(const int4*)(Bv + (q << rn));
              const int4 b1 = *(const int4*)(Bv + ((q + 1) << rn));
              const int4 b2 = *(const int4*)(Bv + ((q + 2) << rn));
              const int4 b3 = *(const int4*)(Bv + ((q + 3) << rn));
              V[0] = max3i(max3i(V[0], a0.x + b0.x, a0.y + b1.x), a0.z + b2.x, a0.w + b3.x);
              V[1] = max3i(max3i(V[1], a0.x + b0.y, a0.y + b1.y), a0.z + b2.y, a0.w + b3.y);
              V[2] = max3i(max3i(V[2], a0.x + b0.z, a0.y + b1.z), a0.z + b2.z, a0.w + b3.z);
              V[3] = max3i(max3i(V[3], a0.x + b0.w, a0.y + b1.w), a0.z + b2.w, a0.w + b3.w);
              V[4] = max3i(max3i(V[4], a1.x + b0.x, a1.y + b1.x), a1.z + b2.x, a1.w + b3.x);
              V[5] = max3i(max3i(V[5], a1.x + b0.y, a1.y + b1.y), a1.z + b2.y, a1.w + b3.y);
              V[6] = max3i(max3i(V[6], a1.x + b0.z, a1.y + b1.z), a1.z + b2.z, a1.w + b3.z);
              V[7] = max3i(max3i(V[7], a1.x + b0.w, a1.y + b1.w), a1.z + b2.w, a1.w + b3.w);
            }
            const uint32_t none[1] = {0u};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              put(o + i, V[i], none);
              put(o + (1 << rn) + i, V[4 + i], none);
            }
          }
        }
      }
      // wide steps: four consecutive n per thread, so that each q costs one
      // read of A and one 16-byte read of B for four outputs
      const bool vec4 = !vec8 && rn >= 2 && (nC >> 2) >= NTHR;
      if (vec4) {
        const int nI = nC >> 2;
        for (int it = tid; it < nI; it += NTHR) {
          const int o = it << 2;
          const int nn = o & ((1 << rn) - 1);
          const int m = (o >> rn) & ((1 << rm) - 1);
          const int b = o >> (rn + rm);
          const int abase = (m << rk) | (b << (rk + rm));
          const int bbase = nn | (b << (rn + rk));
          const int32_t* Av = (const int32_t*)la + abase;
          const int32_t* Bv = (const int32_t*)lb + bbase;
          int32_t V[4] = {INT32_MIN, INT32_MIN, INT32_MIN, INT32_MIN};
          if (K >= 4) {
            // four K steps at a time: one 16-byte read of A (its row starts
            // at a multiple of K), four of B, two three-way maxima per output
            for (int q = 0; q < K; q += 4) {
              const int4 a4 = *(const int4*)(Av + q);
              const int4 b0 = *(const int4*)(Bv + (q << rn));
              const int4 b1 = *(const int4*)(Bv + ((q + 1) << rn));
              const int4 b2 = *(const int4*)(Bv + ((q + 2) << rn));
              const int4 b3 = *(const int4*)(Bv + ((q + 3) << rn));
              V[0] = max3i(max3i(V[0], a4.x + b0.x, a4.y + b1.x), a4.z + b2.x, a4.w + b3.x);
              V[1] = max3i(max3i(V[1], a4.x + b0.y, a4.y + b1.y), a4.z + b2.y, a4.w + b3.y);
              V[2] = max3i(max3i(V[2], a4.x + b0.z, a4.y + b1.z), a4.z + b2.z, a4.w + b3.z);
              V[3] = max3i(max3i(V[3], a4.x + b0.w, a4.y + b1.w), a4.z + b2.w, a4.w + b3.w);
            }
          } else {
            for (int q = 0; q < K; ++q) {
              const int32_t av = Av[q];
              const int4 bv = *(const int4*)(Bv + (q << rn));
              V[0] = max(V[0], av + bv.x);
              V[1] = max(V[1], av + bv.y);
              V[2] = max(V[2], av + bv.z);
              V[3] = max(V[3], av + bv.w);
            }
          }
          uint32_t res[4][KR > 0 ? KR : 1];
          if constexpr (KR > 0) {
            uint64_t acc[4][KR];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
              for (int p = 0; p < KR; ++p) acc[i][p] = 0;
            if (max(max(V[0], V[1]), max(V[2], V[3])) > NEG_CUT) {
              // tie test without a compare: x = (V - 1) - a - b is -1 exactly
              // on a tie and >= 0 otherwise; sums that wrap involve stored
              // zeros, whose residues are 0
              uint32_t vm1[4];
#pragma unroll
              for (int i = 0; i < 4; ++i) vm1[i] = (uint32_t)V[i] - 1u;
              for (int q = 0; q < K; ++q) {
                const uint32_t na = (uint32_t)(-Av[q]);
                const int4 bv = *(const int4*)(Bv + (q << rn));
                uint32_t msk[4];
                msk[0] = (uint32_t)((int32_t)(vm1[0] + na - (uint32_t)bv.x) >> 31);
                msk[1] = (uint32_t)((int32_t)(vm1[1] + na - (uint32_t)bv.y) >> 31);
                msk[2] = (uint32_t)((int32_t)(vm1[2] + na - (uint32_t)bv.z) >> 31);
                msk[3] = (uint32_t)((int32_t)(vm1[3] + na - (uint32_t)bv.w) >> 31);
#pragma unroll
                for (int p = 0; p < KR; ++p) {
                  const uint32_t ac = la[(p + 1) * cap + abase + q];
                  const uint4 bc = *(const uint4*)(lb + (p + 1) * cap + bbase + (q << rn));
                  acc[0][p] += (uint64_t)(ac & msk[0]) * bc.x;
                  acc[1][p] += (uint64_t)(ac & msk[1]) * bc.y;
                  acc[2][p] += (uint64_t)(ac & msk[2]) * bc.z;
                  acc[3][p] += (uint64_t)(ac & msk[3]) * bc.w;
                }
                // at most three products (< 2^62 each) between folds
                if (q % 3 == 2) {
#pragma unroll
                  for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int p = 0; p < KR; ++p) acc[i][p] = pfold(acc[i][p], a.mod.c[p]);
                }
              }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
              for (int p = 0; p < KR; ++p) res[i][p] = pmod(acc[i][p], a.mod.p[p], a.mod.c[p]);
          }
#pragma unroll
          for (int i = 0; i < 4; ++i) put(o + i, V[i], res[i]);
        }
      }
      // threads per output: split K when outputs are few
      int tpo = 1;
      while (tpo * 2 <= NTHR / nC && tpo * 2 <= K) tpo *= 2;
      const int kper = K / tpo;
      const int per_round = NTHR / tpo;
      for (int o0 = (vec4 || vec8) ? nC : 0; o0 < nC; o0 += per_round) {
        const int o = o0 + tid / tpo;
        const int j = tid % tpo;
        int32_t V = INT32_MIN;
        uint32_t res[KR > 0 ? KR : 1];
        if (o < nC) {
          const int nn = o & ((1 << rn) - 1);
          const int m = (o >> rn) & ((1 << rm) - 1);
          const int b = o >> (rn + rm);
          const int abase = (m << rk) | (b << (rk + rm));
          const int bbase = nn | (b << (rn + rk));
          const int q0 = j * kper, q1 = q0 + kper;
          const int32_t* Av = (const int32_t*)la;
          const int32_t* Bv = (const int32_t*)lb;
          for (int q = q0; q < q1; ++q) V = max(V, Av[abase + q] + Bv[bbase + (q << rn)]);
          if constexpr (KR > 0) {
            uint64_t acc[KR];
#pragma unroll
            for (int p = 0; p < KR; ++p) acc[p] = 0;
            if (V > NEG_CUT) {
              int cnt = 0;
              for (int q = q0; q < q1; ++q) {
                const int ia = abase + q, ib = bbase + (q << rn);
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
        if (j == 0 && o < nC) put(o, V, res);
      }
      __syncthreads();
    }
    // ---- branch result = root (.) folded constant
    const int64_t l = tk->out_idx >= 0 ? tk->out_idx + ti : -1;
    const int64_t root_off = tk->root_off;
    if (tid == 0 && l >= 0) {
      const int32_t cv = (int32_t)a.lconst[l];
      // the root scalar: value and residues (an empty program: 0 and 1)
      uint32_t rw[W];
      rw[0] = 0;
#pragma unroll
      for (int p = 0; p < KR; ++p) rw[p + 1] = 1u;
      if (root_off >= 0) {
        if (tk->root_kind == PK_LDS) {
#pragma unroll
          for (int p = 0; p < W; ++p) rw[p] = arena[p * ae + root_off];
        } else {
#pragma unroll
          for (int p = 0; p < W; ++p) rw[p] = scr[p * a.scratch_entries + root_off];
        }
      }
      const int32_t rv = (int32_t)rw[0];
      const bool fin = cv > NEG_CUT && rv > NEG_CUT;
      a.out[l] = (uint32_t)(fin ? cv + rv : NEG);
#pragma unroll
      for (int p = 0; p < KR; ++p) {
        const uint32_t rr = rw[p + 1];
        const uint64_t x = (uint64_t)rr * a.lconst[(p + 1) * a.n_out + l];
        a.out[(p + 1) * a.n_out + l] = fin ? pmod(x, a.mod.p[p], a.mod.c[p]) : 0u;
      }
    }
    __syncthreads();
  }
}

__global__ void zero_kernel(unsigned long long* q) { *q = 0; }

}  // namespace

size_t persist_lds_bytes(int k, int64_t lds_entries, int64_t arena_entries, int threads,
                         int slots) {
  return (size_t)(2 * lds_entries + arena_entries) * (1 + k) * 4 +
         (size_t)threads * 4 * (1 + k) + (size_t)slots * 4;
}

// Raise a kernel's dynamic-LDS limit only when a launch needs more than it
// was last set to (the attribute call is not free on every launch).  The
// default limit is 64 KiB: launches within it make no attribute call, so they
// may be recorded into a graph.
static void raise_lds_limit(const void* fn, int bytes, std::atomic<int>& set) {
  int cur = set.load();
  while (bytes > cur) {
    BBTN_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
    if (set.compare_exchange_weak(cur, bytes)) break;
  }
}

template <int NT>
static void launch_nt(int k, const PersistArgs& a, int n_blocks, size_t lds, hipStream_t st) {
  switch (k) {
#define BBTN_PK(K)                                                                 \
  case K: {                                                                        \
    static std::atomic<int> attr{64 << 10};                                        \
    raise_lds_limit((const void*)persist_kernel<K, NT>, (int)lds, attr);           \
    hipLaunchKernelGGL((persist_kernel<K, NT>), dim3(n_blocks), dim3(NT), lds, st, a); \
    break;                                                                         \
  }
    BBTN_PK(0)
    BBTN_PK(1)
    BBTN_PK(2)
    BBTN_PK(3)
    BBTN_PK(4)
    BBTN_PK(5)
#undef BBTN_PK
    default:
      throw Error(BBTN_E_INVALID_ARG, "k must be in [0, 5]");
  }
}

void launch_persist(int k, const PersistArgs& a, int n_blocks, int threads, hipStream_t st) {
  const size_t lds = persist_lds_bytes(k, a.lds_entries, a.arena_entries, threads, a.max_slots);
  hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(1), 0, st, a.queue);
  BBTN_LAUNCHED("persist queue reset");
  switch (threads) {
    case 64: launch_nt<64>(k, a, n_blocks, lds, st); break;
    case 256: launch_nt<256>(k, a, n_blocks, lds, st); break;
    case 1024: launch_nt<1024>(k, a, n_blocks, lds, st); break;
    default: throw Error(BBTN_E_INTERNAL, "persistent executor: bad workgroup size");
  }
  BBTN_LAUNCHED("persist");
}

}  // namespace bbtn
