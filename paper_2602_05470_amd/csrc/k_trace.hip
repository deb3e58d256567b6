// Recovery of one optimal configuration (a semiring extension named in the
// Discussion section: configurations).  After a values-only recontraction
// of the winning branch that keeps every operand, the steps are walked from
// the root down.  At each step the states of the output variables are
// already known (set by the step that consumed the output), so the step's
// summed variables take the state q that reaches the maximum of
// A[b, m, q] + B[b, q, n] (lowest q on ties).  One workgroup; a parallel
// argmax over q per step.  Latency-bound.
#include "kernels.h"
#include "trace.h"

namespace bbtn {

__global__ void __launch_bounds__(256)
trace_kernel(const TraceStep* steps, int32_t n_steps, const int32_t* vars,
             const int32_t* ws, int8_t* assign, int32_t* status) {
  __shared__ int64_t sbase[2];
  __shared__ int32_t sv[4];
  __shared__ int64_t sq[4];
  for (int32_t s = n_steps - 1; s >= 0; --s) {
    const TraceStep st = steps[s];
    const int32_t* av = vars + st.var_off;                 // [K][M][batch]
    const int32_t* bv = av + (st.rk + st.rm + st.rb);      // [N][K][batch]
    if (threadIdx.x == 0) {
      int64_t ab = 0, bb = 0;
      int bad = 0;
      for (int j = st.rk; j < st.rk + st.rm + st.rb; ++j) {
        const int8_t x = assign[av[j]];
        bad |= x < 0;
        ab |= (int64_t)(x & 1) << j;
      }
      for (int j = 0; j < st.rn + st.rk + st.rb; ++j) {
        if (j >= st.rn && j < st.rn + st.rk) continue;
        const int8_t x = assign[bv[j]];
        bad |= x < 0;
        bb |= (int64_t)(x & 1) << j;
      }
      if (bad) atomicOr(status, 1);
      sbase[0] = ab;
      sbase[1] = bb;
    }
    __syncthreads();
    const int64_t ab = sbase[0], bb = sbase[1];
    int32_t best = INT32_MIN;
    int64_t bq = INT64_MAX;
    const int64_t nq = 1ll << st.rk;
    for (int64_t q = threadIdx.x; q < nq; q += blockDim.x) {
      const int32_t x = ws[st.a_off + ab + q];
      const int32_t y = ws[st.b_off + bb + (q << st.rn)];
      const int32_t v = x + y;
      if (v > NEG_CUT && (v > best || (v == best && q < bq))) { best = v; bq = q; }
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
      const int32_t ov = __shfl_xor(best, d, 64);
      const int64_t oq = __shfl_xor(bq, d, 64);
      if (ov > best || (ov == best && oq < bq)) { best = ov; bq = oq; }
    }
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    if (lane == 0) { sv[wave] = best; sq[wave] = bq; }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int w = 1; w < (int)(blockDim.x / 64); ++w)
        if (sv[w] > best || (sv[w] == best && sq[w] < bq)) { best = sv[w]; bq = sq[w]; }
      if (best == INT32_MIN) {
        atomicOr(status, 2);
        bq = 0;
      }
      for (int j = 0; j < st.rk; ++j) assign[av[j]] = (int8_t)((bq >> j) & 1);
    }
    __syncthreads();
  }
}

void launch_trace(const TraceStep* steps, int32_t n_steps, const int32_t* vars, const int32_t* ws,
                  int8_t* assign, int32_t* status, hipStream_t st) {
  if (n_steps <= 0) return;
  hipLaunchKernelGGL(trace_kernel, dim3(1), dim3(256), 0, st, steps, n_steps, vars, ws, assign,
                     status);
  BBTN_HIP(hipGetLastError());
}

}  // namespace bbtn
