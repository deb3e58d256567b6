// Recovery of one optimal configuration (a semiring extension named in the
// Discussion section: configurations).  After a values-only recontraction
// of the winning branch that keeps every operand, the steps are walked from
// the root down.  At each step the states of the output variables are
// already known (set by the step that consumed the output), so the step's
// summed variables take the state q that reaches the maximum of
// A[b, m, q] + B[b, q, n] (lowest q on ties).  One workgroup; a parallel
// argmax over q per step.  Latency-bound.  Up to 48K variables.
#include "kernels.h"
#include "trace.h"

namespace bbtn {

// One wavefront walks the steps; the variable states live in LDS so that a
// state written by lane 0 is read by the other lanes of the same wave (LDS
// operations of a wave complete in order) without a workgroup barrier.  When
// they fit, the step descriptors and variable lists are first copied into
// LDS too (one coalesced prologue), so that a step costs one round trip to
// memory (the operand values) instead of one per variable.
constexpr int TRACE_LDS_VARS = 48 * 1024;
constexpr size_t TRACE_STAGE_BYTES = 104 * 1024;

template <bool STAGED>
__global__ void __launch_bounds__(64)
trace_kernel(const TraceJob* jobs) {
  const TraceJob* jb = jobs + blockIdx.x;
  const TraceStep* steps = jb->steps;
  const int32_t n_steps = jb->n_steps;
  const int32_t* vars = jb->vars;
  const int32_t n_var_words = jb->n_var_words;
  const int32_t* ws = jb->ws;
  int8_t* assign = jb->assign;
  const int32_t n_vars = jb->n_vars;
  int32_t* status = jb->status;
  __shared__ int8_t sa[TRACE_LDS_VARS];
  extern __shared__ int64_t stage64[];  // STAGED: [steps][vars]
  const int lane = threadIdx.x;
  for (int v = lane; v < n_vars; v += 64) sa[v] = assign[v];
  const TraceStep* S = steps;
  const int32_t* VV = vars;
  if constexpr (STAGED) {
    TraceStep* ls = (TraceStep*)stage64;
    int32_t* lv = (int32_t*)(ls + n_steps);
    const int32_t* gs = (const int32_t*)steps;
    int32_t* ds = (int32_t*)ls;
    const int sw = n_steps * (int)(sizeof(TraceStep) / 4);
    for (int i = lane; i < sw; i += 64) ds[i] = gs[i];
    for (int i = lane; i < n_var_words; i += 64) lv[i] = vars[i];
    S = ls;
    VV = lv;
  }
  __syncthreads();
  int bad = 0;
  for (int32_t s = n_steps - 1; s >= 0; --s) {
    const TraceStep st = S[s];
    const int32_t* av = VV + st.var_off;                   // [K][M][batch]
    const int32_t* bv = av + (st.rk + st.rm + st.rb);      // [N][K][batch]
    // every lane forms the operand bases from the known states
    int64_t ab = 0, bb = 0;
    for (int j = st.rk; j < st.rk + st.rm + st.rb; ++j) {
      const int8_t x = sa[av[j]];
      bad |= x < 0;
      ab |= (int64_t)(x & 1) << j;
    }
    for (int j = 0; j < st.rn + st.rk + st.rb; ++j) {
      if (j >= st.rn && j < st.rn + st.rk) continue;
      const int8_t x = sa[bv[j]];
      bad |= x < 0;
      bb |= (int64_t)(x & 1) << j;
    }
    int32_t best = INT32_MIN;
    int64_t bq = INT64_MAX;
    const int64_t nq = 1ll << st.rk;
    for (int64_t q = lane; q < nq; q += 64) {
      const int32_t v = ws[st.a_off + ab + q] + ws[st.b_off + bb + (q << st.rn)];
      if (v > NEG_CUT && (v > best || (v == best && q < bq))) { best = v; bq = q; }
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
      const int32_t ov = __shfl_xor(best, d, 64);
      const int64_t oq = __shfl_xor(bq, d, 64);
      if (ov > best || (ov == best && oq < bq)) { best = ov; bq = oq; }
    }
    if (best == INT32_MIN) {
      bad |= 2;
      bq = 0;
    }
    for (int j = lane; j < st.rk; j += 64) sa[av[j]] = (int8_t)((bq >> j) & 1);
    __syncthreads();  // a single wave: keeps the LDS writes ordered before the next reads
  }
  for (int v = lane; v < n_vars; v += 64) assign[v] = sa[v];
  // fold every lane's flags into one status word
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) bad |= __shfl_xor(bad, d, 64);
  if (lane == 0 && bad) *status = bad;
}

void launch_trace(const TraceJob* jobs, int32_t n_jobs, int32_t max_steps, int32_t max_var_words,
                  int32_t max_vars, hipStream_t st) {
  if (n_jobs <= 0 || max_steps <= 0) return;
  BBTN_REQUIRE(max_vars <= TRACE_LDS_VARS, "configuration traceback: too many variables");
  const size_t stage = (size_t)max_steps * sizeof(TraceStep) + (size_t)max_var_words * 4;
  if (stage <= TRACE_STAGE_BYTES) {
    BBTN_HIP(hipFuncSetAttribute((const void*)trace_kernel<true>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)stage));
    hipLaunchKernelGGL(trace_kernel<true>, dim3(n_jobs), dim3(64), stage, st, jobs);
  } else {
    hipLaunchKernelGGL(trace_kernel<false>, dim3(n_jobs), dim3(64), 0, st, jobs);
  }
  BBTN_LAUNCHED("trace");
}

}  // namespace bbtn
