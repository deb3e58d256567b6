// Tensor permutation and branch-variable fixing (slicing, T|_{s_Vf = x} of
// Eq. 3), batched over branches.  Output entry (l, i) reads input entry
//   l * in_stride + (fixed_bits[l] & fixed_mask) + sum_runs ((i >> out_lo) &
//   (2^len - 1)) << in_lo
// where a "run" is a maximal range of consecutive output bits that maps onto
// consecutive input bits, so a plain copy is a single run and a typical
// permutation needs a handful.  One thread per output entry, grid-stride;
// writes are coalesced, reads follow the permutation.  HBM-bound.
#include "kernels.h"

namespace bbtn {

struct GatherArgs {
  const uint32_t* in;
  uint32_t* out;
  int64_t pin, pout;
  int64_t L, in_stride;
  const uint64_t* fixed;
  uint64_t fixed_mask;
  int32_t r_out, n_runs;
  GatherRun runs[MAX_RUNS];
};

template <int PLANES>
__global__ void __launch_bounds__(256) gather_kernel(const GatherArgs g) {
  const int64_t total = g.L << g.r_out;
  const int64_t omask = (1ll << g.r_out) - 1;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l = e >> g.r_out;
    const uint64_t i = (uint64_t)(e & omask);
    uint64_t src = 0;
    for (int r = 0; r < g.n_runs; ++r) {
      const GatherRun run = g.runs[r];
      src |= ((i >> run.out_lo) & ((1ull << run.len) - 1)) << run.in_lo;
    }
    if (g.fixed) src |= g.fixed[l] & g.fixed_mask;
    const int64_t s = (int64_t)src + l * g.in_stride;
#pragma unroll
    for (int p = 0; p < PLANES; ++p) g.out[p * g.pout + e] = g.in[p * g.pin + s];
  }
}

void launch_gather(int k, const GatherPlan& gp, int64_t L, int64_t in_stride,
                   const uint64_t* fixed_bits, DevTensor in, DevTensor out,
                   hipStream_t st) {
  GatherArgs g{};
  g.in = in.ptr;
  g.out = out.ptr;
  g.pin = in.pstride;
  g.pout = out.pstride;
  g.L = L;
  g.in_stride = in_stride;
  g.fixed = fixed_bits;
  g.fixed_mask = gp.fixed_mask;
  g.r_out = gp.r_out;
  g.n_runs = gp.n_runs;
  for (int r = 0; r < gp.n_runs; ++r) g.runs[r] = gp.runs[r];
  const int64_t total = L << gp.r_out;
  if (total == 0) return;
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, 256 * 64);
  dim3 grid((unsigned)blocks), block(256);
  switch (k) {
    case 0: hipLaunchKernelGGL(gather_kernel<1>, grid, block, 0, st, g); break;
    case 1: hipLaunchKernelGGL(gather_kernel<2>, grid, block, 0, st, g); break;
    case 2: hipLaunchKernelGGL(gather_kernel<3>, grid, block, 0, st, g); break;
    case 3: hipLaunchKernelGGL(gather_kernel<4>, grid, block, 0, st, g); break;
    case 4: hipLaunchKernelGGL(gather_kernel<5>, grid, block, 0, st, g); break;
    default: throw Error(BBTN_E_INVALID_ARG, "k must be in [0, 4]");
  }
  BBTN_LAUNCHED("gather");
}

}  // namespace bbtn
