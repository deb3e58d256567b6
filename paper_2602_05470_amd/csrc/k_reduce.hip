// Segmented tropical sums and branch bounds.
//
// reduce:  out[o] = (+)_{s<S} in[s*seg_stride + o*elem_stride]  -- sums out
//   variables, merges split-K partial products and merges branch results
//   ("the final result is obtained by summing the contractions of each
//   branch", "Branch-and-Bound Tensor Network" section).  Few long segments
//   use one workgroup per output with a wavefront (DPP/shuffle) + LDS tree;
//   many short segments use one thread per output.
//
// bound:  global pruning ("Branch-and-Bound Tensor Network" section): an
//   upper bound (max form) on everything a branch can reach is its fixed
//   offset plus, for every remaining tensor, the tensor's largest finite
//   entry, because every term of the contraction takes one entry from each
//   tensor.  A branch is kept iff the bound is not below the incumbent; ties
//   are kept because they carry counts.  Kept branch ids are compacted in
//   ascending order.
#include "launch.h"

namespace bbtn {

namespace {

__device__ __forceinline__ uint64_t fold64r(uint64_t x, uint32_t c) {
  return (uint64_t)(uint32_t)(x >> 32) * c + (uint32_t)x;
}
__device__ __forceinline__ uint32_t mod_final_r(uint64_t x, uint32_t p, uint32_t c) {
  x = fold64r(x, c);
  x = fold64r(x, c);
  x = fold64r(x, c);
  x = fold64r(x, c);
  x = x >= p ? x - p : x;
  x = x >= p ? x - p : x;
  return (uint32_t)x;
}

struct ReduceArgs {
  const uint32_t* in;
  uint32_t* out;
  int64_t pin, pout;
  int64_t outer, S, seg, elem;
  Moduli mod;
};

// One thread per output.  Residues are < 2^31, so a 64-bit sum takes 2^33
// terms before it could overflow.
template <int KR>
__global__ void __launch_bounds__(256) reduce_thread_kernel(const ReduceArgs a) {
  for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < a.outer;
       o += (int64_t)gridDim.x * blockDim.x) {
    int32_t v = INT32_MIN;
    uint64_t acc[KR > 0 ? KR : 1] = {};
    for (int64_t s = 0; s < a.S; ++s) {
      const int64_t x = s * a.seg + o * a.elem;
      const int32_t xv = (int32_t)a.in[x];
      if (xv <= NEG_CUT) continue;
      if (xv > v) {
        v = xv;
#pragma unroll
        for (int p = 0; p < KR; ++p) acc[p] = a.in[(p + 1) * a.pin + x];
      } else if (xv == v) {
#pragma unroll
        for (int p = 0; p < KR; ++p) acc[p] += a.in[(p + 1) * a.pin + x];
      }
    }
    const bool fin = v > NEG_CUT;
    a.out[o] = (uint32_t)(fin ? v : NEG);
#pragma unroll
    for (int p = 0; p < KR; ++p)
      a.out[(p + 1) * a.pout + o] = fin ? mod_final_r(acc[p], a.mod.p[p], a.mod.c[p]) : 0u;
  }
}

// Combine two partial (value, residues) pairs; residues already in [0, p).
template <int KR>
__device__ __forceinline__ void combine(int32_t& v, uint32_t* r, int32_t v2,
                                        const uint32_t* r2, const Moduli& m) {
  if (v2 > v) {
    v = v2;
#pragma unroll
    for (int p = 0; p < KR; ++p) r[p] = r2[p];
  } else if (v2 == v) {
#pragma unroll
    for (int p = 0; p < KR; ++p) {
      uint32_t s = r[p] + r2[p];
      r[p] = s >= m.p[p] ? s - m.p[p] : s;
    }
  }
}

// One workgroup (256 threads = 4 wavefronts) per output.
template <int KR>
__global__ void __launch_bounds__(256) reduce_block_kernel(const ReduceArgs a) {
  constexpr int KP = KR > 0 ? KR : 1;
  __shared__ int32_t sv[4];
  __shared__ uint32_t sr[4][KP];
  for (int64_t o = blockIdx.x; o < a.outer; o += gridDim.x) {
    int32_t v = INT32_MIN;
    uint64_t acc[KP] = {};
    for (int64_t s = threadIdx.x; s < a.S; s += blockDim.x) {
      const int64_t x = s * a.seg + o * a.elem;
      const int32_t xv = (int32_t)a.in[x];
      if (xv <= NEG_CUT) continue;
      if (xv > v) {
        v = xv;
#pragma unroll
        for (int p = 0; p < KR; ++p) acc[p] = a.in[(p + 1) * a.pin + x];
      } else if (xv == v) {
#pragma unroll
        for (int p = 0; p < KR; ++p) acc[p] += a.in[(p + 1) * a.pin + x];
      }
    }
    uint32_t r[KP];
#pragma unroll
    for (int p = 0; p < KP; ++p) r[p] = KR > 0 ? mod_final_r(acc[p], a.mod.p[p], a.mod.c[p]) : 0u;
    // wavefront reduction (64 lanes)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const int32_t v2 = __shfl_xor(v, off, 64);
      uint32_t r2[KP];
#pragma unroll
      for (int p = 0; p < KP; ++p) r2[p] = __shfl_xor(r[p], off, 64);
      combine<KR>(v, r, v2, r2, a.mod);
    }
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    if (lane == 0) {
      sv[wave] = v;
#pragma unroll
      for (int p = 0; p < KP; ++p) sr[wave][p] = r[p];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int w = 1; w < (int)(blockDim.x / 64); ++w) combine<KR>(v, r, sv[w], sr[w], a.mod);
      const bool fin = v > NEG_CUT;
      a.out[o] = (uint32_t)(fin ? v : NEG);
#pragma unroll
      for (int p = 0; p < KR; ++p) a.out[(p + 1) * a.pout + o] = fin ? r[p] : 0u;
    }
    __syncthreads();
  }
}

template <int KR>
void reduce_dispatch(const ReduceArgs& a, hipStream_t st) {
  if (a.S >= 512 && a.outer <= 4096) {
    const int64_t blocks = std::min<int64_t>(a.outer, 4096);
    launch_kernel(reduce_block_kernel<KR>, dim3((unsigned)blocks), dim3(256), 0, st, true, a);
  } else {
    const int64_t blocks = std::min<int64_t>((a.outer + 255) / 256, 256 * 256);
    launch_kernel(reduce_thread_kernel<KR>, dim3((unsigned)blocks), dim3(256), 0, st, true, a);
  }
}

// ---------------------------------------------------------------- bound
__global__ void __launch_bounds__(256)
bound_kernel(int64_t n_branch, int32_t T, const int32_t* values, const int64_t* off,
             const int32_t* len, const int64_t* offset, int64_t incumbent,
             int64_t* bound, int32_t* flags) {
  __shared__ long long ssum[4];
  __shared__ int sok[4];
  for (int64_t b = blockIdx.x; b < n_branch; b += gridDim.x) {
    long long sum = 0;
    int ok = 1;
    for (int t = threadIdx.x; t < T; t += blockDim.x) {
      const int64_t o = off[b * T + t];
      const int32_t n = len[b * T + t];
      int32_t mx = INT32_MIN;
      for (int32_t e = 0; e < n; ++e) {
        const int32_t v = values[o + e];
        if (v > NEG_CUT && v > mx) mx = v;
      }
      if (mx == INT32_MIN) ok = 0;
      else sum += mx;
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
      sum += __shfl_xor(sum, d, 64);
      ok &= __shfl_xor(ok, d, 64);
    }
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    if (lane == 0) { ssum[wave] = sum; sok[wave] = ok; }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int w = 1; w < (int)(blockDim.x / 64); ++w) { sum += ssum[w]; ok &= sok[w]; }
      const int64_t bd = offset[b] + sum;
      bound[b] = bd;
      flags[b] = (ok && bd >= incumbent) ? 1 : 0;
    }
    __syncthreads();
  }
}

// Single-workgroup exclusive scan of the flags, writing kept ids in order.
__global__ void __launch_bounds__(1024)
compact_kernel(int64_t n, const int32_t* flags, int32_t* keep_idx, int32_t* n_keep) {
  __shared__ int32_t wsum[16];
  __shared__ int32_t base;
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  for (int64_t start = 0; start < n; start += blockDim.x) {
    const int64_t i = start + threadIdx.x;
    const int32_t f = (i < n) ? flags[i] : 0;
    // inclusive scan within the wavefront
    int32_t x = f;
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int32_t y = __shfl_up(x, d, 64);
      if (lane >= d) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    int32_t before = 0;
    for (int w = 0; w < wave; ++w) before += wsum[w];
    const int32_t pos = base + before + x - f;
    if (f) keep_idx[pos] = (int32_t)i;
    __syncthreads();
    if (threadIdx.x == blockDim.x - 1) base = pos + f;
    __syncthreads();
  }
  if (threadIdx.x == 0) *n_keep = base;
}

}  // namespace

void launch_reduce(int k, const Moduli& mod, int64_t outer, int64_t S,
                   int64_t seg_stride, int64_t elem_stride, DevTensor in,
                   DevTensor out, hipStream_t st) {
  if (outer <= 0) return;
  BBTN_REQUIRE(S >= 1, "reduce: empty segment");
  ReduceArgs a{};
  a.in = in.ptr; a.out = out.ptr;
  a.pin = in.pstride; a.pout = out.pstride;
  a.outer = outer; a.S = S; a.seg = seg_stride; a.elem = elem_stride;
  a.mod = mod;
  switch (k) {
    case 0: reduce_dispatch<0>(a, st); break;
    case 1: reduce_dispatch<1>(a, st); break;
    case 2: reduce_dispatch<2>(a, st); break;
    case 3: reduce_dispatch<3>(a, st); break;
    case 4: reduce_dispatch<4>(a, st); break;
    case 5: reduce_dispatch<5>(a, st); break;
    default: throw Error(BBTN_E_INVALID_ARG, "k must be in [0, 5]");
  }
  BBTN_LAUNCHED("reduce");
}

void launch_bound(int64_t n_branch, int32_t T, const int32_t* values,
                  const int64_t* off, const int32_t* len, const int64_t* offset,
                  int64_t incumbent, int64_t* bound, int32_t* flags,
                  int32_t* keep_idx, int32_t* n_keep, hipStream_t st) {
  if (n_branch > 0) {
    const int64_t blocks = std::min<int64_t>(n_branch, 65536);
    hipLaunchKernelGGL(bound_kernel, dim3((unsigned)blocks), dim3(256), 0, st, n_branch, T,
                       values, off, len, offset, incumbent, bound, flags);
    BBTN_LAUNCHED("bound");
  }
  hipLaunchKernelGGL(compact_kernel, dim3(1), dim3(1024), 0, st, n_branch, flags, keep_idx,
                     n_keep);
  BBTN_LAUNCHED("compact");
}

}  // namespace bbtn

namespace bbtn {
namespace {
// out[l] = a[l] (.) b[l]  (tropical product of two entry vectors)
template <int KR>
__global__ void __launch_bounds__(256) otimes_kernel(int64_t L, const uint32_t* a, int64_t pa,
                                                     const uint32_t* b, int64_t pb, uint32_t* o,
                                                     int64_t po, Moduli mod) {
  for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < L;
       l += (int64_t)gridDim.x * blockDim.x) {
    const int32_t av = (int32_t)a[l], bv = (int32_t)b[l];
    const bool fin = av > NEG_CUT && bv > NEG_CUT;
    o[l] = (uint32_t)(fin ? av + bv : NEG);
#pragma unroll
    for (int p = 0; p < KR; ++p) {
      const uint64_t x = (uint64_t)a[(p + 1) * pa + l] * b[(p + 1) * pb + l];
      o[(p + 1) * po + l] = fin ? (uint32_t)(x % mod.p[p]) : 0u;
    }
  }
}
}  // namespace

void launch_otimes(int k, const Moduli& mod, int64_t L, DevTensor a, DevTensor b,
                   DevTensor out, hipStream_t st) {
  if (L <= 0) return;
  const unsigned blocks = (unsigned)std::min<int64_t>((L + 255) / 256, 4096);
  switch (k) {
    case 0: hipLaunchKernelGGL(otimes_kernel<0>, dim3(blocks), dim3(256), 0, st, L, a.ptr, a.pstride, b.ptr, b.pstride, out.ptr, out.pstride, mod); break;
    case 1: hipLaunchKernelGGL(otimes_kernel<1>, dim3(blocks), dim3(256), 0, st, L, a.ptr, a.pstride, b.ptr, b.pstride, out.ptr, out.pstride, mod); break;
    case 2: hipLaunchKernelGGL(otimes_kernel<2>, dim3(blocks), dim3(256), 0, st, L, a.ptr, a.pstride, b.ptr, b.pstride, out.ptr, out.pstride, mod); break;
    case 3: hipLaunchKernelGGL(otimes_kernel<3>, dim3(blocks), dim3(256), 0, st, L, a.ptr, a.pstride, b.ptr, b.pstride, out.ptr, out.pstride, mod); break;
    case 4: hipLaunchKernelGGL(otimes_kernel<4>, dim3(blocks), dim3(256), 0, st, L, a.ptr, a.pstride, b.ptr, b.pstride, out.ptr, out.pstride, mod); break;
    case 5: hipLaunchKernelGGL(otimes_kernel<5>, dim3(blocks), dim3(256), 0, st, L, a.ptr, a.pstride, b.ptr, b.pstride, out.ptr, out.pstride, mod); break;
    default: throw Error(BBTN_E_INVALID_ARG, "k must be in [0, 5]");
  }
  BBTN_LAUNCHED("otimes");
}

}  // namespace bbtn
