// Tensor permutation and branch-variable fixing (slicing, T|_{s_Vf = x} of
// Eq. 3), batched over branches.  Output entry (l, i) reads input entry
//   l * in_stride + (fixed_bits[l] & fixed_mask) + sum_runs ((i >> out_lo) &
//   (2^len - 1)) << in_lo
// where a "run" is a maximal range of consecutive output bits that maps onto
// consecutive input bits, so a plain copy is a single run and a typical
// permutation needs a handful.  HBM-bound.
//
// Two kernels:
//  * direct: one thread per output entry, grid-stride; writes coalesced,
//    reads follow the permutation.  Used for small outputs and for
//    permutations whose lowest output bits already map onto the lowest free
//    input bits (reads then come in runs of at least 64 entries).
//  * tiled: a workgroup moves one tile through LDS.  The tile's variables T
//    are the (up to) 6 lowest output bits together with the output bits that
//    read the (up to) 6 lowest free input bits, at most 12 bits, 4096
//    entries.  The tile is read in input order (consecutive lanes read
//    consecutive addresses: runs of up to 64 entries) into LDS, then written
//    in output order (runs of up to 64 entries), plane by plane.  Index maps
//    of the tile are split into a low and a high 6-bit half whose offsets add
//    (a bit permutation is additive over disjoint bits), kept as 64-entry
//    tables in LDS.
#include "launch.h"

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
  // U entries a grid stride apart per thread and step, so that a thread has
  // about four loads in flight whatever the number of planes
  constexpr int U = PLANES >= 4 ? 1 : 4 / PLANES;
  const int64_t total = g.L << g.r_out;
  const int64_t omask = (1ll << g.r_out) - 1;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e0 < total;
       e0 += stride * U) {
    uint32_t v[U][PLANES];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = e0 + u * stride;
      if (u > 0 && e >= total) break;
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
      for (int p = 0; p < PLANES; ++p) v[u][p] = g.in[p * g.pin + s];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = e0 + u * stride;
      if (u > 0 && e >= total) break;
#pragma unroll
      for (int p = 0; p < PLANES; ++p) g.out[p * g.pout + e] = v[u][p];
    }
  }
}

// Tile of the LDS kernel: its variables in input order and in output order.
constexpr int TILE_MAX_BITS = 12;
struct GatherTile {
  int32_t tb;                       // tile bits
  int32_t n_rest;                   // output bits outside the tile
  int8_t in_pos[TILE_MAX_BITS];     // input bit of tile variable i (input order)
  int8_t out_pos[TILE_MAX_BITS];    // output bit of tile variable i (output order)
  int8_t rank[TILE_MAX_BITS];       // input-order index of output-order variable i
  int8_t rest[40];                  // output bits outside the tile, ascending
};

// Padded LDS slot of tile entry x (input order): one spare word per 64
// keeps strided output-order reads on distinct banks.
__device__ __forceinline__ int tile_slot(int x) { return x + (x >> 6); }

template <int PLANES>
__global__ void __launch_bounds__(256) gather_tiled_kernel(const GatherArgs g, const GatherTile t) {
  __shared__ uint32_t buf[(1 << TILE_MAX_BITS) + (1 << TILE_MAX_BITS) / 64];
  __shared__ int64_t in_lo[64], in_hi[64], out_lo[64], out_hi[64];
  __shared__ int16_t p_lo[64], p_hi[64];
  const int tid = threadIdx.x;
  if (tid < 64) {
    int64_t a = 0, b = 0, c = 0, d = 0;
    int pl = 0, ph = 0;
    for (int i = 0; i < 6; ++i) {
      if (!(tid >> i & 1)) continue;
      if (i < t.tb) {
        a |= 1ll << t.in_pos[i];
        c |= 1ll << t.out_pos[i];
        pl |= 1 << t.rank[i];
      }
      if (i + 6 < t.tb) {
        b |= 1ll << t.in_pos[i + 6];
        d |= 1ll << t.out_pos[i + 6];
        ph |= 1 << t.rank[i + 6];
      }
    }
    in_lo[tid] = a; in_hi[tid] = b; out_lo[tid] = c; out_hi[tid] = d;
    p_lo[tid] = (int16_t)pl; p_hi[tid] = (int16_t)ph;
  }
  __syncthreads();
  const int tsize = 1 << t.tb;
  const int64_t tiles = g.L << t.n_rest;
  const int64_t rmask = (1ll << t.n_rest) - 1;
  for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int64_t l = tile >> t.n_rest;
    const int64_t h = tile & rmask;
    // output offset of the tile's first entry: h's bits at the rest positions
    uint64_t obase = 0;
    for (int j = 0; j < t.n_rest; ++j) obase |= (uint64_t)(h >> j & 1) << t.rest[j];
    uint64_t src = 0;
    for (int r = 0; r < g.n_runs; ++r) {
      const GatherRun run = g.runs[r];
      src |= ((obase >> run.out_lo) & ((1ull << run.len) - 1)) << run.in_lo;
    }
    if (g.fixed) src |= g.fixed[l] & g.fixed_mask;
    const int64_t ibase = (int64_t)src + l * g.in_stride;
    const int64_t ob = (l << g.r_out) + (int64_t)obase;
#pragma unroll 1
    for (int p = 0; p < PLANES; ++p) {
      const uint32_t* in = g.in + p * g.pin + ibase;
      // all of a thread's loads in flight before the first LDS store
      uint32_t v[(1 << TILE_MAX_BITS) / 256];
#pragma unroll
      for (int j = 0; j < (1 << TILE_MAX_BITS) / 256; ++j) {
        const int x = tid + 256 * j;
        if (x < tsize) v[j] = in[in_lo[x & 63] + in_hi[x >> 6]];
      }
#pragma unroll
      for (int j = 0; j < (1 << TILE_MAX_BITS) / 256; ++j) {
        const int x = tid + 256 * j;
        if (x < tsize) buf[tile_slot(x)] = v[j];
      }
      __syncthreads();
      uint32_t* out = g.out + p * g.pout + ob;
      for (int u = tid; u < tsize; u += 256)
        out[out_lo[u & 63] + out_hi[u >> 6]] = buf[tile_slot(p_lo[u & 63] | p_hi[u >> 6])];
      __syncthreads();
    }
  }
}

// Tile for the LDS kernel, or tb = 0 when the direct kernel reads well
// enough: small outputs, or lowest output bits that already read a run of
// at least 64 (or all) of the lowest free input entries, a whole 256-byte
// segment per wavefront and plane.
static GatherTile choose_tile(const GatherPlan& gp, int k) {
  GatherTile t{};
  const int r_out = gp.r_out;
  if (r_out < 8) return t;
  // input bit -> output bit of every gathered (free) input variable
  int out_of[64];
  for (int i = 0; i < 64; ++i) out_of[i] = -1;
  for (int r = 0; r < gp.n_runs; ++r)
    for (int j = 0; j < gp.runs[r].len; ++j) out_of[gp.runs[r].in_lo + j] = gp.runs[r].out_lo + j;
  int low_free = -1;
  for (int i = 0; i < gp.r_in; ++i)
    if (out_of[i] >= 0) { low_free = i; break; }
  const GatherRun& r0 = gp.runs[0];
  if (gp.n_runs > 0 && r0.out_lo == 0 && r0.in_lo == low_free && r0.len >= std::min(6, r_out))
    return t;
  bool in_t[64] = {};
  for (int j = 0; j < std::min(6, r_out); ++j) in_t[j] = true;
  int taken = 0;
  for (int i = 0; i < gp.r_in && taken < 6; ++i)
    if (out_of[i] >= 0) { in_t[out_of[i]] = true; ++taken; }
  int tb = 0;
  for (int j = 0; j < r_out; ++j) tb += in_t[j];
  BBTN_REQUIRE(tb <= TILE_MAX_BITS, "gather tile too large");
  // where the two sets overlap, the next lowest output bits fill the tile
  // up to its 12 bits: longer output runs and fewer, larger tiles (a tile
  // of 11 bits with three or more planes moves faster as it is)
  if (tb <= 10 || k <= 1)
    for (int j = 0; j < r_out && tb < TILE_MAX_BITS; ++j)
      if (!in_t[j]) { in_t[j] = true; ++tb; }
  t.tb = tb;
  // input order of the tile's variables
  int n = 0;
  int in_rank_of_out[64];
  for (int i = 0; i < gp.r_in; ++i)
    if (out_of[i] >= 0 && in_t[out_of[i]]) {
      in_rank_of_out[out_of[i]] = n;
      t.in_pos[n++] = (int8_t)i;
    }
  n = 0;
  int nr = 0;
  for (int j = 0; j < r_out; ++j) {
    if (in_t[j]) {
      t.out_pos[n] = (int8_t)j;
      t.rank[n++] = (int8_t)in_rank_of_out[j];
    } else {
      t.rest[nr++] = (int8_t)j;
    }
  }
  t.n_rest = nr;
  return t;
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
  const GatherTile t = choose_tile(gp, k);
  if (t.tb > 0) {
    const int64_t tiles = L << t.n_rest;
    const int64_t blocks = std::min<int64_t>(tiles, 256 * 256);
    dim3 grid((unsigned)blocks), block(256);
    switch (k) {
      case 0: launch_kernel(gather_tiled_kernel<1>, grid, block, 0, st, true, g, t); break;
      case 1: launch_kernel(gather_tiled_kernel<2>, grid, block, 0, st, true, g, t); break;
      case 2: launch_kernel(gather_tiled_kernel<3>, grid, block, 0, st, true, g, t); break;
      case 3: launch_kernel(gather_tiled_kernel<4>, grid, block, 0, st, true, g, t); break;
      case 4: launch_kernel(gather_tiled_kernel<5>, grid, block, 0, st, true, g, t); break;
      case 5: launch_kernel(gather_tiled_kernel<6>, grid, block, 0, st, true, g, t); break;
      default: throw Error(BBTN_E_INVALID_ARG, "k must be in [0, 5]");
    }
    BBTN_LAUNCHED("gather (tiled)");
    return;
  }
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, 256 * 256);
  dim3 grid((unsigned)blocks), block(256);
  switch (k) {
    case 0: launch_kernel(gather_kernel<1>, grid, block, 0, st, true, g); break;
    case 1: launch_kernel(gather_kernel<2>, grid, block, 0, st, true, g); break;
    case 2: launch_kernel(gather_kernel<3>, grid, block, 0, st, true, g); break;
    case 3: launch_kernel(gather_kernel<4>, grid, block, 0, st, true, g); break;
    case 4: launch_kernel(gather_kernel<5>, grid, block, 0, st, true, g); break;
    case 5: launch_kernel(gather_kernel<6>, grid, block, 0, st, true, g); break;
    default: throw Error(BBTN_E_INVALID_ARG, "k must be in [0, 5]");
  }
  BBTN_LAUNCHED("gather");
}

}  // namespace bbtn
