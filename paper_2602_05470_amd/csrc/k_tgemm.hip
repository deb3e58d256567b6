// Counting tropical matrix product on the VALU (max form):
//   C[b,m,n] = (+)_q A[b,m,q] (.) B[b,q,n]
// where (.) adds values and multiplies counts and (+) keeps the larger value
// and adds the counts of ties (Eq. 2 with the counting tuple algebra of the
// "Tropical Tensor Networks" section).  This is not a ring product, so the
// matrix cores do not apply; the work is integer VALU arithmetic.
//
// Two passes over K per output tile:
//   1. values only: V[m,n] = max_q (a.v + b.v)   (one add + one max per MAC)
//   2. counts: for every q with a.v + b.v == V, add a.c_i * b.c_i into a
//      64-bit accumulator per residue with v_mad_u64_u32 (full rate on
//      gfx950); the accumulator is folded with one more multiply-add every
//      three terms (x = hi * 2^32 + lo == hi * (2^32 mod p) + lo) and reduced
//      to [0, p) once at the end.
// Operands are staged through LDS in TK-deep slices, transposed so that each
// thread reads its RM (RN) consecutive rows (columns) of a slice.  Workgroups
// are remapped so that each XCD works on a contiguous range of tiles (tiles
// sharing rows of A land in the same L2).
#include <mutex>

#include "launch.h"

namespace bbtn {

const TileCfg kTileCfgs[N_TILE_CFGS] = {
    {64, 64, 4, 4, 24},   // 0: large tiles, 256 threads (TK a multiple of 3: one fold per 3 steps)
    {32, 32, 2, 2, 24},   // 1: medium, 256 threads
    {16, 16, 1, 1, 16},   // 2: small, 256 threads
    {8, 64, 1, 2, 16},    // 3: few rows, 256 threads
    {64, 8, 2, 1, 16},    // 4: few columns, 256 threads
    {1, 256, 1, 1, 12},   // 5: one row (vector-matrix), 256 threads
    {256, 1, 1, 1, 12},   // 6: one column (matrix-vector), 256 threads
    {64, 32, 4, 2, 24},   // 7: tall, 256 threads (fewer accumulators than 0)
    {32, 64, 2, 4, 24},   // 8: wide, 256 threads
    {64, 64, 4, 4, 24},   // 9: as 0, operands staged four words at a time
    {64, 32, 4, 2, 24},   // 10: as 7, four-word staging
    {32, 64, 2, 4, 24},   // 11: as 8, four-word staging
    {32, 64, 2, 4, 12},   // 12: as 11, 12-deep slices (half the LDS): with
                          // four or more residues, three waves per SIMD
};

struct GemmArgs {
  const uint32_t* A;
  const uint32_t* B;
  uint32_t* C;
  int64_t pA, pB, pC;        // plane strides (words)
  int64_t M, N, K, batch;
  int64_t sAb, sBb, sCb;     // batch strides (elements)
  int64_t sCsplit;           // stride between split-K partial outputs
  int64_t kchunk;            // K range per split
  int64_t splits;
  int64_t tiles_m, tiles_n;
  int64_t total;             // tiles * splits * batch (work items of the grid)
  int32_t vec_a, vec_b;      // operands staged four words at a time (aligned rows)
  Moduli mod;
};

__device__ __forceinline__ uint64_t fold64(uint64_t x, uint32_t c) {
  return (uint64_t)(uint32_t)(x >> 32) * c + (uint32_t)x;
}

// x < 2^64  ->  x mod p, for 2^31 - 2^20 < p < 2^31 and c = 2^32 mod p < 2^21.
// Four folds bring x below 2^32 + 2^23 < 3p; two conditional subtractions
// finish.
__device__ __forceinline__ uint32_t mod_final(uint64_t x, uint32_t p, uint32_t c) {
  x = fold64(x, c);
  x = fold64(x, c);
  x = fold64(x, c);
  x = fold64(x, c);
  x = x >= p ? x - p : x;
  x = x >= p ? x - p : x;
  return (uint32_t)x;
}

// Workgroup w runs on XCD w % 8; give each XCD a contiguous block of tiles.
__device__ __forceinline__ int64_t xcd_remap(int64_t w, int64_t G) {
  const int64_t per = G / 8, rem = G % 8;
  const int64_t xcd = w % 8, local = w / 8;
  return xcd < rem ? xcd * (per + 1) + local
                   : rem * (per + 1) + (xcd - rem) * per + local;
}

// Output tile of work item t (after the XCD remap), plus the batch/split
// index `rest`: tiles in groups of GM tile rows, tile rows fastest within a
// group, so that the workgroups running at once on an XCD share column
// blocks of B while the group's rows of A stay in that XCD's L2.
constexpr int64_t GM = 8;
__device__ __forceinline__ void tile_coords(int64_t t, int64_t tiles_m, int64_t tiles_n,
                                            int64_t& tm, int64_t& tn, int64_t& rest) {
  const int64_t per = tiles_m * tiles_n;
  rest = t / per;
  t -= rest * per;
  const int64_t in_group = GM * tiles_n;
  const int64_t g = t / in_group;
  const int64_t first = g * GM;
  const int64_t gsz = min(tiles_m - first, GM);
  const int64_t r = t - g * in_group;
  tm = first + r % gsz;
  tn = r / gsz;
}

// One output tile (tile index w of a.total, before the XCD remap).
template <int KR, int TM, int TN, int RM, int RN, int TK, bool VEC>
__device__ __forceinline__ void tgemm_tile(const GemmArgs& a, int64_t w) {
  constexpr int TX = TN / RN;
  constexpr int TY = TM / RM;
  constexpr int NT = TX * TY;
  constexpr int KP = KR > 0 ? KR : 1;
  // A is staged transposed (k-major): consecutive threads write consecutive
  // k of one row, so rows of TM words would put them all in one LDS bank;
  // four words of padding spread them (rows stay 16-byte aligned)
  constexpr int TMP = TM >= 8 ? TM + 4 : TM;
  // one LDS region per operand: rows [0, TK) hold values, rows
  // [(1 + p) TK, (2 + p) TK) residue plane p; the values pass uses all
  // (1 + KP) TK rows as one deeper slice
  __shared__ __attribute__((aligned(16))) uint32_t As[(1 + KP) * TK][TMP];
  __shared__ __attribute__((aligned(16))) uint32_t Bs[(1 + KP) * TK][TN];
  static_assert(sizeof(As) + sizeof(Bs) <= 65536, "tile exceeds 64 KiB of static LDS");
  auto Av = [&](int kk, int i) -> int32_t& { return *(int32_t*)&As[kk][i]; };
  auto Bv = [&](int kk, int i) -> int32_t& { return *(int32_t*)&Bs[kk][i]; };
  auto Ac = [&](int p, int kk, int i) -> uint32_t& { return As[(1 + p) * TK + kk][i]; };
  auto Bc = [&](int p, int kk, int i) -> uint32_t& { return Bs[(1 + p) * TK + kk][i]; };

  int64_t tm_i, tn_i, t;
  tile_coords(xcd_remap(w, a.total), a.tiles_m, a.tiles_n, tm_i, tn_i, t);
  const int64_t sp = t % a.splits;
  const int64_t b = t / a.splits;
  const int64_t m0 = tm_i * TM, n0 = tn_i * TN;
  const int64_t kbeg = sp * a.kchunk;
  const int64_t kend = min(a.K, kbeg + a.kchunk);
  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = tid / TX;
  const uint32_t* Ab = a.A + b * a.sAb;
  const uint32_t* Bb = a.B + b * a.sBb;

  int32_t V[RM][RN];
#pragma unroll
  for (int r = 0; r < RM; ++r)
#pragma unroll
    for (int c = 0; c < RN; ++c) V[r][c] = INT32_MIN;

  // ---- pass 1: values, in slices (1 + KP) times deeper than pass 2's
  {
    constexpr int TK1 = (1 + KP) * TK;
    for (int64_t k0 = kbeg; k0 < kend; k0 += TK1) {
      if (VEC && a.vec_a) {
        // four consecutive k of one row per load (rows and slices are
        // multiples of four words, so a load is wholly in range or out)
        constexpr int KV = TK1 / 4;
#pragma unroll 1
        for (int idx = tid; idx < TM * KV; idx += NT) {
          const int i = idx / KV, j = (idx % KV) * 4;
          const int64_t m = m0 + i, q = k0 + j;
          uint4 v = make_uint4((uint32_t)NEG, (uint32_t)NEG, (uint32_t)NEG, (uint32_t)NEG);
          if (m < a.M && q < kend) v = *(const uint4*)(Ab + m * a.K + q);
          As[j][i] = v.x;
          As[j + 1][i] = v.y;
          As[j + 2][i] = v.z;
          As[j + 3][i] = v.w;
        }
      } else {
        for (int idx = tid; idx < TM * TK1; idx += NT) {
          const int i = idx / TK1, j = idx % TK1;
          const int64_t m = m0 + i, q = k0 + j;
          Av(j, i) = (m < a.M && q < kend) ? (int32_t)Ab[m * a.K + q] : NEG;
        }
      }
      bool vb = false;
      if constexpr (VEC && TN % 4 == 0) {
        if (a.vec_b) {
          vb = true;
          constexpr int NV = TN / 4;
#pragma unroll 1
          for (int idx = tid; idx < TK1 * NV; idx += NT) {
            const int j = idx / NV, i = (idx % NV) * 4;
            const int64_t n = n0 + i, q = k0 + j;
            uint4 v = make_uint4((uint32_t)NEG, (uint32_t)NEG, (uint32_t)NEG, (uint32_t)NEG);
            if (n < a.N && q < kend) v = *(const uint4*)(Bb + q * a.N + n);
            *(uint4*)&Bs[j][i] = v;
          }
        }
      }
      if (!vb) {
        for (int idx = tid; idx < TK1 * TN; idx += NT) {
          const int j = idx / TN, i = idx % TN;
          const int64_t n = n0 + i, q = k0 + j;
          Bv(j, i) = (n < a.N && q < kend) ? (int32_t)Bb[q * a.N + n] : NEG;
        }
      }
      __syncthreads();
#pragma unroll 4
      for (int kk = 0; kk < TK1; ++kk) {
        int32_t av[RM], bv[RN];
#pragma unroll
        for (int r = 0; r < RM; ++r) av[r] = Av(kk, ty * RM + r);
#pragma unroll
        for (int c = 0; c < RN; ++c) bv[c] = Bv(kk, tx * RN + c);
#pragma unroll
        for (int r = 0; r < RM; ++r)
#pragma unroll
          for (int c = 0; c < RN; ++c) V[r][c] = max(V[r][c], av[r] + bv[c]);
      }
      __syncthreads();
    }
  }

  uint64_t acc[KP][RM][RN];
#pragma unroll
  for (int i = 0; i < KP; ++i)
#pragma unroll
    for (int r = 0; r < RM; ++r)
#pragma unroll
      for (int c = 0; c < RN; ++c) acc[i][r][c] = 0;

  if constexpr (KR > 0) {
    int any_finite = 0;
#pragma unroll
    for (int r = 0; r < RM; ++r)
#pragma unroll
      for (int c = 0; c < RN; ++c) any_finite |= (V[r][c] > NEG_CUT);
    uint32_t vm1[RM][RN];
#pragma unroll
    for (int r = 0; r < RM; ++r)
#pragma unroll
      for (int c = 0; c < RN; ++c) vm1[r][c] = (uint32_t)V[r][c] - 1u;
    // ---- pass 2: counts of the q reaching V (skipped by tiles with no
    // finite output, e.g. fully constrained independent-set blocks)
    if (__syncthreads_or(any_finite)) {
      for (int64_t k0 = kbeg; k0 < kend; k0 += TK) {
        // pass 2 stages negated values: the tie test below is one add3
        if (VEC && a.vec_a) {
          constexpr int KV = TK / 4;
  #pragma unroll 1
        for (int idx = tid; idx < TM * KV; idx += NT) {
            const int i = idx / KV, j = (idx % KV) * 4;
            const int64_t m = m0 + i, q = k0 + j;
            const bool in = (m < a.M && q < kend);
            const int64_t o = m * a.K + q;
            uint4 v = make_uint4((uint32_t)NEG, (uint32_t)NEG, (uint32_t)NEG, (uint32_t)NEG);
            if (in) v = *(const uint4*)(Ab + o);
            Av(j, i) = -(int32_t)v.x;
            Av(j + 1, i) = -(int32_t)v.y;
            Av(j + 2, i) = -(int32_t)v.z;
            Av(j + 3, i) = -(int32_t)v.w;
#pragma unroll
            for (int p = 0; p < KR; ++p) {
              uint4 r = make_uint4(0u, 0u, 0u, 0u);
              if (in) r = *(const uint4*)(Ab + (p + 1) * a.pA + o);
              Ac(p, j, i) = r.x;
              Ac(p, j + 1, i) = r.y;
              Ac(p, j + 2, i) = r.z;
              Ac(p, j + 3, i) = r.w;
            }
          }
        } else {
          for (int idx = tid; idx < TM * TK; idx += NT) {
            const int i = idx / TK, j = idx % TK;
            const int64_t m = m0 + i, q = k0 + j;
            const bool in = (m < a.M && q < kend);
            const int64_t o = m * a.K + q;
            Av(j, i) = in ? -(int32_t)Ab[o] : -NEG;
#pragma unroll
            for (int p = 0; p < KR; ++p) Ac(p, j, i) = in ? Ab[(p + 1) * a.pA + o] : 0u;
          }
        }
        bool vb = false;
        if constexpr (VEC && TN % 4 == 0) {
          if (a.vec_b) {
            vb = true;
            constexpr int NV = TN / 4;
#pragma unroll 1
            for (int idx = tid; idx < TK * NV; idx += NT) {
              const int j = idx / NV, i = (idx % NV) * 4;
              const int64_t n = n0 + i, q = k0 + j;
              const bool in = (n < a.N && q < kend);
              const int64_t o = q * a.N + n;
              uint4 v = make_uint4((uint32_t)NEG, (uint32_t)NEG, (uint32_t)NEG, (uint32_t)NEG);
              if (in) v = *(const uint4*)(Bb + o);
              *(uint4*)&Bs[j][i] = make_uint4((uint32_t)(-(int32_t)v.x), (uint32_t)(-(int32_t)v.y),
                                              (uint32_t)(-(int32_t)v.z), (uint32_t)(-(int32_t)v.w));
#pragma unroll
              for (int p = 0; p < KR; ++p) {
                uint4 r = make_uint4(0u, 0u, 0u, 0u);
                if (in) r = *(const uint4*)(Bb + (p + 1) * a.pB + o);
                *(uint4*)&Bs[(1 + p) * TK + j][i] = r;
              }
            }
          }
        }
        if (!vb) {
          for (int idx = tid; idx < TK * TN; idx += NT) {
            const int j = idx / TN, i = idx % TN;
            const int64_t n = n0 + i, q = k0 + j;
            const bool in = (n < a.N && q < kend);
            const int64_t o = q * a.N + n;
            Bv(j, i) = in ? -(int32_t)Bb[o] : -NEG;
#pragma unroll
            for (int p = 0; p < KR; ++p) Bc(p, j, i) = in ? Bb[(p + 1) * a.pB + o] : 0u;
          }
        }
        __syncthreads();
#pragma unroll 3
        for (int kk = 0; kk < TK; ++kk) {
          int32_t av[RM], bv[RN];
          uint32_t ac[KR][RM], bc[KR][RN];
#pragma unroll
          for (int r = 0; r < RM; ++r) av[r] = Av(kk, ty * RM + r);
#pragma unroll
          for (int c = 0; c < RN; ++c) bv[c] = Bv(kk, tx * RN + c);
#pragma unroll
          for (int p = 0; p < KR; ++p) {
#pragma unroll
            for (int r = 0; r < RM; ++r) ac[p][r] = Ac(p, kk, ty * RM + r);
#pragma unroll
            for (int c = 0; c < RN; ++c) bc[p][c] = Bc(p, kk, tx * RN + c);
          }
          // tie test without a compare: x = V - 1 - a - b is -1 exactly on a
          // tie and >= 0 otherwise (a + b <= V), so x >> 31 is the tie mask.
          // Sums that wrap involve stored zeros, whose residues are 0.
#pragma unroll
          for (int r = 0; r < RM; ++r)
#pragma unroll
            for (int c = 0; c < RN; ++c) {
              const uint32_t x = (uint32_t)av[r] + (uint32_t)bv[c] + vm1[r][c];
              const uint32_t msk = (uint32_t)((int32_t)x >> 31);
#pragma unroll
              for (int p = 0; p < KR; ++p)
                acc[p][r][c] += (uint64_t)(ac[p][r] & msk) * bc[p][c];
            }
          // at most three products (< 2^62 each) between folds (< 2^54)
          if (kk % 3 == 2 || kk == TK - 1) {
#pragma unroll
            for (int p = 0; p < KR; ++p)
#pragma unroll
              for (int r = 0; r < RM; ++r)
#pragma unroll
                for (int c = 0; c < RN; ++c) acc[p][r][c] = fold64(acc[p][r][c], a.mod.c[p]);
          }
        }
        __syncthreads();
      }
    }
  }

  // ---- write
#pragma unroll
  for (int r = 0; r < RM; ++r) {
    const int64_t m = m0 + ty * RM + r;
#pragma unroll
    for (int c = 0; c < RN; ++c) {
      const int64_t n = n0 + tx * RN + c;
      if (m < a.M && n < a.N) {
        const int64_t off = sp * a.sCsplit + b * a.sCb + m * a.N + n;
        const bool fin = V[r][c] > NEG_CUT;
        a.C[off] = (uint32_t)(fin ? V[r][c] : NEG);
        if constexpr (KR > 0) {
#pragma unroll
          for (int p = 0; p < KR; ++p)
            a.C[(p + 1) * a.pC + off] =
                fin ? mod_final(acc[p][r][c], a.mod.p[p], a.mod.c[p]) : 0u;
        }
      }
    }
  }
}

// Waves per SIMD the compiler must leave room for: three for the 32 x 64
// tile with 12-deep slices and four or more residues (its LDS allows five
// workgroups per CU; its registers alone would allow two), else no bound.
template <int KR, int TM, int TN, int TK>
constexpr int kMinWaves = (KR >= 4 && TM == 32 && TN == 64 && TK <= 12) ? 3 : 1;

template <int KR, int TM, int TN, int RM, int RN, int TK, bool VEC>
__global__ void __launch_bounds__((TM / RM) * (TN / RN), (kMinWaves<KR, TM, TN, TK>))
tgemm_kernel(const GemmArgs a) {
  tgemm_tile<KR, TM, TN, RM, RN, TK, VEC>(a, blockIdx.x);
}

// Grids beyond 2^20 tiles: each workgroup walks the tiles with the grid's
// stride (a dispatch must stay below 2^32 work-items).  The stride is a
// multiple of 8, so every tile a workgroup takes maps to the same XCD.
template <int KR, int TM, int TN, int RM, int RN, int TK, bool VEC>
__global__ void __launch_bounds__((TM / RM) * (TN / RN), (kMinWaves<KR, TM, TN, TK>))
tgemm_kernel_strided(const GemmArgs a) {
  for (int64_t w = blockIdx.x; w < a.total; w += gridDim.x) {
    tgemm_tile<KR, TM, TN, RM, RN, TK, VEC>(a, w);
    __syncthreads();  // LDS is restaged for the next tile
  }
}

// ------------------------------------------------------------ thin products
// Products with a short summed range and a narrow side (K <= 32 and M or N
// below 32, power-of-two sizes) move far more bytes than they compute, and
// the LDS tiles above would leave most of their lanes idle.  Here one thread
// computes one output, outputs in memory order (n fastest), with no LDS:
// lanes of a wave that share a row of A read it in one request and lanes
// with consecutive n read consecutive words of B and write consecutive
// words of C.  Values first (max over q), then the counts of the q that
// reach the maximum, as in the tiled kernel.
template <int KR>
__global__ void __launch_bounds__(256) tgemm_thin_kernel(const GemmArgs a, int lm, int ln, int lk) {
  constexpr int KP = KR > 0 ? KR : 1;
  const int64_t total = a.batch << (lm + ln);
  const int K = 1 << lk;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * 256) {
    const int64_t n = t & ((1ll << ln) - 1);
    const int64_t m = (t >> ln) & ((1ll << lm) - 1);
    const int64_t b = t >> (lm + ln);
    const uint32_t* Ar = a.A + b * a.sAb + (m << lk);
    const uint32_t* Bc = a.B + b * a.sBb + n;
    int32_t V = INT32_MIN;
#pragma unroll 4
    for (int q = 0; q < K; ++q) V = max(V, (int32_t)Ar[q] + (int32_t)Bc[(int64_t)q << ln]);
    const bool fin = V > NEG_CUT;
    const int64_t off = b * a.sCb + (m << ln) + n;
    a.C[off] = (uint32_t)(fin ? V : NEG);
    if constexpr (KR > 0) {
      uint64_t acc[KP];
#pragma unroll
      for (int p = 0; p < KP; ++p) acc[p] = 0;
      if (fin) {
        for (int q = 0; q < K; ++q) {
          const int64_t ia = q, ib = (int64_t)q << ln;
          if ((int32_t)Ar[ia] + (int32_t)Bc[ib] != V) continue;
#pragma unroll
          for (int p = 0; p < KR; ++p) {
            acc[p] += (uint64_t)Ar[(p + 1) * a.pA + ia] * Bc[(p + 1) * a.pB + ib];
            acc[p] = fold64(acc[p], a.mod.c[p]);
          }
        }
      }
#pragma unroll
      for (int p = 0; p < KR; ++p)
        a.C[(p + 1) * a.pC + off] = fin ? mod_final(acc[p], a.mod.p[p], a.mod.c[p]) : 0u;
    }
  }
}

// Copies n <= 256 * PER words into LDS, word e from src[index(e)], with
// every load of a thread issued before its first LDS store.
template <int PER, typename F>
__device__ __forceinline__ void stage_words(uint32_t* dst, int n, int tid, F src) {
  uint32_t v[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int e = tid + 256 * j;
    if (e < n) v[j] = src(e);
  }
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int e = tid + 256 * j;
    if (e < n) dst[e] = v[j];
  }
}

// Staged thin products for large contiguous operands (A rows, B and C
// without batch gaps).  The one-thread-per-output kernel above re-reads the
// wide operand once per row of the narrow side, and with gigabyte operands
// those re-reads miss the caches.  Here a workgroup stages one block of the
// wide operand and the whole narrow operand in LDS with consecutive lanes
// reading consecutive words, then computes the block's outputs from LDS and
// writes them in memory order: every operand word crosses HBM once.
//
// Rows form (N <= 16): the block is BR consecutive rows r = b * M + m of A
// (BR * K contiguous words) with the B matrices of the batches they belong
// to (contiguous too); its outputs are BR * N contiguous words of C.
template <int KR>
__global__ void __launch_bounds__(256)
tgemm_thin_rows_kernel(const GemmArgs a, int lm, int ln, int lk, int lbr, int b_cap) {
  constexpr int W = 1 + KR;
  extern __shared__ __attribute__((aligned(16))) uint32_t sm[];
  const int a_cap = 1 << (lbr + lk);
  uint32_t* const As = sm;               // W planes of a_cap words
  uint32_t* const Bs = sm + W * a_cap;   // W planes of b_cap words
  const int tid = threadIdx.x;
  const int64_t R = a.batch << lm;
  const int64_t tiles = (R + (1 << lbr) - 1) >> lbr;
  const int N = 1 << ln, K = 1 << lk;
  for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int64_t r0 = tile << lbr;
    const int rows = (int)min<int64_t>((int64_t)1 << lbr, R - r0);
    const int64_t b0 = r0 >> lm;
    const int nb = (int)(((r0 + rows - 1) >> lm) - b0 + 1);
    const int na = rows << lk, nbe = nb << (lk + ln);
#pragma unroll
    for (int p = 0; p < W; ++p) {
      const uint32_t* srcA = a.A + p * a.pA + (r0 << lk);
      stage_words<4>(As + p * a_cap, na, tid, [&](int e) { return srcA[e]; });
      const uint32_t* srcB = a.B + p * a.pB + (b0 << (lk + ln));
      stage_words<4>(Bs + p * b_cap, nbe, tid, [&](int e) { return srcB[e]; });
    }
    __syncthreads();
    const int nout = rows << ln;
    for (int o = tid; o < nout; o += 256) {
      const int rl = o >> ln, n = o & (N - 1);
      const int bl = (int)(((r0 + rl) >> lm) - b0);
      const int ia0 = rl << lk, ib0 = (bl << (lk + ln)) + n;
      int32_t V = INT32_MIN;
      for (int q = 0; q < K; ++q) V = max(V, (int32_t)As[ia0 + q] + (int32_t)Bs[ib0 + (q << ln)]);
      const bool fin = V > NEG_CUT;
      const int64_t off = (r0 << ln) + o;
      a.C[off] = (uint32_t)(fin ? V : NEG);
      if constexpr (KR > 0) {
        uint64_t acc[KR];
#pragma unroll
        for (int p = 0; p < KR; ++p) acc[p] = 0;
        if (fin) {
          for (int q = 0; q < K; ++q) {
            const int ia = ia0 + q, ib = ib0 + (q << ln);
            if ((int32_t)As[ia] + (int32_t)Bs[ib] != V) continue;
#pragma unroll
            for (int p = 0; p < KR; ++p) {
              acc[p] += (uint64_t)As[(p + 1) * a_cap + ia] * Bs[(p + 1) * b_cap + ib];
              acc[p] = fold64(acc[p], a.mod.c[p]);
            }
          }
        }
#pragma unroll
        for (int p = 0; p < KR; ++p)
          a.C[(p + 1) * a.pC + off] = fin ? mod_final(acc[p], a.mod.p[p], a.mod.c[p]) : 0u;
      }
    }
    __syncthreads();
  }
}

// Columns form (M <= 16, N >= 32): the block is BN consecutive columns
// n0.. of one batch's B (K segments of BN contiguous words) with that
// batch's whole A (M * K words); its outputs are M segments of BN
// contiguous words of C.
template <int KR>
__global__ void __launch_bounds__(256)
tgemm_thin_cols_kernel(const GemmArgs a, int lm, int ln, int lk, int lbn) {
  constexpr int W = 1 + KR;
  extern __shared__ __attribute__((aligned(16))) uint32_t sm[];
  const int a_cap = 1 << (lm + lk), b_cap = 1 << (lk + lbn);
  uint32_t* const As = sm;
  uint32_t* const Bs = sm + W * a_cap;
  const int tid = threadIdx.x;
  const int K = 1 << lk, BN = 1 << lbn;
  const int lblk = ln - lbn;  // column blocks per batch (log2)
  const int64_t tiles = a.batch << lblk;
  for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int64_t b = tile >> lblk;
    const int64_t n0 = (tile & ((1ll << lblk) - 1)) << lbn;
#pragma unroll
    for (int p = 0; p < W; ++p) {
      const uint32_t* srcA = a.A + p * a.pA + (b << (lm + lk));
      stage_words<2>(As + p * a_cap, a_cap, tid, [&](int e) { return srcA[e]; });
      const uint32_t* srcB = a.B + p * a.pB + (b << (lk + ln)) + n0;
      stage_words<8>(Bs + p * b_cap, b_cap, tid, [&](int e) {
        return srcB[((int64_t)(e >> lbn) << ln) + (e & (BN - 1))];
      });
    }
    __syncthreads();
    const int nout = 1 << (lm + lbn);
    for (int o = tid; o < nout; o += 256) {
      const int j = o & (BN - 1), m = o >> lbn;
      const int ia0 = m << lk;
      int32_t V = INT32_MIN;
      for (int q = 0; q < K; ++q) V = max(V, (int32_t)As[ia0 + q] + (int32_t)Bs[(q << lbn) + j]);
      const bool fin = V > NEG_CUT;
      const int64_t off = (b << (lm + ln)) + ((int64_t)m << ln) + n0 + j;
      a.C[off] = (uint32_t)(fin ? V : NEG);
      if constexpr (KR > 0) {
        uint64_t acc[KR];
#pragma unroll
        for (int p = 0; p < KR; ++p) acc[p] = 0;
        if (fin) {
          for (int q = 0; q < K; ++q) {
            const int ia = ia0 + q, ib = (q << lbn) + j;
            if ((int32_t)As[ia] + (int32_t)Bs[ib] != V) continue;
#pragma unroll
            for (int p = 0; p < KR; ++p) {
              acc[p] += (uint64_t)As[(p + 1) * a_cap + ia] * Bs[(p + 1) * b_cap + ib];
              acc[p] = fold64(acc[p], a.mod.c[p]);
            }
          }
        }
#pragma unroll
        for (int p = 0; p < KR; ++p)
          a.C[(p + 1) * a.pC + off] = fin ? mod_final(acc[p], a.mod.p[p], a.mod.c[p]) : 0u;
      }
    }
    __syncthreads();
  }
}

static int exact_log2(int64_t x) {
  if (x <= 0 || (x & (x - 1))) return -1;
  int l = 0;
  while ((1ll << l) < x) ++l;
  return l;
}

// The thin kernel applies: unsplit, power-of-two sizes, K <= 32 and M or N
// below 32.
static bool thin_shape(const GemmShape& s, int splits) {
  const int lm = exact_log2(s.M), ln = exact_log2(s.N), lk = exact_log2(s.K);
  return splits <= 1 && lm >= 0 && ln >= 0 && lk >= 0 && lk <= 5 && (lm < 5 || ln < 5);
}

bool tgemm_is_thin(const GemmShape& s, int splits) { return thin_shape(s, splits); }

// Staged forms, for contiguous operands with at least 4096 outputs.  LDS
// words per plane: A block <= 1024 and B block <= 1024 (rows), A <= 512 and
// B block <= 2048 (columns), so that six planes stay within 64 KiB.
static bool launch_thin_staged(int k, const GemmArgs& a, int lm, int ln, int lk,
                               hipStream_t st) {
  if (a.sAb != a.M * a.K || a.sBb != a.K * a.N || a.sCb != a.M * a.N) return false;
  const int64_t total = a.batch << (lm + ln);
  if (total < 4096) return false;
  const int W = 1 + k;
  if (ln < 5) {
    // rows: BR * K <= 1024 and the batches of a block: ceil(BR / M) * K * N <= 1024
    int lbr = 10 - lk;
    while (lbr > 0 && (lbr > lm ? (1 << (lbr - lm)) : 1) * (1 << (lk + ln)) > 1024) --lbr;
    const int64_t R = a.batch << lm;
    while (lbr > 0 && ((int64_t)1 << lbr) > R) --lbr;
    // blocks start at multiples of BR (M and BR are powers of two): a block
    // holds BR / M whole batches, or lies within one
    const int b_cap = (lbr > lm ? (1 << (lbr - lm)) : 1) << (lk + ln);
    const size_t lds = (size_t)W * ((1u << (lbr + lk)) + b_cap) * 4;
    const int64_t tiles = (R + (1 << lbr) - 1) >> lbr;
    dim3 grid((unsigned)std::min<int64_t>(tiles, 256 * 256)), block(256);
    switch (k) {
#define BBTN_TR(KK) case KK: launch_kernel(tgemm_thin_rows_kernel<KK>, grid, block, (uint32_t)lds, st, true, a, lm, ln, lk, lbr, b_cap); break;
      BBTN_TR(0) BBTN_TR(1) BBTN_TR(2) BBTN_TR(3) BBTN_TR(4) BBTN_TR(5)
#undef BBTN_TR
      default: throw Error(BBTN_E_INVALID_ARG, "k must be in [0, 5]");
    }
    BBTN_LAUNCHED("tgemm (thin rows)");
    return true;
  }
  if (lm < 5) {
    // columns: K * BN <= 2048, BN <= N, M * K <= 512 always
    int lbn = std::min(ln, 11 - lk);
    lbn = std::min(lbn, 10);
    const size_t lds = (size_t)W * ((1u << (lm + lk)) + (1u << (lk + lbn))) * 4;
    const int64_t tiles = a.batch << (ln - lbn);
    dim3 grid((unsigned)std::min<int64_t>(tiles, 256 * 256)), block(256);
    switch (k) {
#define BBTN_TC(KK) case KK: launch_kernel(tgemm_thin_cols_kernel<KK>, grid, block, (uint32_t)lds, st, true, a, lm, ln, lk, lbn); break;
      BBTN_TC(0) BBTN_TC(1) BBTN_TC(2) BBTN_TC(3) BBTN_TC(4) BBTN_TC(5)
#undef BBTN_TC
      default: throw Error(BBTN_E_INVALID_ARG, "k must be in [0, 5]");
    }
    BBTN_LAUNCHED("tgemm (thin columns)");
    return true;
  }
  return false;
}

static void launch_thin(int k, const GemmArgs& a, hipStream_t st) {
  const int lm = exact_log2(a.M), ln = exact_log2(a.N), lk = exact_log2(a.K);
  if (launch_thin_staged(k, a, lm, ln, lk, st)) return;
  const int64_t total = a.batch << (lm + ln);
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, 256 * 256);
  dim3 grid((unsigned)blocks), block(256);
  switch (k) {
    case 0: launch_kernel(tgemm_thin_kernel<0>, grid, block, 0, st, true, a, lm, ln, lk); break;
    case 1: launch_kernel(tgemm_thin_kernel<1>, grid, block, 0, st, true, a, lm, ln, lk); break;
    case 2: launch_kernel(tgemm_thin_kernel<2>, grid, block, 0, st, true, a, lm, ln, lk); break;
    case 3: launch_kernel(tgemm_thin_kernel<3>, grid, block, 0, st, true, a, lm, ln, lk); break;
    case 4: launch_kernel(tgemm_thin_kernel<4>, grid, block, 0, st, true, a, lm, ln, lk); break;
    case 5: launch_kernel(tgemm_thin_kernel<5>, grid, block, 0, st, true, a, lm, ln, lk); break;
    default: throw Error(BBTN_E_INVALID_ARG, "k must be in [0, 5]");
  }
  BBTN_LAUNCHED("tgemm (thin, grid " + std::to_string(total) + ")");
}

// ------------------------------------------------ values in packed 16 bits
// Max-plus product (values only) with two values per 32-bit word: the
// operands' finite values satisfy |v| < 2^12 (the caller's guarantee: the
// sum of the network's |couplings| and |fields|, or of its weights, bounds
// every partial sum), so in 16 bits a finite sum lies in (-2^13, 2^13), a
// sum with a stored zero (-2^14 in 16 bits) lies below -2^13 + 1 and two
// stored zeros give -2^15 exactly: no sum wraps.  Each thread keeps RM x RN
// outputs as RM x RN/2 pairs of adjacent columns; one packed add and one
// packed max (v_pk_add_u16, v_pk_max_i16) advance two outputs by one q.
// A is staged with its value in both halves, B as pairs of adjacent columns.
typedef short s16x2 __attribute__((ext_vector_type(2)));
constexpr int32_t NEG16 = -(1 << 14);
constexpr int32_t NEG_CUT16 = -(1 << 13);

__device__ __forceinline__ uint32_t to16(int32_t v) {
  return (uint32_t)(uint16_t)(int16_t)(v > NEG_CUT ? v : NEG16);
}

// Moves the N items of a tile slice through registers: thread tid handles
// items tid, tid + NT, ..., loading G of them (all in flight together)
// before storing those G, which bounds the registers the batch holds.
template <int NT, int N, int G = 4, typename Load, typename Store>
__device__ __forceinline__ void stage_tile(int tid, Load ld, Store stv) {
  constexpr int PER = (N + NT - 1) / NT;
  constexpr int GG = PER < G ? PER : G;
#pragma unroll 1
  for (int u0 = 0; u0 < PER; u0 += GG) {
    decltype(ld(0)) v[GG];
#pragma unroll
    for (int u = 0; u < GG; ++u) {
      const int idx = tid + (u0 + u) * NT;
      if ((N % NT == 0 && PER % GG == 0) || (u0 + u < PER && idx < N)) v[u] = ld(idx);
    }
#pragma unroll
    for (int u = 0; u < GG; ++u) {
      const int idx = tid + (u0 + u) * NT;
      if ((N % NT == 0 && PER % GG == 0) || (u0 + u < PER && idx < N)) stv(idx, v[u]);
    }
  }
}

// perm of x over layout bits [lo, lo + n)
__device__ __forceinline__ int64_t fperm(const FusedOp& f, int64_t x, int lo, int n) {
  int64_t r = 0;
  for (int j = 0; j < n; ++j)
    if ((x >> j) & 1) r |= 1ll << f.bits[lo + j];
  return r;
}

template <int TM, int TN, int RM, int RN, int TK, bool FA = false, bool FB = false>
__device__ __forceinline__ void tgemm_v16_tile(const GemmArgs& a, int64_t w, const FusedOp& fa,
                                               const FusedOp& fb) {
  constexpr int TX = TN / RN, TY = TM / RM, NT = TX * TY;
  constexpr int RP = RN / 2;          // packed column pairs per thread
  constexpr int TMP = TM + 4;         // padded rows of the transposed A tile
  // loads in flight per thread while staging: four for the 64-wide tiles,
  // two (one when reading in place) for the 128-wide ones, whose 32
  // accumulator registers leave less room (more would cut their occupancy)
  constexpr int SG = TM < 128 ? 4 : (FA || FB) ? 1 : 2;
  __shared__ __attribute__((aligned(16))) uint32_t As[TK][TMP];
  __shared__ __attribute__((aligned(16))) uint32_t Bs[TK][TN / 2];
  // fused operands: source offsets of the tile's low row and k indices
  __shared__ int32_t a_row[FA ? TM : 1], a_k[FA ? TK : 1], b_col[FB ? TN : 1], b_k[FB ? TK : 1];
  int64_t tm_i, tn_i, t;
  tile_coords(xcd_remap(w, a.total), a.tiles_m, a.tiles_n, tm_i, tn_i, t);
  const int64_t sp = t % a.splits;
  const int64_t b = t / a.splits;
  const int64_t m0 = tm_i * TM, n0 = tn_i * TN;
  const int64_t kbeg = sp * a.kchunk;
  const int64_t kend = min(a.K, kbeg + a.kchunk);
  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = tid / TX;
  const uint32_t* Ab = a.A + b * a.sAb;
  const uint32_t* Bb = a.B + b * a.sBb;
  // log2 sizes (M, N, K are powers of two on the fused paths)
  int lm = 0, ln = 0, lk = 0;
  const uint32_t* fsA = nullptr;
  const uint32_t* fsB = nullptr;
  if constexpr (FA || FB) {
    while ((1ll << lm) < a.M) ++lm;
    while ((1ll << ln) < a.N) ++ln;
    while ((1ll << lk) < a.K) ++lk;
  }
  if constexpr (FA) {
    // A layout bits: k [0, lk), m [lk, lk + lm), batch [lk + lm, + rb)
    const int64_t l = b >> fa.rb, bb = b & ((1ll << fa.rb) - 1);
    fsA = fa.src + l * fa.stride + (fperm(fa, m0, lk, lm) | fperm(fa, bb, lk + lm, fa.rb));
    for (int i = tid; i < TM; i += NT) a_row[i] = (int32_t)fperm(fa, i, lk, lm);
    for (int j = tid; j < TK; j += NT) a_k[j] = (int32_t)fperm(fa, j, 0, lk);
  }
  if constexpr (FB) {
    // B layout bits: n [0, ln), k [ln, ln + lk), batch [ln + lk, + rb)
    const int64_t l = b >> fb.rb, bb = b & ((1ll << fb.rb) - 1);
    fsB = fb.src + l * fb.stride + (fperm(fb, n0, 0, ln) | fperm(fb, bb, ln + lk, fb.rb));
    for (int i = tid; i < TN; i += NT) b_col[i] = (int32_t)fperm(fb, i, 0, ln);
    for (int j = tid; j < TK; j += NT) b_k[j] = (int32_t)fperm(fb, j, ln, lk);
  }
  if constexpr (FA || FB) __syncthreads();
  s16x2 V[RM][RP];
#pragma unroll
  for (int r = 0; r < RM; ++r)
#pragma unroll
    for (int c = 0; c < RP; ++c) V[r][c] = s16x2{-32768, -32768};
  for (int64_t k0 = kbeg; k0 < kend; k0 += TK) {
    // Staging: each thread issues all of its loads of the slice before its
    // first LDS store (stage_tile), so they are in flight together.
    if constexpr (FA) {
      const uint32_t* src = fsA + fperm(fa, k0, 0, lk);
      if (fa.fast) {
        stage_tile<NT, TM * TK, SG>(tid, [&](int idx) {
          const int i = idx % TM, j = idx / TM;
          return (m0 + i < a.M && k0 + j < kend) ? (int32_t)src[a_row[i] | a_k[j]] : NEG;
        }, [&](int idx, int32_t v) { As[idx / TM][idx % TM] = to16(v) * 0x10001u; });
      } else {
        stage_tile<NT, TM * TK, SG>(tid, [&](int idx) {
          const int i = idx / TK, j = idx % TK;
          return (m0 + i < a.M && k0 + j < kend) ? (int32_t)src[a_row[i] | a_k[j]] : NEG;
        }, [&](int idx, int32_t v) { As[idx % TK][idx / TK] = to16(v) * 0x10001u; });
      }
    } else if (a.vec_a) {
      constexpr int KV = TK / 4;
      stage_tile<NT, TM * KV, SG>(tid, [&](int idx) {
        const int64_t m = m0 + idx / KV, q = k0 + (idx % KV) * 4;
        uint4 v = make_uint4((uint32_t)NEG, (uint32_t)NEG, (uint32_t)NEG, (uint32_t)NEG);
        if (m < a.M && q < kend) v = *(const uint4*)(Ab + m * a.K + q);
        return v;
      }, [&](int idx, uint4 v) {
        const int i = idx / KV, j = (idx % KV) * 4;
        As[j][i] = to16((int32_t)v.x) * 0x10001u;
        As[j + 1][i] = to16((int32_t)v.y) * 0x10001u;
        As[j + 2][i] = to16((int32_t)v.z) * 0x10001u;
        As[j + 3][i] = to16((int32_t)v.w) * 0x10001u;
      });
    } else {
      stage_tile<NT, TM * TK, SG>(tid, [&](int idx) {
        const int64_t m = m0 + idx / TK, q = k0 + idx % TK;
        return (m < a.M && q < kend) ? (int32_t)Ab[m * a.K + q] : NEG;
      }, [&](int idx, int32_t v) { As[idx % TK][idx / TK] = to16(v) * 0x10001u; });
    }
    if constexpr (FB) {
      const uint32_t* src = fsB + fperm(fb, k0, ln, lk);
      if (fb.fast) {
        stage_tile<NT, TK * (TN / 2), SG>(tid, [&](int idx) {
          const int j = idx / (TN / 2), i = (idx % (TN / 2)) * 2;
          const bool in = k0 + j < kend;
          const int32_t v0 = (in && n0 + i < a.N) ? (int32_t)src[b_col[i] | b_k[j]] : NEG;
          const int32_t v1 = (in && n0 + i + 1 < a.N) ? (int32_t)src[b_col[i + 1] | b_k[j]] : NEG;
          return make_int2(v0, v1);
        }, [&](int idx, int2 v) {
          Bs[idx / (TN / 2)][idx % (TN / 2)] = to16(v.x) | to16(v.y) << 16;
        });
      } else {
        stage_tile<NT, TK * (TN / 2), SG>(tid, [&](int idx) {
          const int j = idx % TK, i = (idx / TK) * 2;
          const bool in = k0 + j < kend;
          const int32_t v0 = (in && n0 + i < a.N) ? (int32_t)src[b_col[i] | b_k[j]] : NEG;
          const int32_t v1 = (in && n0 + i + 1 < a.N) ? (int32_t)src[b_col[i + 1] | b_k[j]] : NEG;
          return make_int2(v0, v1);
        }, [&](int idx, int2 v) {
          Bs[idx % TK][idx / TK] = to16(v.x) | to16(v.y) << 16;
        });
      }
    } else if (a.vec_b) {
      constexpr int NV = TN / 4;
      stage_tile<NT, TK * NV, SG>(tid, [&](int idx) {
        const int64_t n = n0 + (idx % NV) * 4, q = k0 + idx / NV;
        uint4 v = make_uint4((uint32_t)NEG, (uint32_t)NEG, (uint32_t)NEG, (uint32_t)NEG);
        if (n < a.N && q < kend) v = *(const uint4*)(Bb + q * a.N + n);
        return v;
      }, [&](int idx, uint4 v) {
        *(uint2*)&Bs[idx / NV][(idx % NV) * 2] =
            make_uint2(to16((int32_t)v.x) | to16((int32_t)v.y) << 16,
                       to16((int32_t)v.z) | to16((int32_t)v.w) << 16);
      });
    } else {
      stage_tile<NT, TK * (TN / 2), SG>(tid, [&](int idx) {
        const int j = idx / (TN / 2), i = (idx % (TN / 2)) * 2;
        const int64_t n = n0 + i, q = k0 + j;
        const bool in = q < kend;
        const int32_t v0 = (in && n < a.N) ? (int32_t)Bb[q * a.N + n] : NEG;
        const int32_t v1 = (in && n + 1 < a.N) ? (int32_t)Bb[q * a.N + n + 1] : NEG;
        return make_int2(v0, v1);
      }, [&](int idx, int2 v) {
        Bs[idx / (TN / 2)][idx % (TN / 2)] = to16(v.x) | to16(v.y) << 16;
      });
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < TK; ++kk) {
      s16x2 av[RM], bv[RP];
#pragma unroll
      for (int r = 0; r < RM; ++r) av[r] = __builtin_bit_cast(s16x2, As[kk][ty * RM + r]);
#pragma unroll
      for (int c = 0; c < RP; ++c) bv[c] = __builtin_bit_cast(s16x2, Bs[kk][tx * RP + c]);
#pragma unroll
      for (int r = 0; r < RM; ++r)
#pragma unroll
        for (int c = 0; c < RP; ++c) V[r][c] = __builtin_elementwise_max(V[r][c], av[r] + bv[c]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < RM; ++r) {
    const int64_t m = m0 + ty * RM + r;
    if (m >= a.M) continue;
#pragma unroll
    for (int c = 0; c < RP; ++c) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int64_t n = n0 + tx * RN + 2 * c + h;
        if (n < a.N) {
          const int32_t v = V[r][c][h];
          a.C[sp * a.sCsplit + b * a.sCb + m * a.N + n] = (uint32_t)(v > NEG_CUT16 ? v : NEG);
        }
      }
    }
  }
}

// The 64-wide tiles are held to five waves per SIMD (at most 102 registers;
// they need about 110 unbounded, which allows four).
template <int TM, int TN, int RM, int RN, int TK>
__global__ void __launch_bounds__((TM / RM) * (TN / RN), (TM < 128 ? 5 : 1))
tgemm_v16_kernel(const GemmArgs a) {
  const FusedOp none{};
  for (int64_t w = blockIdx.x; w < a.total; w += gridDim.x) {
    tgemm_v16_tile<TM, TN, RM, RN, TK>(a, w, none, none);
    __syncthreads();
  }
}

template <int TM, int TN, int RM, int RN, int TK, bool FA, bool FB>
__global__ void __launch_bounds__((TM / RM) * (TN / RN), (TM < 128 ? 5 : 1))
tgemm_v16_fused_kernel(const GemmArgs a, const FusedOp fa, const FusedOp fb) {
  for (int64_t w = blockIdx.x; w < a.total; w += gridDim.x) {
    tgemm_v16_tile<TM, TN, RM, RN, TK, FA, FB>(a, w, fa, fb);
    __syncthreads();
  }
}

// Tiles of the packed kernel: 128 x 128 outputs, 8 x 8 per thread, 32-deep
// slices; products with M or N below 128 take 64 x 64 tiles, 4 x 4 per
// thread (less of the tile past the edge).
constexpr int V16_TM = 128, V16_TN = 128, V16_RM = 8, V16_RN = 8, V16_TK = 32;
constexpr int V16S_TM = 64, V16S_TN = 64, V16S_RM = 4, V16S_RN = 4;

// LDS slice depth for KR residues: the configuration's TK, halved while the
// tile's operand slices (values and KR residue planes) would pass 64 KiB.
constexpr int tk_for(int KR, int TM, int TN, int TK) {
  const int kp = KR > 0 ? KR : 1;
  const int tmp = TM >= 8 ? TM + 4 : TM;
  int tk = TK;
  while ((1 + kp) * tk * (tmp + TN) * 4 > 65536) tk /= 2;
  return tk;
}

template <int KR>
static void launch_cfg(int cfg, dim3 grid, const GemmArgs& a, hipStream_t st, bool last) {
  switch (cfg) {
#define BBTN_TG_CASE(I, TM, TN, RM, RN, TK, VEC)                                  \
  case I: {                                                                        \
    constexpr int TKK = tk_for(KR, TM, TN, TK);                                    \
    if (a.total == (int64_t)grid.x)                                                \
      launch_kernel((tgemm_kernel<KR, TM, TN, RM, RN, TKK, VEC>), grid,             \
                    dim3((TM / RM) * (TN / RN)), 0, st, last, a);                  \
    else                                                                           \
      launch_kernel((tgemm_kernel_strided<KR, TM, TN, RM, RN, TKK, VEC>), grid,     \
                    dim3((TM / RM) * (TN / RN)), 0, st, last, a);                  \
  }                                                                                \
    break;
    BBTN_TG_CASE(0, 64, 64, 4, 4, 24, false)
    BBTN_TG_CASE(1, 32, 32, 2, 2, 24, false)
    BBTN_TG_CASE(2, 16, 16, 1, 1, 16, false)
    BBTN_TG_CASE(3, 8, 64, 1, 2, 16, false)
    BBTN_TG_CASE(4, 64, 8, 2, 1, 16, false)
    BBTN_TG_CASE(5, 1, 256, 1, 1, 12, false)
    BBTN_TG_CASE(6, 256, 1, 1, 1, 12, false)
    BBTN_TG_CASE(7, 64, 32, 4, 2, 24, false)
    BBTN_TG_CASE(8, 32, 64, 2, 4, 24, false)
    BBTN_TG_CASE(9, 64, 64, 4, 4, 24, true)
    BBTN_TG_CASE(10, 64, 32, 4, 2, 24, true)
    BBTN_TG_CASE(11, 32, 64, 2, 4, 24, true)
    BBTN_TG_CASE(12, 32, 64, 2, 4, 12, true)
#undef BBTN_TG_CASE
    default:
      throw Error(BBTN_E_INTERNAL, "bad tile config");
  }
}

static void launch_core(int k, const GemmArgs& a0, int cfg, hipStream_t st, bool last = true) {
  const TileCfg& tc = kTileCfgs[cfg];
  GemmArgs a = a0;
  a.tiles_m = (a.M + tc.tm - 1) / tc.tm;
  a.tiles_n = (a.N + tc.tn - 1) / tc.tn;
  const int64_t total = a.tiles_m * a.tiles_n * a.splits * a.batch;
  BBTN_REQUIRE(total > 0, "empty tgemm grid");
  a.total = total;
  // four-word staging needs 16-byte aligned rows, planes and batches, and K
  // slices that are whole multiples of four
  auto al16 = [](const void* p) { return ((uintptr_t)p & 15u) == 0; };
  a.vec_a = a.K % 4 == 0 && a.kchunk % 4 == 0 && al16(a.A) && (k == 0 || a.pA % 4 == 0) &&
            (a.batch == 1 || a.sAb % 4 == 0);
  a.vec_b = a.N % 4 == 0 && al16(a.B) && (k == 0 || a.pB % 4 == 0) &&
            (a.batch == 1 || a.sBb % 4 == 0);
  // at most 2^20 workgroups of <= 256 threads, a multiple of 8 when capped
  const int64_t cap = 1ll << 20;
  dim3 grid((unsigned)(total <= cap ? total : cap));
  switch (k) {
    case 0: launch_cfg<0>(cfg, grid, a, st, last); break;
    case 1: launch_cfg<1>(cfg, grid, a, st, last); break;
    case 2: launch_cfg<2>(cfg, grid, a, st, last); break;
    case 3: launch_cfg<3>(cfg, grid, a, st, last); break;
    case 4: launch_cfg<4>(cfg, grid, a, st, last); break;
    case 5: launch_cfg<5>(cfg, grid, a, st, last); break;
    default: throw Error(BBTN_E_INVALID_ARG, "k must be in [0, 5]");
  }
  BBTN_LAUNCHED("tgemm (tile config " + std::to_string(cfg) + ", k " + std::to_string(k) +
                ", grid " + std::to_string(total) + ")");
}

void launch_tgemm(int k, const Moduli& mod, const GemmShape& s, DevTensor A,
                  DevTensor B, DevTensor C, int cfg, int splits,
                  DevTensor partial, hipStream_t st) {
  BBTN_REQUIRE(cfg >= 0 && cfg < N_TILE_CFGS, "tile config out of range");
  BBTN_REQUIRE(s.M >= 1 && s.N >= 1 && s.K >= 1 && s.batch >= 1, "empty tgemm");
  GemmArgs a{};
  a.A = A.ptr; a.B = B.ptr;
  a.pA = A.pstride; a.pB = B.pstride;
  a.M = s.M; a.N = s.N; a.K = s.K; a.batch = s.batch;
  a.sAb = s.sAb; a.sBb = s.sBb;
  a.mod = mod;
  const int tk = kTileCfgs[cfg].tk;
  if (splits <= 1 || s.K <= tk) {
    a.C = C.ptr; a.pC = C.pstride; a.sCb = s.sCb; a.sCsplit = 0;
    a.splits = 1; a.kchunk = s.K;
    if (thin_shape(s, 1)) launch_thin(k, a, st);
    else launch_core(k, a, cfg, st);
    return;
  }
  int64_t kchunk = (s.K + splits - 1) / splits;
  kchunk = (kchunk + tk - 1) / tk * tk;
  const int64_t nsp = (s.K + kchunk - 1) / kchunk;
  const int64_t outer = s.batch * s.M * s.N;
  BBTN_REQUIRE(partial.ptr != nullptr && partial.pstride >= nsp * outer,
               "split-K partial buffer too small");
  a.C = partial.ptr; a.pC = partial.pstride;
  a.sCb = s.M * s.N; a.sCsplit = outer;
  a.splits = nsp; a.kchunk = kchunk;
  launch_core(k, a, cfg, st, false);
  BBTN_REQUIRE(s.sCb == s.M * s.N, "split-K output must be contiguous");
  launch_reduce(k, mod, outer, nsp, outer, 1, partial, C, st);
}

void launch_tgemm_values16(const GemmShape& s, DevTensor A, DevTensor B, DevTensor C,
                           int splits, DevTensor partial, hipStream_t st) {
  BBTN_REQUIRE(s.M >= 1 && s.N >= 1 && s.K >= 1 && s.batch >= 1, "empty tgemm");
  GemmArgs a{};
  a.A = A.ptr; a.B = B.ptr;
  a.pA = A.pstride; a.pB = B.pstride;
  a.M = s.M; a.N = s.N; a.K = s.K; a.batch = s.batch;
  a.sAb = s.sAb; a.sBb = s.sBb;
  a.mod = make_moduli(0, nullptr);
  constexpr int tk = V16_TK;
  int64_t nsp = 1, kchunk = s.K;
  if (splits > 1 && s.K > tk) {
    kchunk = (s.K + splits - 1) / splits;
    kchunk = (kchunk + tk - 1) / tk * tk;
    nsp = (s.K + kchunk - 1) / kchunk;
  }
  const int64_t outer = s.batch * s.M * s.N;
  if (nsp > 1) {
    BBTN_REQUIRE(partial.ptr != nullptr && partial.pstride >= nsp * outer,
                 "split-K partial buffer too small");
    BBTN_REQUIRE(s.sCb == s.M * s.N, "split-K output must be contiguous");
    a.C = partial.ptr; a.pC = partial.pstride; a.sCb = s.M * s.N; a.sCsplit = outer;
  } else {
    a.C = C.ptr; a.pC = C.pstride; a.sCb = s.sCb; a.sCsplit = 0;
  }
  a.splits = nsp; a.kchunk = kchunk;
  const bool small = a.M < V16_TM || a.N < V16_TN;
  const int tm = small ? V16S_TM : V16_TM, tn = small ? V16S_TN : V16_TN;
  a.tiles_m = (a.M + tm - 1) / tm;
  a.tiles_n = (a.N + tn - 1) / tn;
  a.total = a.tiles_m * a.tiles_n * a.splits * a.batch;
  auto al16 = [](const void* p) { return ((uintptr_t)p & 15u) == 0; };
  a.vec_a = a.K % 4 == 0 && a.kchunk % 4 == 0 && al16(a.A) && (a.batch == 1 || a.sAb % 4 == 0);
  a.vec_b = a.N % 4 == 0 && al16(a.B) && (a.batch == 1 || a.sBb % 4 == 0);
  const int64_t cap = 1ll << 20;
  dim3 grid((unsigned)(a.total <= cap ? a.total : cap));
  if (small)
    launch_kernel((tgemm_v16_kernel<V16S_TM, V16S_TN, V16S_RM, V16S_RN, V16_TK>), grid,
                  dim3((V16S_TM / V16S_RM) * (V16S_TN / V16S_RN)), 0, st, nsp <= 1, a);
  else
    launch_kernel((tgemm_v16_kernel<V16_TM, V16_TN, V16_RM, V16_RN, V16_TK>), grid,
                  dim3((V16_TM / V16_RM) * (V16_TN / V16_RN)), 0, st, nsp <= 1, a);
  BBTN_LAUNCHED("tgemm (packed 16-bit values, grid " + std::to_string(a.total) + ")");
  if (nsp > 1) launch_reduce(0, a.mod, outer, nsp, outer, 1, partial, C, st);
}

void launch_tgemm_values16_fused(const GemmShape& s, const FusedOp* fa, DevTensor A,
                                 const FusedOp* fb, DevTensor B, DevTensor C, hipStream_t st) {
  BBTN_REQUIRE(s.M >= 1 && s.N >= 1 && s.K >= 1 && s.batch >= 1, "empty tgemm");
  BBTN_REQUIRE(fa || fb, "fused product without a fused operand");
  for (int64_t x : {s.M, s.N, s.K})
    BBTN_REQUIRE((x & (x - 1)) == 0, "fused product needs power-of-two sizes");
  GemmArgs a{};
  a.A = A.ptr; a.B = B.ptr;
  a.pA = A.pstride; a.pB = B.pstride;
  a.M = s.M; a.N = s.N; a.K = s.K; a.batch = s.batch;
  a.sAb = s.sAb; a.sBb = s.sBb;
  a.mod = make_moduli(0, nullptr);
  a.C = C.ptr; a.pC = C.pstride; a.sCb = s.sCb; a.sCsplit = 0;
  a.splits = 1; a.kchunk = s.K;
  const bool small = a.M < V16_TM || a.N < V16_TN;
  const int tm = small ? V16S_TM : V16_TM, tn = small ? V16S_TN : V16_TN;
  a.tiles_m = (a.M + tm - 1) / tm;
  a.tiles_n = (a.N + tn - 1) / tn;
  a.total = a.tiles_m * a.tiles_n * a.batch;
  auto al16 = [](const void* p) { return ((uintptr_t)p & 15u) == 0; };
  a.vec_a = !fa && a.K % 4 == 0 && al16(a.A) && (a.batch == 1 || a.sAb % 4 == 0);
  a.vec_b = !fb && a.N % 4 == 0 && al16(a.B) && (a.batch == 1 || a.sBb % 4 == 0);
  const FusedOp none{};
  const FusedOp& ra = fa ? *fa : none;
  const FusedOp& rbo = fb ? *fb : none;
  const int64_t cap = 1ll << 20;
  dim3 grid((unsigned)(a.total <= cap ? a.total : cap));
#define BBTN_FV(TM_, TN_, RM_, RN_, FA_, FB_)                                                 \
  launch_kernel((tgemm_v16_fused_kernel<TM_, TN_, RM_, RN_, V16_TK, FA_, FB_>), grid,        \
                dim3((TM_ / RM_) * (TN_ / RN_)), 0, st, true, a, ra, rbo)
  if (small) {
    if (fa && fb) BBTN_FV(V16S_TM, V16S_TN, V16S_RM, V16S_RN, true, true);
    else if (fa) BBTN_FV(V16S_TM, V16S_TN, V16S_RM, V16S_RN, true, false);
    else BBTN_FV(V16S_TM, V16S_TN, V16S_RM, V16S_RN, false, true);
  } else {
    if (fa && fb) BBTN_FV(V16_TM, V16_TN, V16_RM, V16_RN, true, true);
    else if (fa) BBTN_FV(V16_TM, V16_TN, V16_RM, V16_RN, true, false);
    else BBTN_FV(V16_TM, V16_TN, V16_RM, V16_RN, false, true);
  }
#undef BBTN_FV
  BBTN_LAUNCHED("tgemm (packed 16-bit values, permuted operands, grid " +
                std::to_string(a.total) + ")");
}

void launch_tgemm_values(const GemmShape& s, const int32_t* A, const int32_t* B,
                         int32_t* C, hipStream_t st) {
  GemmArgs a{};
  a.A = (const uint32_t*)A; a.B = (const uint32_t*)B; a.C = (uint32_t*)C;
  a.M = s.M; a.N = s.N; a.K = s.K; a.batch = s.batch;
  a.sAb = s.sAb; a.sBb = s.sBb; a.sCb = s.sCb;
  a.splits = 1; a.kchunk = s.K;
  a.mod = make_moduli(0, nullptr);
  int cfg = (s.M >= 32 && s.N >= 32) ? 0 : (s.M == 1 ? 5 : (s.N == 1 ? 6 : 2));
  launch_core(0, a, cfg, st);
}

// ---------------------------------------------------- allocation-free product
// Split-K partial results of bbtn_tgemm_noalloc live in this file-scope device
// array (kNoAllocScratchWords 32-bit words, 64 MiB), which every device the
// library runs on holds until the process ends.  In host code the name below
// is only a stand-in for the device copy: host code takes the address that
// hipGetSymbolAddress returns for the current device and never passes the
// name itself to a kernel or a copy.
static __device__ __align__(256) uint32_t scratch[kNoAllocScratchWords];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};
}  // namespace

void noalloc_scratch_init(int device) {
  BBTN_REQUIRE(device >= 0 && device < kMaxScratchDevices, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return;
  int cur = -1;
  BBTN_HIP(hipGetDevice(&cur));
  BBTN_REQUIRE(cur == device, "scratch set-up needs its device to be current");
  void* p = nullptr;
  BBTN_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  BBTN_REQUIRE(p != nullptr, "no device address for the scratch array");
  g_scratch_ptr[device] = p;
}

uint32_t* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return (uint32_t*)g_scratch_ptr[device];
}

int64_t tgemm_partial_entries(int cfg, int splits, int64_t K, int64_t outer) {
  BBTN_REQUIRE(cfg >= 0 && cfg < N_TILE_CFGS, "tile config out of range");
  const int tk = kTileCfgs[cfg].tk;
  if (splits <= 1 || K <= tk) return 0;
  int64_t kchunk = (K + splits - 1) / splits;
  kchunk = (kchunk + tk - 1) / tk * tk;
  return (K + kchunk - 1) / kchunk * outer;
}

}  // namespace bbtn
