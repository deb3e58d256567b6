// Running step programs on the device.
#pragma once
#include <vector>
#include "ctx.h"
#include "kernels.h"
#include "plan.h"

namespace bbtn {

// Base tensors of a network uploaded with the residues of `k` primes
// (indices into prime_table()).
struct BaseDev {
  int k = 0;
  std::vector<int64_t> off;  // entry offset of every base tensor
  int64_t total = 0;         // entries
  DevTensor t;
};
void upload_base(bbtn_ctx* ctx, const Network& net, const int* prime_idx, int k,
                 BaseDev& bd, DevBuf& buf);
// Base tensors of several networks in one buffer: tensor t of network i at
// offs[i][t]; bd.off stays empty.
void upload_bases(bbtn_ctx* ctx, const std::vector<const Network*>& nets, const int* prime_idx,
                  int k, BaseDev& bd, std::vector<std::vector<int64_t>>& offs, DevBuf& buf);

// Time the candidate tile configurations for one shape bucket.
TuneVal autotune_shape(bbtn_ctx* ctx, int k, int64_t batch, int64_t M, int64_t N, int64_t K,
                       const TuneVal& heuristic);
void save_tune_cache(bbtn_ctx* ctx, const char* path);

// Pick a tile configuration (and split-K factor) for one product: the
// autotuner's cached choice, else (tuning when a cache path is set) a
// measured one, else a shape heuristic.
TuneVal choose_tiles(bbtn_ctx* ctx, int k, int64_t batch, int64_t M, int64_t N, int64_t K);
// The same choice without tuning: the cached measured choice, else the shape
// heuristic.  Allocates nothing on the device.
TuneVal cached_or_heuristic_tiles(const bbtn_ctx* ctx, int k, int64_t batch, int64_t M,
                                  int64_t N, int64_t K);

// Run the program `g` for L branches.  assign[l * |S| + j] is the state of
// the j-th fixed variable (ascending ids) of branch l.  Writes, for every
// branch, root (.) folded constant into `out` (tensor buffer of L entries).
// With reuse (the same program will run again with the same shapes) the
// launches are captured into a hipGraph once and replayed.  A group whose
// branches run in several chunks passes its branch count as L_group (the
// forest of small steps depends on it) and, for every chunk after the first
// of a pass, shared_ready: the shared steps (and the forest) already ran
// for the first chunk with the same workspaces, and their results are read
// again instead of being recomputed.
void run_group(bbtn_ctx* ctx, const Network& net, const GroupPlan& g, const BaseDev& bd,
               const Moduli& mod, const uint8_t* assign, int64_t L, DevTensor out,
               hipStream_t st, bool reuse = false, bool shared_ready = false,
               int64_t L_group = -1);

// Per-branch folded constants on the host: value and k residues.
void leaf_constants(const Network& net, const GroupPlan& g, const int* prime_idx, int k,
                    const uint8_t* assign, int64_t L, std::vector<uint32_t>& host);

}  // namespace bbtn
