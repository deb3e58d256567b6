/*
 * bbtn.h -- C ABI of the branch-and-bound tensor network (BBTN) hot path on
 * one AMD Instinct MI355X (gfx950).
 *
 * The method (Wang, Gao, Zhang, Pan, Liu, "Branch-and-Bound Tensor Networks
 * for Exact Ground-State Characterization", arXiv:2602.05470):
 *   - the ground energy of the spin glass of Eq. 1, or the maximum weight of
 *     an independent set (MWIS paragraph of the "Tropical Tensor Networks"
 *     section), is the tropical contraction of Eq. 2;
 *   - its degeneracy is obtained by carrying a count with every entry (the
 *     counting tuple algebra of the same section);
 *   - a network too large for memory is split by fixing variables into
 *     sub-networks whose results are tropically summed ("Branch-and-Bound
 *     Tensor Network" section, Eq. 3-4 and the characteristic equation).
 *
 * Conventions shared by every entry point
 *   - All functions return bbtn_status; nothing throws across the ABI.
 *   - The caller owns every input and output buffer.  The library copies what
 *     it needs before returning and never frees caller memory.  The context
 *     owns its device workspace and frees it in bbtn_destroy.
 *   - One context per host thread; different contexts are independent.
 *   - Device encoding of an entry of the counting tropical algebra, max form:
 *     an int32 value v and k residues c_i in [0, p_i) of its count.  The
 *     tropical zero ("minus infinity", the paper's (inf, 0) tuple read in max
 *     form) is stored as v = BBTN_NEG with every residue 0.  Every other value
 *     must satisfy |v| < 2^28.  The sum keeps the larger value and adds the
 *     counts on a tie; the product adds values and multiplies counts.
 *   - Spin glasses are solved in max form on the negated energy: the device
 *     value is -H and the reported E0 is minus the maximum.
 *   - A tensor over r binary variables has 2^r entries; bit j of the flat
 *     index is the state of the tensor's j-th variable.  A "tensor buffer"
 *     with E entries and k residues is (1 + k) * E consecutive 32-bit words:
 *     the int32 value plane, then residue plane 0, ..., residue plane k-1.
 *   - Residues are taken modulo primes p with 2^31 - 2^20 < p < 2^31 (every
 *     prime the library picks, and every prime a caller passes, must lie in
 *     this range: the kernels reduce 64-bit sums with 2^32 mod p < 2^21).
 */
#ifndef BBTN_H
#define BBTN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BBTN_NEG (-(1 << 30))      /* stored tropical zero (max form)      */
#define BBTN_NEG_CUT (-(1 << 29))  /* any value <= this is the tropical zero */
#define BBTN_MAX_PRIMES 32
#define BBTN_MAX_RESIDUES 4        /* residues per pass (k) */

typedef enum {
  BBTN_OK = 0,
  BBTN_E_INVALID_ARG = -1,       /* bad size, pointer, vertex id, prime ... */
  BBTN_E_OOM = -2,               /* device or host allocation failed        */
  BBTN_E_DEVICE = -3,            /* a HIP call failed                       */
  BBTN_E_COUNT_UNCERTIFIED = -4, /* count not certified within max_primes   */
  BBTN_E_TIMEOUT = -5,           /* time_limit_s exceeded                   */
  BBTN_E_BUFFER_TOO_SMALL = -6,  /* count_capacity < count_words            */
  BBTN_E_INTERNAL = -7
} bbtn_status;

typedef struct bbtn_ctx bbtn_ctx;

/* Solver options.  Fill with bbtn_default_options, then override. */
typedef struct {
  int32_t device;            /* HIP device ordinal                              */
  int32_t residues_per_pass; /* k in [0, 4]: residues carried per entry; 0 =
                                values only (ground value and one optimal
                                configuration, no count: count_words = 0,
                                n_primes = 0, certified = 0)               */
  int32_t max_primes;        /* certification adds passes up to this many primes */
  int32_t log2_target;       /* log2 T_target of Eq. 4 (entries of the largest
                                intermediate tensor); <= 0: no branching        */
  int32_t branching;         /* 0: contract the whole network (no branching);
                                1: plain planner; 2: learned scorer orders the
                                branching region (falls back to 1 without
                                weights)                                        */
  int32_t batched;           /* 0: per-branch step-by-step launches;
                                1: all branch sub-networks in one persistent
                                   work-queue launch where they fit; in the
                                   programs that do not fit, the small steps
                                   that run once per pass (subtrees whose
                                   operands fit LDS) go through one persistent
                                   launch per program, the rest step by step;
                                2: as 1 without that fusion of small steps  */
  int32_t region_max;        /* largest branching region |R| (<= 16)            */
  int32_t local_search;      /* > 0: seed the incumbent of global pruning with
                                this many local-search sweeps                   */
  int32_t graphs;            /* 1: a step program that runs repeatedly (chunks,
                                one branch at a time) is captured once into a
                                hipGraph and replayed; 0: plain launches        */
  const char* scorer_weights;/* path of learned-scorer weights, or NULL         */
  const char* autotune_cache;/* path of the tile autotuner cache, or NULL       */
  double time_limit_s;       /* <= 0: none                                      */
  void* stream;              /* hipStream_t to run on, or NULL for the
                                context's own stream                           */
  int32_t host_threads;      /* host threads that plan the instances of a call
                                (network build, order, search); <= 0: one per
                                hardware thread.  Several contexts used
                                concurrently share the host's cores.          */
  int32_t order_refine;      /* 0: greedy contraction order; n > 0: also n
                                annealed refinements of it (local rotations),
                                the min-fill order and one refinement of that,
                                each scored by a branch-and-bound search of the
                                first instance of a structure; the cheapest
                                (leaf MACs plus search nodes) is cached for the
                                structure.  n <= 64.  -1: the min-fill order
                                alone (a min-fill elimination order of the
                                variables, tensors holding each eliminated
                                variable contracted pairwise).                */
  uint64_t device_mem_cap;   /* bytes of device memory the context (with its
                                configuration-recovery context) may hold;
                                branch chunks are sized to it, and a solve
                                that cannot fit fails with BBTN_E_OOM.
                                0: no cap beyond the free memory.             */
  int32_t spin_flip;         /* 1: a zero-field spin glass is solved with one
                                spin fixed to +1 and the count doubled (the
                                spin-flip symmetry H(sigma) = H(-sigma) maps
                                the ground states with that spin at +1 one to
                                one onto those with it at -1): the same ground
                                energy and degeneracy with half the leaves
                                when the fixed spin is one the search would
                                branch on (the spin of largest overflow
                                participation, else of largest share of the
                                contraction's multiply-accumulates); the
                                configuration has that spin at +1.  Ignored
                                for instances with a nonzero field and for
                                MWIS.  0: off.                                */
} bbtn_options;

/* Result of a solve.  `count` and `config` are caller-owned. */
typedef struct {
  int64_t value;       /* spin glass: E0 = min H; MWIS: max total weight       */
  int32_t n_primes;    /* primes used, and count residues modulo each          */
  uint32_t primes[BBTN_MAX_PRIMES];
  uint32_t residues[BBTN_MAX_PRIMES];
  int32_t certified;   /* 1 iff the CRT count was confirmed by an extra prime  */
  int32_t count_words; /* 32-bit words of the exact count (always set)         */
  uint32_t* count;     /* caller buffer, little-endian words, or NULL          */
  int32_t count_capacity;
  int8_t* config;      /* caller buffer [n] or NULL: one optimal configuration,
                          sigma in {-1,+1} (spin glass) or x in {0,1} (MWIS)   */
  uint64_t leaves;     /* branch sub-networks contracted                       */
  uint64_t pruned;     /* branches discarded by global pruning                 */
  uint64_t nodes;      /* search-tree nodes expanded                           */
  uint64_t macs;       /* semiring multiply-accumulates on the device          */
  double seconds[8];   /* [0] total [1] build+plan [2] search [3] contraction
                          [4] CRT+certification [5] configuration [6] H2D/D2H
                          [7] values pass (part of [3])                      */
} bbtn_result;

void bbtn_default_options(bbtn_options* opt);

/* Create a context on opt->device.  *out is set on success. */
bbtn_status bbtn_create(const bbtn_options* opt, bbtn_ctx** out);
void bbtn_destroy(bbtn_ctx* ctx);

/* Message for the last failing call on ctx (valid until the next call). */
const char* bbtn_last_error(const bbtn_ctx* ctx);

/*
 * Spin glass of Eq. 1: H(sigma) = sum_E -J_ij s_i s_j + sum_V -h_i s_i.
 * n spins, m edges; edge_uv[2m] holds vertex ids in [0, n); J[m]; h[n] or
 * NULL (zero field).  Duplicate edges are merged by adding their couplings.
 * Self-loops, ids outside [0, n), or sum|J| + sum|h| >= 2^27 give
 * BBTN_E_INVALID_ARG.  Fills value = E0, the degeneracy (count) and one
 * ground configuration.  Host pointers.
 */
bbtn_status bbtn_solve_spinglass(bbtn_ctx* ctx, int32_t n, int32_t m,
                                 const int32_t* edge_uv, const int32_t* J,
                                 const int32_t* h, bbtn_result* res);

/*
 * Maximum weight independent set (MWIS paragraph): max sum_{i in S} w_i over
 * independent sets S.  w[n] positive or NULL (unit weights).  Duplicate edges
 * are ignored.  Fills value = W*, the number of optimal sets and one of them.
 * Host pointers.
 */
bbtn_status bbtn_solve_mwis(bbtn_ctx* ctx, int32_t n, int32_t m,
                            const int32_t* edge_uv, const int32_t* w,
                            bbtn_result* res);

/* ------------------------------------------------------------------------
 * Kernel-level entry points (device pointers, caller-owned; asynchronous on
 * `stream`, a hipStream_t, where NULL is the null (default) stream).
 * primes: host array [k]; every p in (2^31 - 2^20, 2^31).
 * ---------------------------------------------------------------------- */

/*
 * Counting tropical matrix product (Eq. 2 applied to one pairwise
 * contraction):  C[b,m,n] = (+)_q A[b,m,q] (.) B[b,q,n].
 * A: tensor buffer of batch*M*K entries, row-major [batch][M][K];
 * B: batch*K*N entries, [batch][K][N];  C: batch*M*N entries, [batch][M][N].
 * k in [1, 4]; K >= 1.  C may not alias A or B.
 */
bbtn_status bbtn_tgemm(bbtn_ctx* ctx, int32_t k, const uint32_t* primes,
                       int64_t batch, int64_t M, int64_t N, int64_t K,
                       const void* A, const void* B, void* C, void* stream);

/*
 * Values-only (max-plus) product of Eq. 2:  C[b,m,n] = max_q A[b,m,q] +
 * B[b,q,n], on int32 value planes laid out as in bbtn_tgemm (no residue
 * planes).  Values <= BBTN_NEG_CUT are the tropical zero and come out as
 * BBTN_NEG.  max_abs: the caller's bound on |v| of every other value of A
 * and B (< 2^28); below 2^12 the product runs with two values per 32-bit
 * word (packed 16-bit adds and maxima), otherwise in 32 bits.  A value
 * outside the stated bound gives undefined results (never a fault).
 */
bbtn_status bbtn_tgemm_values(bbtn_ctx* ctx, int64_t batch, int64_t M, int64_t N, int64_t K,
                              const int32_t* A, const int32_t* B, int32_t* C, int32_t max_abs,
                              void* stream);

/*
 * bbtn_tgemm for callers that cannot allocate device memory (code under
 * hipGraph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same product, arguments and errors, with no device allocation, no
 * hipFree and no tile autotuning in the call (tiles come from the context's
 * cached tuning or the shape heuristic).  When the product is split along K,
 * the partial results go to a static device array of 2^24 32-bit words
 * (64 MiB) that each device the library runs on holds until the process
 * ends; the split factor is lowered until (1 + k) * splits * batch * M * N
 * words fit in it, down to an unsplit product that needs none, so no size
 * within bbtn_tgemm's limits is refused for its sake.  The array is shared by
 * every call on a device and keeps the last call's partials (each call writes
 * every partial it reads): calls on one device that overlap in time (on
 * different streams, or from different host threads) race on it and must be
 * serialised by the caller.  The context must have been created on this
 * device (bbtn_create sets the array up).
 */
bbtn_status bbtn_tgemm_noalloc(bbtn_ctx* ctx, int32_t k, const uint32_t* primes,
                               int64_t batch, int64_t M, int64_t N, int64_t K,
                               const void* A, const void* B, void* C, void* stream);

/*
 * Permutation and branch-variable fixing of a tensor (slicing,
 * T|_{s_Vf = x} of Eq. 3), batched over L outputs.
 * Input: tensor buffer of in_entries entries over r_in variables (in_entries
 * = 2^r_in when in_stride == 0, or L * 2^r_in when in_stride == 2^r_in, i.e.
 * one input per output).  Output: tensor buffer of L * 2^r_out entries.
 * Output variable j is input variable src_bits[j] (host array [r_out]).
 * Input variables not named in src_bits are fixed: their states are the bits
 * of fixed_bits[l] (device array [L] of uint64, already placed at the input
 * bit positions; NULL means all zero).
 * Output entry (l, i) = input entry (l * in_stride) + sum_j bit_j(i) <<
 * src_bits[j] | fixed_bits[l].
 */
bbtn_status bbtn_gather(bbtn_ctx* ctx, int32_t k, int32_t r_in, int32_t r_out,
                        const int32_t* src_bits, int64_t L, int64_t in_stride,
                        const uint64_t* fixed_bits, const void* in,
                        int64_t in_entries, void* out, void* stream);

/*
 * Tropical sum over segments (sum-out of variables, merge of branch
 * results): out[o] = (+)_{s < S} in[s * seg_stride + o * elem_stride] for
 * o < outer.  in: tensor buffer of in_entries entries; out: outer entries.
 */
bbtn_status bbtn_reduce(bbtn_ctx* ctx, int32_t k, const uint32_t* primes,
                        int64_t outer, int64_t S, int64_t seg_stride,
                        int64_t elem_stride, const void* in, int64_t in_entries,
                        void* out, void* stream);

/*
 * Branch bounds for global pruning: for each branch b < n_branch,
 * bound[b] = offset[b] + sum over its tensors of the largest finite value;
 * keep[b] = 1 iff every tensor has a finite entry and bound[b] >= incumbent
 * (ties are kept: they carry counts).  Tensor t of branch b is the slice
 * [tensor_off[b*T + t], tensor_off[b*T + t] + tensor_len[b*T + t]) of the
 * int32 value array `values`; T = tensors_per_branch.  All device pointers.
 * *n_keep (device int32) receives the number of kept branches and
 * keep_idx[0..n_keep) their indices in ascending order.
 */
bbtn_status bbtn_bound(bbtn_ctx* ctx, int64_t n_branch, int32_t tensors_per_branch,
                       const int32_t* values, const int64_t* tensor_off,
                       const int32_t* tensor_len, const int64_t* offset,
                       int64_t incumbent, int64_t* bound, int32_t* keep_idx,
                       int32_t* n_keep, void* stream);

/* Semiring multiply-accumulates performed by the last solve on ctx. */
uint64_t bbtn_last_macs(const bbtn_ctx* ctx);

/* ------------------------------------------------------------------------
 * Kernel timing.  When enabled, HIP events are recorded on the launch stream
 * around every launch of the kernels below, and their durations, launch
 * counts and algorithmic work are accumulated.  Enabling or disabling clears
 * the counters.  Kernel ids: 0 counting tropical product on LDS tiles
 * (bbtn_tgemm, bbtn_tgemm_values and the step-by-step executor), 1
 * persistent work-queue executor, 2 gather (permutation / slicing), 3
 * segmented reduction (not instrumented yet), 4 thin product (the same
 * products when the summed range is short and one side narrow: one thread
 * per output, no LDS).
 * ops: semiring operations, (2 + 2k) per multiply-accumulate (one value add
 * and one max, one modular multiply and one modular add per residue).
 * bytes: algorithmic bytes (operands read once + results written once).
 * ---------------------------------------------------------------------- */
typedef struct {
  uint64_t launches;
  double seconds;
  double ops;
  double bytes;
} bbtn_kernel_stats;

bbtn_status bbtn_profile(bbtn_ctx* ctx, int32_t enable);
/* As bbtn_profile, timing only the kernels whose id bit is set in mask
 * (bit i: kernel id i; 0 disables): fewer events in the launch stream when
 * only one kernel's figures are wanted. */
bbtn_status bbtn_profile_mask(bbtn_ctx* ctx, uint32_t mask);
bbtn_status bbtn_get_kernel_stats(bbtn_ctx* ctx, int32_t kernel, bbtn_kernel_stats* out);

/* ------------------------------------------------------------------------
 * Learned branching scorer.  A perceptron 32 -> 128 -> 128 -> 1 with ReLU
 * scores candidate branching variables; the planner uses the scores only to
 * order the variables it grows regions from (seeds and growth order), so the
 * branches it builds stay complete and orthogonal and results are unchanged.
 * Parameter layout: bfloat16 weights W [W1 (128 x 32, row-major) | W2 (128 x
 * 128) | w3 (128)] = 20608 values; float32 biases [b1 (128) | b2 (128) | b3].
 * Inputs X: rows x 32 bfloat16 (standardised features); all accumulation and
 * hidden activations are float32.
 * ---------------------------------------------------------------------- */

/* y[r] = w3 . relu(W2 relu(W1 x_r + b1) + b2) + b3.  h1, h2 (rows x 128
 * float32, device) receive the hidden activations when non-NULL (both or
 * neither).  Device pointers. */
bbtn_status bbtn_mlp_forward(bbtn_ctx* ctx, int64_t rows, const uint16_t* X, const uint16_t* W,
                             const float* bias, float* y, float* h1, float* h2, void* stream);

/* Gradient of the mean squared error (1/rows) sum (y - t)^2 with respect to
 * every parameter, given the forward pass's y, h1, h2.  grad (device, 20866
 * float32): [W1 | W2 | w3 | b1 | b2 | b3] followed by the sum of squared
 * errors.  Deterministic (per-block partial sums added in block order). */
bbtn_status bbtn_mlp_backward(bbtn_ctx* ctx, int64_t rows, const uint16_t* X, const uint16_t* W,
                              const float* y, const float* t, const float* h1, const float* h2,
                              float* grad, void* stream);

/* One Adam step (step >= 1, bias-corrected) on the float32 master copy
 * master[20865] = [weights | biases] with moments m, v; refreshes the
 * bfloat16 weights W and the float32 biases.  Device pointers. */
bbtn_status bbtn_mlp_adam(bbtn_ctx* ctx, float* master, uint16_t* W, float* bias, float* m,
                          float* v, const float* grad, float lr, float beta1, float beta2,
                          float eps, int32_t step, void* stream);

/* Load trained weights (file written by bbtn_scorer_train) into ctx; used
 * when branching == 2. */
bbtn_status bbtn_scorer_load(bbtn_ctx* ctx, const char* path);

/* Several independent instances of one problem in one call (ensembles of
 * seeded instances, "Applications" section).  The instances are built,
 * ordered and searched on parallel host threads; then the branch
 * sub-networks of all instances share each device launch: one persistent
 * launch for the values pass, one for the counting pass, one for
 * configuration recovery and one traceback launch.
 * kind 0: spin glass, weights[i] = J of instance i (m[i] entries), h[i] =
 * its field or NULL (h itself may be NULL: no fields); kind 1: MWIS,
 * weights[i] = w (n[i] entries) or NULL for unit weights, h unused.
 * edge_uv[i]: 2 m[i] vertex ids.  results[i] as for the single-instance
 * calls (caller-owned count and config buffers); status[i] (caller-owned,
 * n_inst entries) receives each instance's status.  Returns BBTN_OK when
 * every instance succeeded, else the first failing instance's status (the
 * others' results are still filled); a device failure fails every
 * instance. */
bbtn_status bbtn_solve_batch(bbtn_ctx* ctx, int32_t kind, int32_t n_inst, const int32_t* n,
                             const int32_t* m, const int32_t* const* edge_uv,
                             const int32_t* const* weights, const int32_t* const* h,
                             bbtn_result* results, bbtn_status* status);

/* The planner alone, on the host (ctx may be NULL; no device is used): build
 * the network of a spin-glass (kind 0: weights = J, h) or MWIS (kind 1:
 * weights = w, h unused) instance, choose its contraction order (as the
 * option order_refine does, with order_refine in [-1, 64]; 0 = greedy,
 * -1 = min-fill), take
 * the local-search incumbent (local_search sweeps; 0 = no incumbent) and run
 * the branch-and-bound search with T_target = 2^log2_target and regions of
 * at most region_max variables ("Branch-and-Bound Tensor Network" section).
 * values_only != 0 selects the values-only pruning of residues_per_pass = 0.
 * Leaf l is written to leaves[l*n .. l*n + n): -1 for a free variable, else
 * its fixed state (s, with s = 1 meaning sigma = +1; or x).  *n_leaves
 * receives the leaf count; pass leaves = NULL to query it.  *incumbent
 * receives the incumbent's value in the problem's convention (energy or
 * weight), or INT64_MIN when there is none.  Errors: BBTN_E_INVALID_ARG,
 * BBTN_E_BUFFER_TOO_SMALL (capacity < *n_leaves with leaves != NULL). */
bbtn_status bbtn_plan_leaves(bbtn_ctx* ctx, int32_t kind, int32_t n, int32_t m,
                             const int32_t* edge_uv, const int32_t* weights, const int32_t* h,
                             int32_t log2_target, int32_t region_max, int32_t local_search,
                             int32_t values_only, int32_t order_refine, int8_t* leaves,
                             int64_t capacity, int64_t* n_leaves, int64_t* incumbent);

/* Complexity of the contraction order the planner uses for an instance
 * (host only, no context; "Tropical Tensor Networks" section): the order is
 * chosen as bbtn_options.order_refine does (0: greedy; -1: min-fill;
 * n in [1, 64]: the cheapest of the greedy tree, n annealed refinements,
 * the min-fill tree and one refinement of it, each scored by a
 * branch-and-bound search with T_target = 2^log2_target and regions of at
 * most region_max variables).  Outputs: *tc_log2 = log2 of the semiring
 * multiply-accumulates of the unsliced contraction, *sc = log2 entries of
 * its largest intermediate, *rho = the overflow measure of Eq. 4, the sum
 * over intermediates of max(0, log2 size - log2_target).  Errors:
 * BBTN_E_INVALID_ARG (bad graph, kind, sizes or NULL outputs). */
bbtn_status bbtn_order_complexity(int32_t kind, int32_t n, int32_t m, const int32_t* edge_uv,
                                  const int32_t* weights, const int32_t* h, int32_t order_refine,
                                  int32_t log2_target, int32_t region_max, double* tc_log2,
                                  int32_t* sc, int64_t* rho);

/* Contraction orders chosen by measurement ("Tropical Tensor Networks"
 * section: the cost of a contraction order; Eq. 4 for the overflow that the
 * branching removes).  The probe score that bbtn_options.order_refine uses
 * models device time from multiply-accumulates and memory traffic, but the
 * time of a solve also depends on which leaves hold the optimum (only those
 * are counted), so a caller that solves many instances of one structure may
 * time a few orders and keep the fastest:
 *   bbtn_order_candidates builds, for the structure of the given instance
 *   (its simplified tensors' variable lists; couplings and weights do not
 *   matter), the candidate orders of order_refine = n = max(1, the
 *   context's order_refine): the greedy tree, the n refinements, the
 *   min-fill tree and its refinement, and n more refinements under varied
 *   annealing objectives (lighter overflow weight, memory traffic in the
 *   move score), each probed with the context's log2_target and
 *   region_max (budget 2^22 search nodes), and keeps those that finish,
 *   cheapest probe score first, in the context (once per structure; later
 *   calls return the same list).  *n_out receives their number.
 *   bbtn_order_use makes candidate `which` (0 = cheapest probe score) the
 *   structure's order for every later solve on this context.
 * Host only (ctx holds the lists; no device work).  Errors:
 * BBTN_E_INVALID_ARG (NULL ctx or output, bad graph or kind, log2_target of
 * the context <= 0, `which` out of range or no candidates built for the
 * structure). */
bbtn_status bbtn_order_candidates(bbtn_ctx* ctx, int32_t kind, int32_t n, int32_t m,
                                  const int32_t* edge_uv, const int32_t* weights,
                                  const int32_t* h, int32_t* n_out);
bbtn_status bbtn_order_use(bbtn_ctx* ctx, int32_t kind, int32_t n, int32_t m,
                           const int32_t* edge_uv, const int32_t* weights, const int32_t* h,
                           int32_t which);

/* Training data from the search itself: run the planner on an instance
 * (kind 0: spin glass with weights = J, h; kind 1: MWIS with weights = w)
 * with T_target = 2^log2_target for up to max_nodes nodes; at each node,
 * cand_per_node candidate seed variables give one row each: 32 features and
 * the label log2(gamma) of the best branching rule the planner grows from
 * that seed (the characteristic equation's branching factor, which reflects
 * both the problem-size reduction and the configurations pruned), minus the
 * smallest such label among the node's candidates (the scorer ranks the
 * candidates of one node).  Host arrays X[capacity*32], y[capacity];
 * *rows receives the row count (pass X = y = NULL to query it).  Host-only:
 * ctx may be NULL (region size 8) or a context (its region_max). */
bbtn_status bbtn_scorer_collect(bbtn_ctx* ctx, int32_t kind, int32_t n, int32_t m,
                                const int32_t* edge_uv, const int32_t* weights, const int32_t* h,
                                int32_t log2_target, int32_t max_nodes, int32_t cand_per_node,
                                float* X, float* y, int64_t capacity, int64_t* rows);

/* Train the scorer on the GPU with the kernels above (minibatches of `batch`
 * rows, Adam at learning rate lr, `epochs` passes, initialisation from seed).
 * Features and labels are standardised; loss_out[epochs] (host, or NULL)
 * receives the standardised mean squared error after every epoch.  The
 * weights are written to save_path (or not, if NULL) and loaded into ctx. */
bbtn_status bbtn_scorer_train(bbtn_ctx* ctx, const float* X, const float* y, int64_t rows,
                              int32_t epochs, int32_t batch, float lr, uint64_t seed,
                              float* loss_out, const char* save_path);

#ifdef __cplusplus
}
#endif
#endif /* BBTN_H */
