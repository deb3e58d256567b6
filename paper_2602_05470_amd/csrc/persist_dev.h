// Device-side layout of the persistent executor's step programs.
#pragma once
#include "kernels.h"

namespace bbtn {

// largest operand rank of a staged operand (bytes of the bit-position table)
constexpr int P_MAX_RANK = 16;

struct PFix {
  int32_t pos;  // bit position in the base tensor
  int32_t idx;  // index of the variable in the group's fixed-variable list
};

// The fixed bits of one base operand of a program: the OR of its fixes,
// evaluated once per task (slot j of the task's table).
struct PSlot {
  int32_t fix_off, n_fix;
};

// where an operand is read from / an output is written to
enum PKind { PK_SCRATCH = 0, PK_BASE = 1, PK_SHARED = 2, PK_LDS = 3 };

// Offsets of base and shared operands are relative to the task's base_off
// and shared_off, so that instances with the same contraction tree share one
// copy of the program.
struct POperand {
  int32_t kind;      // PKind: workgroup scratch, base tensors, shared region
                     // or the workgroup's LDS arena (src_off = entry offset there)
  int32_t rank;      // rank of the operand in the step's layout
  int64_t src_off;
  int32_t stride;    // PK_SHARED: plane stride in entries (0: the region's)
  int32_t slot;      // fixed-bit slot of a base operand, -1 if none
  int64_t mat_off;   // >= 0: also write the staged operand to scratch here
  // byte j of the table: the source bit of bit j of the step's layout
  // (j < rank; zero beyond)
  uint32_t bitpos[P_MAX_RANK / 4];
};

struct PStep {
  int32_t rb, rm, rn, rk;
  int64_t c_off;     // entry offset of the output (scratch or shared region)
  int32_t c_kind;    // PK_SCRATCH, PK_SHARED or PK_LDS
  int32_t c_stride;  // PK_SHARED: plane stride of the output (0: the region's)
  POperand a, b;
};

// A run of consecutive tasks of one program (steps [step_off,
// step_off + n_steps)): task first + i reads its fixed states at
// assign_off + i * assign_stride and, in a branch run (out_idx >= 0), writes
// root (.) folded constant to out[out_idx + i]; a shared-subtree run
// (out_idx < 0) only fills the shared region.
struct PTask {
  int32_t step_off, n_steps;
  int32_t slot_off, n_slots;  // fixed-bit slots of the program
  int64_t first;          // global index of the run's first task
  int64_t assign_off;     // byte offset of the first task's fixed states
  int64_t assign_stride;  // bytes of fixed states per task
  int64_t out_idx;        // output slot of the first task, or -1
  int64_t root_off;       // entry offset of the root scalar, -1 if none
  int32_t root_kind;      // PK_SCRATCH or PK_LDS: where the root scalar is
  int32_t pad;
  int64_t base_off;       // entry offset of the instance's base tensors
  int64_t shared_off;     // entry offset of the instance's shared region
};

struct PersistArgs {
  const PStep* steps;
  const PFix* fixes;
  const PSlot* slots;
  int32_t max_slots;  // words of the per-task fixed-bit table in LDS
  int32_t pad0;
  const PTask* tasks;  // runs, ascending by first
  int64_t n_runs;
  int64_t n_tasks;     // tasks over all runs
  const uint8_t* assign;
  const uint32_t* base;
  int64_t base_total;
  const uint32_t* lconst;  // (1 + k) planes of n_out entries
  uint32_t* out;           // (1 + k) planes of n_out entries
  int64_t n_out;
  uint32_t* scratch;       // per workgroup: (1 + k) planes of scratch_entries
  int64_t scratch_entries;
  uint32_t* shared;        // (1 + k) planes of shared_entries
  int64_t shared_entries;
  int64_t lds_entries;     // entries per operand staging buffer
  int64_t arena_entries;   // entries per plane of the LDS arena
  int32_t per_task_scratch;   // scratch of task i at i * (1 + k) * scratch_entries
  int32_t pad;
  unsigned long long* queue;  // task counter, zeroed before the launch
  Moduli mod;
};

// workgroup sizes: 64 (one wavefront), 256 or 1024 threads
size_t persist_lds_bytes(int k, int64_t lds_entries, int64_t arena_entries, int threads,
                         int slots);
void launch_persist(int k, const PersistArgs& a, int n_blocks, int threads, hipStream_t st);

}  // namespace bbtn
