// Persistent work-queue executor: every branch sub-network whose operands
// fit in LDS is contracted by one workgroup; all such branches, of every
// group, go through one launch whose workgroups pop branches from a device
// queue.
#pragma once
#include "exec.h"
#include "persist_dev.h"

namespace bbtn {

// Largest operand rank the persistent executor takes for k residues.
int persist_max_rank(int k);
bool persist_fits(const GroupPlan& g, int k);

// Contract the selected branches of several groups, possibly of several
// networks, in one launch.  assign holds L * |S| states; results go to out
// (value plane and k residue planes, host arrays filled on return).  The
// job's base tensors sit at base_off[t] (entries) in the base buffer passed
// to run_persistent.
struct PersistJob {
  const GroupPlan* plan;
  const Network* net;
  const int64_t* base_off;
  const uint8_t* assign;  // L * |S| states
  int64_t L;
  std::vector<uint32_t>* out;  // (1 + k) * L words on return
};
// per_task_scratch: task i (jobs in order, branches in order) keeps its
// scratch at i * (1 + k) * scratch_entries words of the workspace, where
// configuration recovery reads it; *scratch_entries receives the size.
void run_persistent(bbtn_ctx* ctx, const std::vector<PersistJob>& jobs, const BaseDev& bd,
                    const Moduli& mod, hipStream_t st, bool per_task_scratch = false,
                    int64_t* scratch_entries = nullptr);

// The small steps of a program run step by step: steps that run once per
// pass (shared steps, or every step when the program runs for one branch),
// read no per-branch fixed bits, and whose operands and output fit the
// executor's LDS staging, with every intermediate operand produced by another
// such step.  They form a forest; each maximal subtree is one task of one
// persistent launch (one workgroup, its steps in order, intermediates in the
// workgroup's scratch), and each subtree root is written to a root region of
// its own, where the remaining steps read it.  One launch then replaces two
// to three launches per small step.
struct SmallForest {
  std::vector<char> in;           // per step of the program: runs in the forest
  std::vector<int64_t> root_off;  // per buffer: entry offset in the root region, or -1
  int64_t root_entries = 0;       // entries of the root region
  int64_t scratch_entries = 0;    // entries per workgroup scratch plane
  int32_t max_rank = 0;           // largest operand rank (LDS staging)
  int32_t threads = 256;          // workgroup size of the launch
  std::vector<PStep> steps;       // the tasks' steps, task after task
  std::vector<PTask> tasks;       // largest first
  double ops = 0, bytes = 0;      // semiring operations and operand bytes
  // A program that keeps every intermediate (configuration recovery: one
  // branch, values only) runs its forest in place: every output and every
  // staged operand is written to its own buffer of the program's
  // workspace, where the traceback reads it (no root region, no scratch).
  bool in_place = false;
};
// base_off: entry offset of every base tensor in the base buffer; L: branches
// the program runs for.
SmallForest plan_small_forest(const GroupPlan& g, const std::vector<int64_t>& base_off, int k,
                              int64_t L);
// Bytes of device memory the forest needs (root region, scratch, program).
size_t small_forest_bytes(const SmallForest& f, int k);
// Host image of the forest's program, to be copied to dev + small_forest_prog_off(f, k).
size_t small_forest_prog_off(const SmallForest& f, int k);
std::vector<uint8_t> small_forest_image(const SmallForest& f);
// Launch the forest (program already copied to the device buffer at dev);
// base tensors as in BaseDev; `workspace`: the program's workspace, for a
// forest run in place.
void launch_small_forest(const SmallForest& f, int k, const Moduli& mod, const BaseDev& bd,
                         uint8_t* dev, hipStream_t st, uint32_t* workspace = nullptr);

}  // namespace bbtn
