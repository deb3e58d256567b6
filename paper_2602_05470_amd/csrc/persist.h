// Persistent work-queue executor: every branch sub-network whose operands
// fit in LDS is contracted by one workgroup; all such branches, of every
// group, go through one launch whose workgroups pop branches from a device
// queue.
#pragma once
#include "exec.h"

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

}  // namespace bbtn
