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

// Contract the selected branches of several groups in one launch.
// assign[gi] holds count[gi] * |S_gi| states; results go to out[gi][i]
// (value plane and k residue planes, host arrays filled on return).
struct PersistJob {
  const GroupPlan* plan;
  const uint8_t* assign;  // L * |S| states
  int64_t L;
  std::vector<uint32_t>* out;  // (1 + k) * L words on return
};
void run_persistent(bbtn_ctx* ctx, const Network& net, const std::vector<PersistJob>& jobs,
                    const BaseDev& bd, const Moduli& mod, hipStream_t st);

}  // namespace bbtn
