// The solve pipeline over one or several instances: build and plan each
// instance on the host (in parallel threads), then run the values pass, the
// counting pass and configuration recovery of all instances through shared
// device launches.
#pragma once
#include <functional>
#include <string>
#include <vector>
#include "ctx.h"
#include "network.h"

namespace bbtn {

struct Instance {
  // when set, fills net and ls_x on a planning thread (errors become this
  // instance's status)
  std::function<void(Instance&)> build;
  Network net;
  std::vector<uint8_t> ls_x;     // local-search configuration (may be empty)
  bbtn_result* res = nullptr;    // caller's result
  bbtn_status status = BBTN_OK;  // outcome of this instance
  std::string err;
};

// Solve every instance.  An instance's own failure (time limit, count not
// certified, buffer too small, no feasible configuration) is recorded in its
// status; a device failure throws and ends the call for every instance.
void solve_instances(bbtn_ctx* ctx, std::vector<Instance>& insts);

// Contraction orders measured by the caller: the candidates of net's
// structure ranked by probe score (rank_orders with the context's
// order_refine, T_target and region size), computed once per structure and
// context; returns how many there are.  order_use installs candidate
// `which` as the structure's order for every later solve on the context.
int order_candidates(bbtn_ctx* ctx, const Network& net);
void order_use(bbtn_ctx* ctx, const Network& net, int which);

}  // namespace bbtn
