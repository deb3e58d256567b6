// Learned branching scorer (placeholder until the MLP lands).
#pragma once
#include "search.h"
#include "ctx.h"

namespace bbtn {
void load_scorer(bbtn_ctx* ctx, const char* path);
VarScorer make_var_scorer(bbtn_ctx* ctx, const Network& net, const Tree& tree, int log2_target);
void load_tune_cache(bbtn_ctx* ctx, const char* path);
}  // namespace bbtn
