#include "scorer.h"

namespace bbtn {
void load_scorer(bbtn_ctx*, const char*) {}
VarScorer make_var_scorer(bbtn_ctx*, const Network&, const Tree&, int) { return VarScorer(); }
void load_tune_cache(bbtn_ctx*, const char*) {}
}  // namespace bbtn
