#pragma once
#include "common.h"

namespace bbtn {

// One step of the configuration traceback (device layout).
struct TraceStep {
  int32_t rb, rm, rn, rk;
  int64_t a_off, b_off;  // word offsets of the step's operands (values only)
  int32_t var_off;       // offset of [A layout vars][B layout vars] in `vars`
  int32_t pad;
};
static_assert(sizeof(TraceStep) % 8 == 0, "TraceStep is copied as whole words");

// vars holds n_var_words entries (every step's variable lists).
void launch_trace(const TraceStep* steps, int32_t n_steps, const int32_t* vars,
                  int32_t n_var_words, const int32_t* ws, int8_t* assign, int32_t n_vars,
                  int32_t* status, hipStream_t st);

}  // namespace bbtn
