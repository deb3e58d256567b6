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

// One traceback: a program of n_steps steps over the values-only workspace
// ws (the step operands at a_off / b_off), the variable lists of every step
// (n_var_words entries), and the states of the n_vars variables (fixed ones
// set, the others -1 on entry; all set on return).  status receives a
// non-zero code when a step finds no finite entry or reads an unset state.
struct TraceJob {
  const TraceStep* steps;
  const int32_t* vars;
  const int32_t* ws;
  int8_t* assign;
  int32_t* status;
  int32_t n_steps, n_var_words, n_vars, pad;
};

// One workgroup (one wavefront) per job; jobs is a device array.  The
// maxima over the jobs size the launch.
void launch_trace(const TraceJob* jobs, int32_t n_jobs, int32_t max_steps, int32_t max_var_words,
                  int32_t max_vars, hipStream_t st);

}  // namespace bbtn
