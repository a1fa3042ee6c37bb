// mhd_opt32.hip -- the mixed path's kernels of the slope kinds other than
// the default, built like mhd_fp32.hip (FMA contraction allowed).
#include "mhd_step.hpp"

int mhd_enqueue_opt32(const mhd::StepCtx& sc) { return mhd::enqueue_step_options<float>(sc); }
