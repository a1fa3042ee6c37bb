// mhd_opt64.hip -- FP64 kernels of the slope kinds other than the default
// (characteristic reconstruction; monotonised central and van Leer
// limiters), in a translation unit of their own so that the library builds
// in parallel.  No FMA contraction: FP64 results are reproducible bit for
// bit, as in the default kernels.
#include "mhd_step.hpp"

int mhd_enqueue_opt64(const mhd::StepCtx& sc) { return mhd::enqueue_step_options<double>(sc); }
