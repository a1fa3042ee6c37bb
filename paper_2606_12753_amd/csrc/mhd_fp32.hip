// mhd_fp32.hip -- instantiation of the mixed path's kernels (FP32
// reconstruction, Riemann solver, face fluxes and EMFs; FP64 state,
// residual and RK accumulation).  Built in its own translation unit with
// FMA contraction allowed: the mixed path is checked against the FP64 oracle
// by tolerance, not bit for bit, so fused multiply-adds are free to shorten
// its instruction stream.
#include "mhd_step.hpp"

int mhd_enqueue_fp32(const mhd::StepCtx& sc) { return mhd::enqueue_step_sl<float, 0>(sc); }
