// mhd_step.hpp -- the launch sequence of one Runge-Kutta step.
//
// Every stage (two, or three for SSP-RK3) runs: the x sweep (stage 1 also
// reduces the CFL rate of the start-of-step state, and the per-box dt
// follows), the y and z marches (the z march applies the RK stage combine
// to the cells; with one cell along z in every box the y march does, and
// no z march runs), the corner-EMF kernel and the face update (RK stage
// combine of the faces).
// Included by the two translation units that instantiate the kernels: the
// FP64 one (no FMA contraction, results reproducible bit for bit) and the
// FP32 one of the mixed path (contraction allowed).
#pragma once

#include "../../include/mhd.h"
#include "mhd_kernels.hpp"

namespace mhd {

// launches of one step: five per stage, plus the time step after stage 1
constexpr int kLaunchesPerStep = 3 * 5 + 1;

struct StepCtx {
  Launch L;            // boxes, tile table, box count
  const int* total;    // tiles per kernel kind over all boxes
  const int* grid;     // persistent grid size per kind (0: one group per tile)
  int var_x, var_m;    // launch variants of the x sweep and the marches; var_x
                       // = 0 or 2: the x faces are computed by the y march
                       // (k_sweep_march_xy), no x sweep runs and var_m
                       // chooses the z march's variant only
  int rk;              // Runge-Kutta stages: 2 or 3
  int rs;              // Riemann solver: 0 HLLD (HLL fallback), 1 HLL
  int sl;              // slope kind: reconstruction (0 primitive, 1
                       // characteristic variables) + 2 * limiter (0 minmod,
                       // 1 monotonised central, 2 van Leer)
  int fz;              // every box has one cell along z and more along y:
                       // the y march completes each stage, no z march
  int xcd;             // XCD-grouped tile order, bit k for kernel kind k
                       // (kXS .. kCTF)
  int uct;             // corner EMFs by the upwind CT (k_ct_uct)
  int emf;             // corner average of k_ct_edge (0 contact-upwinded,
                       // 1 E0, 2 arithmetic)
  hipStream_t stream;
  hipEvent_t* ev;      // timing: an event pair per launch, or null
  int* ev_kind;        // timing: kernel kind of each pair
};

template <typename real, int RS, int SL>
inline void launch_x(int wpe, dim3 g, hipStream_t st, const Launch& L) {
  if constexpr (SL != 0) {
    // other slope kinds: one variant (unconstrained registers)
    hipLaunchKernelGGL((k_sweep_x<real, 1, RS, SL>), g, dim3(kTPB), 0, st, L);
    return;
  }
  switch (wpe) {
    case 3: hipLaunchKernelGGL((k_sweep_x<real, 3, RS, 0>), g, dim3(kTPB), 0, st, L); break;
    case 4: hipLaunchKernelGGL((k_sweep_x<real, 4, RS, 0>), g, dim3(kTPB), 0, st, L); break;
    default: hipLaunchKernelGGL((k_sweep_x<real, 1, RS, 0>), g, dim3(kTPB), 0, st, L); break;
  }
}

// march variants: 1 = unconstrained registers, update inputs prefetched;
// 2 = unconstrained, no prefetch; 3, 4 = at least 3 / 4 waves per SIMD, no
// prefetch; 5, 6, 7 = window in LDS with (5) no register constraint and
// prefetch, (6) no constraint and no prefetch, (7) at least 3 waves per
// SIMD and no prefetch; 8, 9, 10 = variants 2, 6, 7 with the z march's
// swept state kept in an LDS ring for the RK combine (the y march has no
// combine and runs 2, 6, 7)
template <typename real, int D, int RS, int FZ, int SL>
inline void launch_march(int var, dim3 g, hipStream_t st, const Launch& L) {
  if constexpr (SL != 0) {
    // other slope kinds: one variant (register window, no prefetch)
    hipLaunchKernelGGL((k_sweep_march<real, D, 1, 0, 0, 0, RS, FZ, SL>), g, dim3(kTPB), 0, st, L);
    return;
  }
  if (D == 1 && var >= 8) var = var == 8 ? 2 : var == 9 ? 6 : 7;
  switch (var) {
    case 2: hipLaunchKernelGGL((k_sweep_march<real, D, 1, 0, 0, 0, RS, FZ, 0>), g, dim3(kTPB), 0, st, L); break;
    case 3: hipLaunchKernelGGL((k_sweep_march<real, D, 3, 0, 0, 0, RS, FZ, 0>), g, dim3(kTPB), 0, st, L); break;
    case 4: hipLaunchKernelGGL((k_sweep_march<real, D, 4, 0, 0, 0, RS, FZ, 0>), g, dim3(kTPB), 0, st, L); break;
    case 5: hipLaunchKernelGGL((k_sweep_march<real, D, 1, 1, 1, 0, RS, FZ, 0>), g, dim3(kTPB), 0, st, L); break;
    case 6: hipLaunchKernelGGL((k_sweep_march<real, D, 1, 0, 1, 0, RS, FZ, 0>), g, dim3(kTPB), 0, st, L); break;
    case 7: hipLaunchKernelGGL((k_sweep_march<real, D, 3, 0, 1, 0, RS, FZ, 0>), g, dim3(kTPB), 0, st, L); break;
    case 8:
      if constexpr (D == 2)
        hipLaunchKernelGGL((k_sweep_march<real, D, 1, 0, 0, 1, RS, FZ, 0>), g, dim3(kTPB), 0, st, L);
      break;
    case 9:
      if constexpr (D == 2)
        hipLaunchKernelGGL((k_sweep_march<real, D, 1, 0, 1, 1, RS, FZ, 0>), g, dim3(kTPB), 0, st, L);
      break;
    case 10:
      if constexpr (D == 2)
        hipLaunchKernelGGL((k_sweep_march<real, D, 3, 0, 1, 1, RS, FZ, 0>), g, dim3(kTPB), 0, st, L);
      break;
    default: hipLaunchKernelGGL((k_sweep_march<real, D, 1, 1, 0, 0, RS, FZ, 0>), g, dim3(kTPB), 0, st, L); break;
  }
}

// the y march with the x faces: x variant 0 keeps its window in registers
// and runs workgroups of 2 * kTPB lanes (kYXW columns per tile); x variant 2
// (mixed path only: the FP64 kernel's three-row ring leaves no LDS for it)
// keeps it in LDS with kTPB lanes.  The march variant then applies to the z
// march alone.
template <typename real, int RS>
inline void launch_march_xy(int var_x, dim3 g, hipStream_t st, const Launch& L) {
  if constexpr (sizeof(real) == 4) {
    if (var_x == 2) {
      hipLaunchKernelGGL((k_sweep_march_xy<real, 1, RS, kTPB>), g, dim3(kTPB), 0, st, L);
      return;
    }
  }
  hipLaunchKernelGGL((k_sweep_march_xy<real, 0, RS, kYXW>), g, dim3(kYXW), 0, st, L);
}

// Enqueues one step on sc.stream with slope kind SL (reconstruction
// SL & 1, limiter SL >> 1); returns the number of timed launches.
template <typename real, int SL>
inline int enqueue_step_sl(const StepCtx& sc) {
  Launch L = sc.L;
  L.xcd = 0;
  auto grid = [&](int kind) {
    int g = (sc.xcd >> kind) & 1 ? ((sc.total[kind] + 7) >> 3) << 3 : sc.total[kind];
    if (sc.grid[kind] > 0 && sc.grid[kind] < g) g = sc.grid[kind];
    return g < 1 ? 1 : g;
  };
  int slot = 0;
  auto mark = [&](int kind, bool before) {
    if (!sc.ev) return;
    if (before) {
      sc.ev_kind[slot] = kind;
      (void)hipEventRecord(sc.ev[2 * slot], sc.stream);
    } else {
      (void)hipEventRecord(sc.ev[2 * slot + 1], sc.stream);
      slot++;
    }
  };
  // per stage: the state swept, the state written and the combine kind
  // (SSP-RK2: 0 -> 1 first, 1 -> 0 half; SSP-RK3: 0 -> 1 first, 1 -> 2
  // three quarters / one quarter, 2 -> 0 one third / two thirds)
  static const int kSrc[2][3] = {{0, 1, 0}, {0, 1, 2}};
  static const int kDst[2][3] = {{1, 0, 0}, {1, 2, 0}};
  static const int kComb[2][3] = {{0, 1, 0}, {0, 2, 3}};
  const int r = sc.rk == 3 ? 1 : 0;
  for (int s = 0; s < (r ? 3 : 2); s++) {
    L.stage = kSrc[r][s];
    L.dst = kDst[r][s];
    L.comb = kComb[r][s];
    const bool fused = SL == 0 && (sc.var_x == 0 || sc.var_x == 2);
    if (fused) {
      // the y march computes the x faces and, in the first stage, the CFL
      // rate of its cells; the time step follows it
      L.lam = s == 0;
      L.ntiles = sc.total[kYS];
      L.xcd = (sc.xcd >> kYS) & 1;
      mark(MHD_K_SWEEP_Y, true);
      if (sc.rs)
        launch_march_xy<real, 1>(sc.var_x, dim3(grid(kYS)), sc.stream, L);
      else
        launch_march_xy<real, 0>(sc.var_x, dim3(grid(kYS)), sc.stream, L);
      mark(MHD_K_SWEEP_Y, false);
      L.lam = 0;
      if (s == 0) {
        mark(MHD_K_DT, true);
        hipLaunchKernelGGL(k_dt, dim3(L.nboxes), dim3(kTPB), 0, sc.stream, L.boxes, 0, (int)kYS);
        mark(MHD_K_DT, false);
      }
    } else {
      L.lam = s == 0;
      L.ntiles = sc.total[kXS];
      L.xcd = (sc.xcd >> kXS) & 1;
      mark(MHD_K_SWEEP_X, true);
      if (sc.rs)
        launch_x<real, 1, SL>(sc.var_x, dim3(grid(kXS)), sc.stream, L);
      else
        launch_x<real, 0, SL>(sc.var_x, dim3(grid(kXS)), sc.stream, L);
      mark(MHD_K_SWEEP_X, false);
      L.lam = 0;
      if (s == 0) {
        mark(MHD_K_DT, true);
        hipLaunchKernelGGL(k_dt, dim3(L.nboxes), dim3(kTPB), 0, sc.stream, L.boxes, 0, (int)kXS);
        mark(MHD_K_DT, false);
      }
      L.ntiles = sc.total[kYS];
      L.xcd = (sc.xcd >> kYS) & 1;
      mark(MHD_K_SWEEP_Y, true);
      if (sc.fz) {
        if (sc.rs)
          launch_march<real, 1, 1, 1, SL>(sc.var_m, dim3(grid(kYS)), sc.stream, L);
        else
          launch_march<real, 1, 0, 1, SL>(sc.var_m, dim3(grid(kYS)), sc.stream, L);
      } else {
        if (sc.rs)
          launch_march<real, 1, 1, 0, SL>(sc.var_m, dim3(grid(kYS)), sc.stream, L);
        else
          launch_march<real, 1, 0, 0, SL>(sc.var_m, dim3(grid(kYS)), sc.stream, L);
      }
      mark(MHD_K_SWEEP_Y, false);
    }
    if (!sc.fz) {
      L.ntiles = sc.total[kZS];
      L.xcd = (sc.xcd >> kZS) & 1;
      mark(MHD_K_SWEEP_Z, true);
      if (sc.rs)
        launch_march<real, 2, 1, 0, SL>(sc.var_m, dim3(grid(kZS)), sc.stream, L);
      else
        launch_march<real, 2, 0, 0, SL>(sc.var_m, dim3(grid(kZS)), sc.stream, L);
      mark(MHD_K_SWEEP_Z, false);
    }
    L.ntiles = sc.total[kCTE];
    L.xcd = (sc.xcd >> kCTE) & 1;
    mark(MHD_K_CT_EDGE, true);
    if (sc.uct)
      hipLaunchKernelGGL(k_ct_uct<real>, dim3(grid(kCTE)), dim3(kTPB), 0, sc.stream, L);
    else if (sc.emf == 1)
      hipLaunchKernelGGL((k_ct_edge<real, 1>), dim3(grid(kCTE)), dim3(kTPB), 0, sc.stream, L);
    else if (sc.emf == 2)
      hipLaunchKernelGGL((k_ct_edge<real, 2>), dim3(grid(kCTE)), dim3(kTPB), 0, sc.stream, L);
    else
      hipLaunchKernelGGL((k_ct_edge<real, 0>), dim3(grid(kCTE)), dim3(kTPB), 0, sc.stream, L);
    mark(MHD_K_CT_EDGE, false);
    L.ntiles = sc.total[kCTF];
    L.xcd = (sc.xcd >> kCTF) & 1;
    mark(MHD_K_CT_FACE, true);
    hipLaunchKernelGGL(k_ct_face<real>, dim3(grid(kCTF)), dim3(kTPB), 0, sc.stream, L);
    mark(MHD_K_CT_FACE, false);
  }
  return slot;
}

// slope kinds other than the default (primitive variables, minmod); their
// kernels are instantiated in translation units of their own
template <typename real>
inline int enqueue_step_options(const StepCtx& sc) {
  switch (sc.sl) {
    case 1: return enqueue_step_sl<real, 1>(sc);
    case 2: return enqueue_step_sl<real, 2>(sc);
    case 3: return enqueue_step_sl<real, 3>(sc);
    case 4: return enqueue_step_sl<real, 4>(sc);
    default: return enqueue_step_sl<real, 5>(sc);
  }
}

}  // namespace mhd
