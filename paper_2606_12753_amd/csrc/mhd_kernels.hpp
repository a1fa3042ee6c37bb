// mhd_kernels.hpp -- HIP kernels of the ideal-MHD update for gfx950 (CDNA4).
//
// The update is the main cycle of arXiv 2606.12753 §2.2.3: per direction,
// reconstruct primitive variables, solve a Riemann problem at each interface
// and apply the flux-conservative update; constrained transport (CT) evolves
// the face-centred magnetic field; Runge-Kutta integrates in time.  The
// component algorithms are the published ones:
//   * PLM reconstruction of (rho, v_n, v_t1, v_t2, p, B_t1, B_t2) with the
//     minmod limiter, normal field from the face;
//   * HLLD (Miyoshi & Kusano 2005) with an HLL fallback on unphysical stars;
//   * contact-upwinded CT corner EMFs (Gardiner & Stone 2005) and the face
//     update as the discrete curl;
//   * two-stage SSP Runge-Kutta (Shu & Osher 1988) and the CFL time step from
//     the fast magnetosonic rate.
//
// Layout in HBM: structure of arrays, C order [z][y][x], x fastest; every
// wavefront's lanes run along x so that all global loads and stores are
// coalesced, whatever the sweep direction:
//   * the x sweep stages a row segment of primitives in LDS (one load and one
//     primitive recovery per cell) and computes one x face per lane;
//   * the y and z sweeps march each lane along its column: a register window
//     of four cells slides along the strided axis, so the strided access
//     never reaches HBM as strided; each new cell is one coalesced row load.
// Periodic axes wrap cell indices and store n faces per axis (face n is face
// 0); outflow axes clamp cell indices (ghost = copy of the boundary cell) and
// store n+1 faces.
//
// Every kernel takes a tile table: tiles of all boxes of an ensemble are
// numbered consecutively and a workgroup finds its box by a binary search of
// the per-box tile offsets, so one launch covers uneven boxes; the grid may
// be smaller than the tile count (persistent grid-stride loop).
//
// The arithmetic type `real` is double (FP64 path) or float (mixed path:
// FP32 reconstruction, Riemann solver, face fluxes and EMFs; the state, the
// primitive recovery, the flux differences and residual, the RK
// accumulation, the face-field curl and the time step stay FP64).  In
// FP64 every operation is written in the order of the method's defining
// formulas and the library is built without FMA contraction, so that the
// result does not depend on tiling or launch shape.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mhd {

constexpr int kNQ = 5;      // hydro conserved variables
constexpr int kTPB = 256;   // threads per workgroup (4 wave64)
constexpr int kLdsCells = 320;  // x-sweep LDS capacity (cells per tile)

// Device descriptor of one box.  Work arrays are typed by the precision in
// use (double or float) and stored as void* here.
struct Box {
  int n[3];      // cells per axis
  int nf[3];     // faces along each axis normal: n (periodic) or n+1 (outflow)
  int per[3];    // periodic axis
  int act[3];    // active axis (n > 1)
  double dx[3];
  double gamma, cfl, pfloor;
  double* U[2][kNQ];  // conserved state: [0] start of step, [1] stage state
  double* B[2][3];    // face field, same two copies
  void* Ec[3];        // cell EMF  E = -v x B
  void* FX[kNQ];      // hydro flux on x faces
  void* EF[3][2];     // EMF (E_t1, E_t2) on the faces normal to each axis
  void* MF[3];        // mass flux for the CT upwinding, per face direction
  double* R[kNQ];     // cell residual (FP64 in both paths: the flux
                      // differences telescope exactly, so the update
                      // conserves to FP64 rounding)
  void* ED[3];        // corner EMF along each axis
  double* lam;        // per-tile max CFL rate
  double* scal;       // [0] dt, [1] t, [2] t_stop, [3] dt of the current state
  unsigned long long* cnt;  // [0] floor hits, [1] HLL fallbacks, [2] bad cells
  int xw, xr, xseg;   // x sweep: faces per segment, rows per tile, segments/row
  int ysl, yseg;      // y march: cells per segment, segments
  int zsl, zseg;      // z march
  int ntile[6];       // tiles per kernel kind
};

enum Kind { kXS = 0, kYS = 1, kZS = 2, kCTE = 3, kCTF = 4, kLAM = 5 };

// Per-launch arguments.
struct Launch {
  const Box* boxes;
  const int* base;  // base[kind*(nboxes+1) + b]: first tile of box b
  int nboxes;
  int ntiles;       // tiles of this kind over all boxes
  int stage;        // 0: read state 0 (stage 1); 1: read state 1 (stage 2)
};

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ int find_box(const int* base, int nb, int t) {
  int lo = 0, hi = nb - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (base[mid] <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// cell index along an axis for a (possibly ghost) position
__device__ __forceinline__ int map_cell(int i, int n, int per) {
  if (per) {
    while (i < 0) i += n;
    while (i >= n) i -= n;
    return i;
  }
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// upper face of cell i along an axis
__device__ __forceinline__ int face_up(int i, int n, int per) {
  int f = i + 1;
  return (per && f == n) ? 0 : f;
}

__device__ __forceinline__ size_t cidx(const Box& b, int i, int j, int k) {
  return ((size_t)k * b.n[1] + j) * b.n[0] + i;
}

// element of the face array normal to axis d
__device__ __forceinline__ size_t fidx(const Box& b, int d, int i, int j, int k) {
  int ex = d == 0 ? b.nf[0] : b.n[0];
  int ey = d == 1 ? b.nf[1] : b.n[1];
  return ((size_t)k * ey + j) * ex + i;
}

// element of the corner-EMF array along axis c: face extents on the two
// other axes, cell extent along c
__device__ __forceinline__ size_t eidx(const Box& b, int c, int i, int j, int k) {
  int ex = c == 0 ? b.n[0] : b.nf[0];
  int ey = c == 1 ? b.n[1] : b.nf[1];
  return ((size_t)k * ey + j) * ex + i;
}

template <typename T>
__device__ __forceinline__ T ld(const void* p, size_t i) {
  return static_cast<const T*>(p)[i];
}
template <typename T>
__device__ __forceinline__ void st(void* p, size_t i, T v) {
  static_cast<T*>(p)[i] = v;
}

// division and square root: IEEE in FP64; hardware reciprocal / square root
// (about 1 ulp) in the FP32 work of the mixed path
__device__ __forceinline__ double dv(double a, double b) { return a / b; }
__device__ __forceinline__ float dv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double sq(double a) { return __builtin_sqrt(a); }
__device__ __forceinline__ float sq(float a) { return __builtin_amdgcn_sqrtf(a); }
__device__ __forceinline__ double ab(double a) { return __builtin_fabs(a); }
__device__ __forceinline__ float ab(float a) { return __builtin_fabsf(a); }
__device__ __forceinline__ bool finite(double a) { return __builtin_isfinite(a); }
__device__ __forceinline__ bool finite(float a) { return __builtin_isfinite(a); }

// thresholds of the Riemann solver and the CT upwinding, per precision
template <typename real> struct Eps;
template <> struct Eps<double> {
  static constexpr double deg = 1e-12;   // degenerate HLLD denominator
  static constexpr double bsmall = 1e-12;  // B_n ~ 0: no double-star states
  static constexpr double mflux = 1e-12;   // mass flux zero up to rounding
};
template <> struct Eps<float> {
  static constexpr float deg = 1e-6f;
  static constexpr float bsmall = 1e-6f;
  static constexpr float mflux = 1e-6f;
};

// ---------------------------------------------------------------- physics

struct PrimD {
  double r, vx, vy, vz, p, bx, by, bz;
};

// conserved -> primitive in FP64 (both paths).  Returns bit0 floor hit,
// bit1 non-physical.  The floor changes the primitive pressure only.
__device__ __forceinline__ int cons_to_prim(double u0, double u1, double u2, double u3,
                                            double u4, double bx, double by, double bz,
                                            double gamma, double pfloor, PrimD& w) {
  double vx = u1 / u0;
  double vy = u2 / u0;
  double vz = u3 / u0;
  double ek = 0.5 * u0 * (vx * vx + vy * vy + vz * vz);
  double em = 0.5 * (bx * bx + by * by + bz * bz);
  double p = (gamma - 1.0) * (u4 - ek - em);
  int fl = 0;
  if (p < pfloor) {
    p = pfloor;
    fl |= 1;
  }
  if (!(u0 > 0.0) || !finite(u0) || !finite(vx) || !finite(vy) || !finite(vz) || !finite(p))
    fl |= 2;
  w.r = u0; w.vx = vx; w.vy = vy; w.vz = vz; w.p = p;
  w.bx = bx; w.by = by; w.bz = bz;
  return fl;
}

// primitives of mapped cell (i, j, k) of state s, with the face-averaged field
__device__ __forceinline__ int load_prim(const Box& b, int s, int i, int j, int k, PrimD& w) {
  const size_t c = cidx(b, i, j, k);
  const double* Bx = b.B[s][0];
  const double* By = b.B[s][1];
  const double* Bz = b.B[s][2];
  double bx = 0.5 * (Bx[fidx(b, 0, i, j, k)] + Bx[fidx(b, 0, face_up(i, b.n[0], b.per[0]), j, k)]);
  double by = 0.5 * (By[fidx(b, 1, i, j, k)] + By[fidx(b, 1, i, face_up(j, b.n[1], b.per[1]), k)]);
  double bz = 0.5 * (Bz[fidx(b, 2, i, j, k)] + Bz[fidx(b, 2, i, j, face_up(k, b.n[2], b.per[2]))]);
  return cons_to_prim(b.U[s][0][c], b.U[s][1][c], b.U[s][2][c], b.U[s][3][c], b.U[s][4][c],
                      bx, by, bz, b.gamma, b.pfloor, w);
}

// face-frame state (rho, v_n, v_t1, v_t2, p, B_t1, B_t2), (n,t1,t2) cyclic
template <typename real>
struct St7 {
  real v[7];
};

template <typename real>
__device__ __forceinline__ St7<real> rotate(const PrimD& w, int d) {
  St7<real> q;
  q.v[0] = (real)w.r;
  q.v[4] = (real)w.p;
  if (d == 0) {
    q.v[1] = (real)w.vx; q.v[2] = (real)w.vy; q.v[3] = (real)w.vz;
    q.v[5] = (real)w.by; q.v[6] = (real)w.bz;
  } else if (d == 1) {
    q.v[1] = (real)w.vy; q.v[2] = (real)w.vz; q.v[3] = (real)w.vx;
    q.v[5] = (real)w.bz; q.v[6] = (real)w.bx;
  } else {
    q.v[1] = (real)w.vz; q.v[2] = (real)w.vx; q.v[3] = (real)w.vy;
    q.v[5] = (real)w.bx; q.v[6] = (real)w.by;
  }
  return q;
}

template <typename real>
__device__ __forceinline__ real minmod(real a, real b) {
  if (a > (real)0 && b > (real)0) return a < b ? a : b;
  if (a < (real)0 && b < (real)0) return a > b ? a : b;
  return (real)0;
}

// PLM interface values between cells c-1 and c from q(c-2), q(c-1), q(c),
// q(c+1)
template <typename real>
__device__ __forceinline__ void plm(real qm2, real qm1, real q0, real qp1, real& ql, real& qr) {
  real dm1 = minmod(qm1 - qm2, q0 - qm1);
  real d0 = minmod(q0 - qm1, qp1 - q0);
  ql = qm1 + (real)0.5 * dm1;
  qr = q0 - (real)0.5 * d0;
}

template <typename real>
__device__ __forceinline__ real fast_speed(real rho, real p, real bn, real bt1, real bt2,
                                           real gamma) {
  real a2 = dv(gamma * p, rho);
  real b2 = dv(bn * bn + bt1 * bt1 + bt2 * bt2, rho);
  real bn2 = dv(bn * bn, rho);
  real s = a2 + b2;
  real disc = s * s - (real)4 * a2 * bn2;
  if (disc < (real)0) disc = (real)0;
  return sq((real)0.5 * (s + sq(disc)));
}

// physical flux F and conserved vector U of a face-frame state
template <typename real>
__device__ __forceinline__ void phys_flux(const St7<real>& w, real bn, real gamma, real* f,
                                          real* u) {
  const real rho = w.v[0], vn = w.v[1], vt1 = w.v[2], vt2 = w.v[3], p = w.v[4];
  const real b1 = w.v[5], b2 = w.v[6];
  real bsq = bn * bn + b1 * b1 + b2 * b2;
  real pt = p + (real)0.5 * bsq;
  real vb = vn * bn + vt1 * b1 + vt2 * b2;
  real en = dv(p, gamma - (real)1) + (real)0.5 * rho * (vn * vn + vt1 * vt1 + vt2 * vt2) +
            (real)0.5 * bsq;
  u[0] = rho;
  u[1] = rho * vn;
  u[2] = rho * vt1;
  u[3] = rho * vt2;
  u[4] = en;
  u[5] = b1;
  u[6] = b2;
  f[0] = rho * vn;
  f[1] = rho * vn * vn + pt - bn * bn;
  f[2] = rho * vn * vt1 - bn * b1;
  f[3] = rho * vn * vt2 - bn * b2;
  f[4] = (en + pt) * vn - bn * vb;
  f[5] = vn * b1 - vt1 * bn;
  f[6] = vn * b2 - vt2 * bn;
}

template <typename real>
struct Star {
  real rho, vt1, vt2, bt1, bt2, en, vb;
  real u[7];
};

// HLLD single-star state of one side
template <typename real>
__device__ __forceinline__ void star_side(const St7<real>& w, const real* u, real pt, real sa,
                                          real sm, real pts, real bn, Star<real>& s) {
  real sd = sa - w.v[1];
  real sms = sa - sm;
  real rs = dv(w.v[0] * sd, sms);
  real dd = w.v[0] * sd * sms - bn * bn;
  real vt1s, vt2s, bt1s, bt2s;
  if (ab(dd) <= Eps<real>::deg * pts) {
    vt1s = w.v[2];
    vt2s = w.v[3];
    bt1s = w.v[5];
    bt2s = w.v[6];
  } else {
    real cv = dv(bn * (sm - w.v[1]), dd);
    real cb = dv(w.v[0] * sd * sd - bn * bn, dd);
    vt1s = w.v[2] - w.v[5] * cv;
    vt2s = w.v[3] - w.v[6] * cv;
    bt1s = w.v[5] * cb;
    bt2s = w.v[6] * cb;
  }
  real vb = w.v[1] * bn + w.v[2] * w.v[5] + w.v[3] * w.v[6];
  real vbs = sm * bn + vt1s * bt1s + vt2s * bt2s;
  real ens = dv(sd * u[4] - pt * w.v[1] + pts * sm + bn * (vb - vbs), sms);
  s.rho = rs;
  s.vt1 = vt1s;
  s.vt2 = vt2s;
  s.bt1 = bt1s;
  s.bt2 = bt2s;
  s.en = ens;
  s.vb = vbs;
  s.u[0] = rs;
  s.u[1] = rs * sm;
  s.u[2] = rs * vt1s;
  s.u[3] = rs * vt2s;
  s.u[4] = ens;
  s.u[5] = bt1s;
  s.u[6] = bt2s;
}

template <typename real>
__device__ __forceinline__ real star_pressure(const Star<real>& s, real sm, real bn, real gamma) {
  return (gamma - (real)1) *
         (s.en - (real)0.5 * s.rho * (sm * sm + s.vt1 * s.vt1 + s.vt2 * s.vt2) -
          (real)0.5 * (bn * bn + s.bt1 * s.bt1 + s.bt2 * s.bt2));
}

// Riemann flux at one face: HLLD, HLL when the HLLD star states are not
// physical.  f[7] = (mass, mom n, mom t1, mom t2, energy, B_t1, B_t2); *fm is
// the mass flux handed to the CT upwinding (zero when zero up to rounding).
// Returns 1 when HLL was used.
template <typename real>
__device__ __forceinline__ int riemann(const St7<real>& wl, const St7<real>& wr, real bn,
                                       real gamma, real* f, real* fm) {
  real uL[7], fL[7], uR[7], fR[7];
  phys_flux(wl, bn, gamma, fL, uL);
  phys_flux(wr, bn, gamma, fR, uR);
  real cfl = fast_speed(wl.v[0], wl.v[4], bn, wl.v[5], wl.v[6], gamma);
  real cfr = fast_speed(wr.v[0], wr.v[4], bn, wr.v[5], wr.v[6], gamma);
  real cmax = cfl > cfr ? cfl : cfr;
  real umin = wl.v[1] < wr.v[1] ? wl.v[1] : wr.v[1];
  real umax = wl.v[1] > wr.v[1] ? wl.v[1] : wr.v[1];
  real sl = umin - cmax;
  real sr = umax + cmax;
  int used = 0;
  if (sl > (real)0) {
#pragma unroll
    for (int c = 0; c < 7; c++) f[c] = fL[c];
  } else if (sr < (real)0) {
#pragma unroll
    for (int c = 0; c < 7; c++) f[c] = fR[c];
  } else {
    real ptl = wl.v[4] + (real)0.5 * (bn * bn + wl.v[5] * wl.v[5] + wl.v[6] * wl.v[6]);
    real ptr = wr.v[4] + (real)0.5 * (bn * bn + wr.v[5] * wr.v[5] + wr.v[6] * wr.v[6]);
    real sdl = sl - wl.v[1];
    real sdr = sr - wr.v[1];
    real den = sdr * wr.v[0] - sdl * wl.v[0];
    real sm = dv(sdr * wr.v[0] * wr.v[1] - sdl * wl.v[0] * wl.v[1] - ptr + ptl, den);
    real pts = dv(sdr * wr.v[0] * ptl - sdl * wl.v[0] * ptr +
                      wl.v[0] * wr.v[0] * sdr * sdl * (wr.v[1] - wl.v[1]),
                  den);
    bool ok = (sl < sm) && (sm < sr) && (pts > (real)0);
    real fo[7];
    if (ok) {
      Star<real> stl, str;
      star_side(wl, uL, ptl, sl, sm, pts, bn, stl);
      star_side(wr, uR, ptr, sr, sm, pts, bn, str);
      if (!(star_pressure(stl, sm, bn, gamma) > (real)0) ||
          !(star_pressure(str, sm, bn, gamma) > (real)0))
        ok = false;
      if (ok) {
        if ((real)0.5 * bn * bn <= Eps<real>::bsmall * pts) {
          if (sm > (real)0) {
#pragma unroll
            for (int c = 0; c < 7; c++) fo[c] = fL[c] + sl * (stl.u[c] - uL[c]);
          } else {
#pragma unroll
            for (int c = 0; c < 7; c++) fo[c] = fR[c] + sr * (str.u[c] - uR[c]);
          }
        } else {
          real sql = sq(stl.rho), sqr = sq(str.rho);
          real ssl = sm - dv(ab(bn), sql);
          real ssr = sm + dv(ab(bn), sqr);
          real sgn = bn > (real)0 ? (real)1 : (real)-1;
          real ssum = sql + sqr;
          real vt1ss = dv(sql * stl.vt1 + sqr * str.vt1 + (str.bt1 - stl.bt1) * sgn, ssum);
          real vt2ss = dv(sql * stl.vt2 + sqr * str.vt2 + (str.bt2 - stl.bt2) * sgn, ssum);
          real bt1ss = dv(sql * str.bt1 + sqr * stl.bt1 + sql * sqr * (str.vt1 - stl.vt1) * sgn, ssum);
          real bt2ss = dv(sql * str.bt2 + sqr * stl.bt2 + sql * sqr * (str.vt2 - stl.vt2) * sgn, ssum);
          real vbss = sm * bn + vt1ss * bt1ss + vt2ss * bt2ss;
          if (sm > (real)0) {
            real fs[7];
#pragma unroll
            for (int c = 0; c < 7; c++) fs[c] = fL[c] + sl * (stl.u[c] - uL[c]);
            if (ssl > (real)0) {
#pragma unroll
              for (int c = 0; c < 7; c++) fo[c] = fs[c];
            } else {
              real uss[7];
              uss[0] = stl.rho;
              uss[1] = stl.rho * sm;
              uss[2] = stl.rho * vt1ss;
              uss[3] = stl.rho * vt2ss;
              uss[4] = stl.en - sql * (stl.vb - vbss) * sgn;
              uss[5] = bt1ss;
              uss[6] = bt2ss;
#pragma unroll
              for (int c = 0; c < 7; c++) fo[c] = fs[c] + ssl * (uss[c] - stl.u[c]);
            }
          } else {
            real fs[7];
#pragma unroll
            for (int c = 0; c < 7; c++) fs[c] = fR[c] + sr * (str.u[c] - uR[c]);
            if (ssr < (real)0) {
#pragma unroll
              for (int c = 0; c < 7; c++) fo[c] = fs[c];
            } else {
              real uss[7];
              uss[0] = str.rho;
              uss[1] = str.rho * sm;
              uss[2] = str.rho * vt1ss;
              uss[3] = str.rho * vt2ss;
              uss[4] = str.en + sqr * (str.vb - vbss) * sgn;
              uss[5] = bt1ss;
              uss[6] = bt2ss;
#pragma unroll
              for (int c = 0; c < 7; c++) fo[c] = fs[c] + ssr * (uss[c] - str.u[c]);
            }
          }
        }
#pragma unroll
        for (int c = 0; c < 7; c++)
          if (!finite(fo[c])) ok = false;
      }
    }
    if (ok) {
#pragma unroll
      for (int c = 0; c < 7; c++) f[c] = fo[c];
    } else {
      used = 1;
      if (sl >= (real)0) {
#pragma unroll
        for (int c = 0; c < 7; c++) f[c] = fL[c];
      } else if (sr <= (real)0) {
#pragma unroll
        for (int c = 0; c < 7; c++) f[c] = fR[c];
      } else {
#pragma unroll
        for (int c = 0; c < 7; c++)
          f[c] = dv(sr * fL[c] - sl * fR[c] + sl * sr * (uR[c] - uL[c]), sr - sl);
      }
    }
  }
  real thr = Eps<real>::mflux * (wl.v[0] + wr.v[0]) * (ab(sl) + ab(sr));
  *fm = ab(f[0]) <= thr ? (real)0 : f[0];
  return used;
}

// PLM on the seven face-frame variables of a four-cell stencil
template <typename real>
__device__ __forceinline__ void plm_face(const St7<real>& q0, const St7<real>& q1,
                                         const St7<real>& q2, const St7<real>& q3,
                                         St7<real>& wl, St7<real>& wr) {
#pragma unroll
  for (int v = 0; v < 7; v++) plm(q0.v[v], q1.v[v], q2.v[v], q3.v[v], wl.v[v], wr.v[v]);
}

__device__ __forceinline__ void count(unsigned long long* c, int fl) {
  if (fl & 1) atomicAdd(&c[0], 1ull);
  if (fl & 2) atomicAdd(&c[2], 1ull);
}

// upwind choice of the CT average: flux > 0 -> lower side, < 0 -> upper,
// 0 -> mean
template <typename real>
__device__ __forceinline__ real upwind(real m, real lower, real upper) {
  if (m > (real)0) return lower;
  if (m < (real)0) return upper;
  return (real)0.5 * (lower + upper);
}

// ---------------------------------------------------------------- kernels

// x sweep: row segments staged in LDS; one x face per lane.  Writes the
// hydro flux, the face EMFs (E_y, E_z), the CT mass flux and the cell EMF of
// every owned cell.
template <typename real>
__global__ __launch_bounds__(kTPB) void k_sweep_x(Launch L) {
  __shared__ real sw[7][kLdsCells];
  const int s = L.stage;
  for (int tile = blockIdx.x; tile < L.ntiles; tile += gridDim.x) {
    const int bi = find_box(L.base + kXS * (L.nboxes + 1), L.nboxes, tile);
    const Box& b = L.boxes[bi];
    const int lt = tile - L.base[kXS * (L.nboxes + 1) + bi];
    const int nx = b.n[0], ny = b.n[1], nz = b.n[2];
    const int nrows = ny * nz;
    int W, R, r0, i0;
    if (b.xseg == 1) {
      W = b.nf[0];
      R = b.xr;
      r0 = lt * R;
      i0 = 0;
    } else {
      const int seg = lt % b.xseg;
      r0 = lt / b.xseg;
      R = 1;
      i0 = seg * b.xw;
      W = min(b.xw, b.nf[0] - i0);
    }
    if (b.act[0]) {
      const int WL = W + 3;
      const int ncell = R * WL;
      for (int sidx = threadIdx.x; sidx < ncell; sidx += kTPB) {
        const int r = sidx / WL;
        const int o = sidx - r * WL;
        const int row = r0 + r;
        if (row >= nrows) continue;
        const int j = row % ny, k = row / ny;
        const int i = i0 - 2 + o;
        const int im = map_cell(i, nx, b.per[0]);
        PrimD w;
        const int fl = load_prim(b, s, im, j, k, w);
        sw[0][sidx] = (real)w.r;
        sw[1][sidx] = (real)w.vx;
        sw[2][sidx] = (real)w.vy;
        sw[3][sidx] = (real)w.vz;
        sw[4][sidx] = (real)w.p;
        sw[5][sidx] = (real)w.by;
        sw[6][sidx] = (real)w.bz;
        if (o >= 2 && o < W + 2 && i >= 0 && i < nx) {
          const size_t c = cidx(b, i, j, k);
          st<real>(b.Ec[0], c, (real)(w.vz * w.by - w.vy * w.bz));
          st<real>(b.Ec[1], c, (real)(w.vx * w.bz - w.vz * w.bx));
          st<real>(b.Ec[2], c, (real)(w.vy * w.bx - w.vx * w.by));
          if (fl) count(b.cnt, fl);
        }
      }
      __syncthreads();
      for (int t = threadIdx.x; t < R * W; t += kTPB) {
        const int r = t / W;
        const int f = i0 + (t - r * W);
        const int row = r0 + r;
        if (row >= nrows) continue;
        const int j = row % ny, k = row / ny;
        const int o = r * WL + (f - i0);
        St7<real> q[4];
#pragma unroll
        for (int m = 0; m < 4; m++)
#pragma unroll
          for (int v = 0; v < 7; v++) q[m].v[v] = sw[v][o + m];
        St7<real> wl, wr;
        plm_face(q[0], q[1], q[2], q[3], wl, wr);
        const size_t fi = fidx(b, 0, f, j, k);
        const real bn = (real)b.B[s][0][fi];
        real F[7], fm;
        const int used = riemann(wl, wr, bn, (real)b.gamma, F, &fm);
        st<real>(b.FX[0], fi, F[0]);
        st<real>(b.FX[1], fi, F[1]);
        st<real>(b.FX[2], fi, F[2]);
        st<real>(b.FX[3], fi, F[3]);
        st<real>(b.FX[4], fi, F[4]);
        st<real>(b.EF[0][0], fi, F[6]);
        st<real>(b.EF[0][1], fi, -F[5]);
        st<real>(b.MF[0], fi, fm);
        if (used) atomicAdd(&b.cnt[1], 1ull);
      }
      __syncthreads();
    } else {
      // inactive x: the face carries the cell's physical flux (no divergence)
      for (int t = threadIdx.x; t < R * W; t += kTPB) {
        const int r = t / W;
        const int f = i0 + (t - r * W);
        const int row = r0 + r;
        if (row >= nrows) continue;
        const int j = row % ny, k = row / ny;
        const int im = map_cell(f, nx, b.per[0]);
        PrimD w;
        const int fl = load_prim(b, s, im, j, k, w);
        const double ecy = w.vx * w.bz - w.vz * w.bx;
        const double ecz = w.vy * w.bx - w.vx * w.by;
        const size_t fi = fidx(b, 0, f, j, k);
        st<real>(b.EF[0][0], fi, (real)ecy);
        st<real>(b.EF[0][1], fi, (real)ecz);
        st<real>(b.MF[0], fi, (real)b.U[s][1][cidx(b, im, j, k)]);
        if (f == 0) {
          const size_t c = cidx(b, 0, j, k);
          st<real>(b.Ec[0], c, (real)(w.vz * w.by - w.vy * w.bz));
          st<real>(b.Ec[1], c, (real)ecy);
          st<real>(b.Ec[2], c, (real)ecz);
          if (fl) count(b.cnt, fl);
        }
      }
    }
  }
}

// Marching sweep along axis D (1 = y, 2 = z).  Each lane owns one column of
// cells along D (lanes run along x) and slides a four-cell register window
// down its segment; one Riemann solve per face.  Y: adds the x and y flux
// divergence and writes the residual.  Z: adds the z divergence to the
// residual and applies the SSP-RK2 stage combine.
template <typename real, int D>
__device__ __forceinline__ void march_column(const Box& b, int s, int i, int tr, int j0, int j1) {
  // (i, tr): x index and the index along the remaining axis (z for D=1, y
  // for D=2); positions along D from j0 to j1 (cells [j0, j1))
  const int n = b.n[D];
  const int per = b.per[D];
  auto pos = [&](int a, int& ii, int& jj, int& kk) {
    ii = i;
    if (D == 1) { jj = a; kk = tr; } else { jj = tr; kk = a; }
  };
  St7<real> q0, q1, q2, q3;
  {
    int ii, jj, kk;
    PrimD w;
    pos(map_cell(j0 - 2, n, per), ii, jj, kk);
    load_prim(b, s, ii, jj, kk, w);
    q0 = rotate<real>(w, D);
    pos(map_cell(j0 - 1, n, per), ii, jj, kk);
    load_prim(b, s, ii, jj, kk, w);
    q1 = rotate<real>(w, D);
    pos(map_cell(j0, n, per), ii, jj, kk);
    load_prim(b, s, ii, jj, kk, w);
    q2 = rotate<real>(w, D);
  }
  real fprev[kNQ];
  const int lastface = j1;  // faces j0..j1
  const bool extra = (j1 == n) && (b.nf[D] == n + 1);
  for (int f = j0; f <= lastface; ++f) {
    int ii, jj, kk;
    pos(map_cell(f + 1, n, per), ii, jj, kk);
    PrimD w;
    load_prim(b, s, ii, jj, kk, w);
    q3 = rotate<real>(w, D);
    St7<real> wl, wr;
    plm_face(q0, q1, q2, q3, wl, wr);
    int fi_, fj_, fk_;
    pos(f, fi_, fj_, fk_);
    // face index f along D is in [0, n]; periodic face n is face 0
    if (per && f == n) {
      if (D == 1) fj_ = 0; else fk_ = 0;
    }
    const size_t fi = fidx(b, D, fi_, fj_, fk_);
    const real bn = (real)b.B[s][D][fi];
    real F[7], fm;
    const int used = riemann(wl, wr, bn, (real)b.gamma, F, &fm);
    // lab-frame hydro flux: (rho, mx, my, mz, E)
    real fl[kNQ];
    fl[0] = F[0];
    fl[4] = F[4];
    if (D == 1) { fl[2] = F[1]; fl[3] = F[2]; fl[1] = F[3]; }
    else { fl[3] = F[1]; fl[1] = F[2]; fl[2] = F[3]; }
    if (f < j1 || (f == n && extra)) {
      st<real>(b.EF[D][0], fi, F[6]);
      st<real>(b.EF[D][1], fi, -F[5]);
      st<real>(b.MF[D], fi, fm);
      if (used) atomicAdd(&b.cnt[1], 1ull);
    }
    if (f > j0) {
      // cell f-1 is complete
      int ci, cj, ck;
      pos(f - 1, ci, cj, ck);
      const size_t c = cidx(b, ci, cj, ck);
      const double dxD = b.dx[D];
      if (D == 1) {
        const size_t f0 = fidx(b, 0, ci, cj, ck);
        const size_t f1 = fidx(b, 0, face_up(ci, b.n[0], b.per[0]), cj, ck);
#pragma unroll
        for (int q = 0; q < kNQ; q++) {
          double r = 0.0;
          if (b.act[0])
            r = r - ((double)ld<real>(b.FX[q], f1) - (double)ld<real>(b.FX[q], f0)) / b.dx[0];
          r = r - ((double)fl[q] - (double)fprev[q]) / dxD;
          b.R[q][c] = r;
        }
      } else {
        const double dt = b.scal[0];
#pragma unroll
        for (int q = 0; q < kNQ; q++) {
          double r = b.R[q][c];
          r = r - ((double)fl[q] - (double)fprev[q]) / dxD;
          if (s == 0) {
            b.U[1][q][c] = b.U[0][q][c] + dt * (double)r;
          } else {
            b.U[0][q][c] = 0.5 * (b.U[0][q][c] + (b.U[1][q][c] + dt * (double)r));
          }
        }
      }
    }
#pragma unroll
    for (int q = 0; q < kNQ; q++) fprev[q] = fl[q];
    q0 = q1;
    q1 = q2;
    q2 = q3;
  }
}

// inactive axis D: residual from the earlier axes only, face data from the
// cell (EMF = cell EMF, mass flux = momentum)
template <typename real, int D>
__device__ __forceinline__ void inactive_column(const Box& b, int s, int i, int tr) {
  auto pos = [&](int a, int& ii, int& jj, int& kk) {
    ii = i;
    if (D == 1) { jj = a; kk = tr; } else { jj = tr; kk = a; }
  };
  const int t1 = (D + 1) % 3, t2 = (D + 2) % 3;
  for (int f = 0; f < b.nf[D]; ++f) {
    int ii, jj, kk;
    pos(map_cell(f, b.n[D], b.per[D]), ii, jj, kk);
    const size_t c = cidx(b, ii, jj, kk);
    int fi_, fj_, fk_;
    pos(f, fi_, fj_, fk_);
    const size_t fi = fidx(b, D, fi_, fj_, fk_);
    st<real>(b.EF[D][0], fi, ld<real>(b.Ec[t1], c));
    st<real>(b.EF[D][1], fi, ld<real>(b.Ec[t2], c));
    st<real>(b.MF[D], fi, (real)b.U[s][1 + D][c]);
  }
  int ci, cj, ck;
  pos(0, ci, cj, ck);
  const size_t c = cidx(b, ci, cj, ck);
  if (D == 1) {
    const size_t f0 = fidx(b, 0, ci, cj, ck);
    const size_t f1 = fidx(b, 0, face_up(ci, b.n[0], b.per[0]), cj, ck);
#pragma unroll
    for (int q = 0; q < kNQ; q++) {
      double r = 0.0;
      if (b.act[0])
        r = r - ((double)ld<real>(b.FX[q], f1) - (double)ld<real>(b.FX[q], f0)) / b.dx[0];
      b.R[q][c] = r;
    }
  } else {
    const double dt = b.scal[0];
#pragma unroll
    for (int q = 0; q < kNQ; q++) {
      double r = b.R[q][c];
      if (s == 0)
        b.U[1][q][c] = b.U[0][q][c] + dt * (double)r;
      else
        b.U[0][q][c] = 0.5 * (b.U[0][q][c] + (b.U[1][q][c] + dt * (double)r));
    }
  }
}

template <typename real, int D>
__global__ __launch_bounds__(kTPB) void k_sweep_march(Launch L) {
  const int kind = D == 1 ? kYS : kZS;
  for (int tile = blockIdx.x; tile < L.ntiles; tile += gridDim.x) {
    const int bi = find_box(L.base + kind * (L.nboxes + 1), L.nboxes, tile);
    const Box& b = L.boxes[bi];
    const int lt = tile - L.base[kind * (L.nboxes + 1) + bi];
    const int nseg = D == 1 ? b.yseg : b.zseg;
    const int sl = D == 1 ? b.ysl : b.zsl;
    const int seg = lt % nseg;
    const int ct = lt / nseg;
    const int ntr = D == 1 ? b.n[2] : b.n[1];
    const int ncols = b.n[0] * ntr;
    const int col = ct * kTPB + (int)threadIdx.x;
    if (col >= ncols) continue;
    const int i = col % b.n[0];
    const int tr = col / b.n[0];
    if (b.act[D]) {
      const int j0 = seg * sl;
      const int j1 = min(j0 + sl, b.n[D]);
      march_column<real, D>(b, L.stage, i, tr, j0, j1);
    } else {
      inactive_column<real, D>(b, L.stage, i, tr);
    }
  }
}

// Corner EMFs: for every corner position one lane computes the EMF along
// each axis c whose range contains it (contact-upwinded average).
template <typename real>
__global__ __launch_bounds__(kTPB) void k_ct_edge(Launch L) {
  for (int tile = blockIdx.x; tile < L.ntiles; tile += gridDim.x) {
    const int bi = find_box(L.base + kCTE * (L.nboxes + 1), L.nboxes, tile);
    const Box& b = L.boxes[bi];
    const int lt = tile - L.base[kCTE * (L.nboxes + 1) + bi];
    const long long p = (long long)lt * kTPB + threadIdx.x;
    const long long P = (long long)b.nf[0] * b.nf[1] * b.nf[2];
    if (p >= P) continue;
    int pos[3];
    pos[0] = (int)(p % b.nf[0]);
    pos[1] = (int)((p / b.nf[0]) % b.nf[1]);
    pos[2] = (int)(p / ((long long)b.nf[0] * b.nf[1]));
#pragma unroll
    for (int c = 0; c < 3; c++) {
      const int a = (c + 1) % 3, bb = (c + 2) % 3;
      if (pos[c] >= b.n[c]) continue;
      const int ia = pos[a], ib = pos[bb];
      const int ma1 = map_cell(ia, b.n[a], b.per[a]);
      const int ma0 = map_cell(ia - 1, b.n[a], b.per[a]);
      const int mb1 = map_cell(ib, b.n[bb], b.per[bb]);
      const int mb0 = map_cell(ib - 1, b.n[bb], b.per[bb]);
      int q[3];
      // a-faces (ia; ib) and (ia; ib-1)
      q[c] = pos[c];
      q[a] = ia;
      q[bb] = mb1;
      const size_t fa1i = fidx(b, a, q[0], q[1], q[2]);
      q[bb] = mb0;
      const size_t fa0i = fidx(b, a, q[0], q[1], q[2]);
      // b-faces (ib; ia) and (ib; ia-1)
      q[bb] = ib;
      q[a] = ma1;
      const size_t fb1i = fidx(b, bb, q[0], q[1], q[2]);
      q[a] = ma0;
      const size_t fb0i = fidx(b, bb, q[0], q[1], q[2]);
      // cells (ia-1, ib-1), (ia, ib-1), (ia-1, ib), (ia, ib)
      real ec[4];
      q[a] = ma0; q[bb] = mb0; ec[0] = ld<real>(b.Ec[c], cidx(b, q[0], q[1], q[2]));
      q[a] = ma1; q[bb] = mb0; ec[1] = ld<real>(b.Ec[c], cidx(b, q[0], q[1], q[2]));
      q[a] = ma0; q[bb] = mb1; ec[2] = ld<real>(b.Ec[c], cidx(b, q[0], q[1], q[2]));
      q[a] = ma1; q[bb] = mb1; ec[3] = ld<real>(b.Ec[c], cidx(b, q[0], q[1], q[2]));
      const real fa1 = ld<real>(b.EF[a][1], fa1i);
      const real fa0 = ld<real>(b.EF[a][1], fa0i);
      const real fb1 = ld<real>(b.EF[bb][0], fb1i);
      const real fb0 = ld<real>(b.EF[bb][0], fb0i);
      const real m_a1 = ld<real>(b.MF[a], fa1i);
      const real m_a0 = ld<real>(b.MF[a], fa0i);
      const real m_b1 = ld<real>(b.MF[bb], fb1i);
      const real m_b0 = ld<real>(b.MF[bb], fb0i);
      const real dbp = upwind(m_a1, ec[2] - fb0, ec[3] - fb1);
      const real dbm = upwind(m_a0, fb0 - ec[0], fb1 - ec[1]);
      const real dap = upwind(m_b1, ec[1] - fa0, ec[3] - fa1);
      const real dam = upwind(m_b0, fa0 - ec[0], fa1 - ec[2]);
      const real e = (real)0.25 * (fa1 + fa0 + fb1 + fb0) + (real)0.25 * (dbm - dbp) +
                     (real)0.25 * (dam - dap);
      st<real>(b.ED[c], eidx(b, c, pos[0], pos[1], pos[2]), e);
    }
  }
}

// Face update: dB_d/dt = -[(E_f(e+1/2) - E_f(e-1/2))/dx_e
//                          - (E_e(f+1/2) - E_e(f-1/2))/dx_f], (d, e, f)
// cyclic, formed in FP64, then the SSP-RK2 stage combine.
template <typename real>
__global__ __launch_bounds__(kTPB) void k_ct_face(Launch L) {
  for (int tile = blockIdx.x; tile < L.ntiles; tile += gridDim.x) {
    const int bi = find_box(L.base + kCTF * (L.nboxes + 1), L.nboxes, tile);
    const Box& b = L.boxes[bi];
    const int lt = tile - L.base[kCTF * (L.nboxes + 1) + bi];
    const long long p = (long long)lt * kTPB + threadIdx.x;
    const long long P = (long long)b.nf[0] * b.nf[1] * b.nf[2];
    if (p >= P) continue;
    int pos[3];
    pos[0] = (int)(p % b.nf[0]);
    pos[1] = (int)((p / b.nf[0]) % b.nf[1]);
    pos[2] = (int)(p / ((long long)b.nf[0] * b.nf[1]));
    const double dt = b.scal[0];
#pragma unroll
    for (int d = 0; d < 3; d++) {
      const int e = (d + 1) % 3, f = (d + 2) % 3;
      if (pos[e] >= b.n[e] || pos[f] >= b.n[f]) continue;
      double t1 = 0.0, t2 = 0.0;
      const size_t e0f = eidx(b, f, pos[0], pos[1], pos[2]);
      const size_t e0e = eidx(b, e, pos[0], pos[1], pos[2]);
      if (b.act[e]) {
        int q[3] = {pos[0], pos[1], pos[2]};
        q[e] = face_up(pos[e], b.n[e], b.per[e]);
        const double hi = (double)ld<real>(b.ED[f], eidx(b, f, q[0], q[1], q[2]));
        const double lo = (double)ld<real>(b.ED[f], e0f);
        t1 = (hi - lo) / b.dx[e];
      }
      if (b.act[f]) {
        int q[3] = {pos[0], pos[1], pos[2]};
        q[f] = face_up(pos[f], b.n[f], b.per[f]);
        const double hi = (double)ld<real>(b.ED[e], eidx(b, e, q[0], q[1], q[2]));
        const double lo = (double)ld<real>(b.ED[e], e0e);
        t2 = (hi - lo) / b.dx[f];
      }
      const double rate = -(t1 - t2);
      const size_t fi = fidx(b, d, pos[0], pos[1], pos[2]);
      if (L.stage == 0)
        b.B[1][d][fi] = b.B[0][d][fi] + dt * rate;
      else
        b.B[0][d][fi] = 0.5 * (b.B[0][d][fi] + (b.B[1][d][fi] + dt * rate));
    }
  }
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    double w = __shfl_xor(v, o, 64);
    v = w > v ? w : v;
  }
  return v;
}

// block-wide max: wavefront butterfly, then across the four wavefronts
__device__ __forceinline__ double block_max(double v) {
  __shared__ double part[kTPB / 64];
  v = wave_max(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) part[wid] = v;
  __syncthreads();
  double m = part[0];
#pragma unroll
  for (int w = 1; w < kTPB / 64; w++) m = part[w] > m ? part[w] : m;
  __syncthreads();
  return m;
}

// CFL rate of every cell of state s, reduced to one max per tile
__global__ __launch_bounds__(kTPB) void k_lambda(Launch L) {
  for (int tile = blockIdx.x; tile < L.ntiles; tile += gridDim.x) {
    const int bi = find_box(L.base + kLAM * (L.nboxes + 1), L.nboxes, tile);
    const Box& b = L.boxes[bi];
    const int lt = tile - L.base[kLAM * (L.nboxes + 1) + bi];
    const long long p = (long long)lt * kTPB + threadIdx.x;
    const long long N = (long long)b.n[0] * b.n[1] * b.n[2];
    double lmax = 0.0;
    if (p < N) {
      const int i = (int)(p % b.n[0]);
      const int j = (int)((p / b.n[0]) % b.n[1]);
      const int k = (int)(p / ((long long)b.n[0] * b.n[1]));
      PrimD w;
      load_prim(b, L.stage, i, j, k, w);
      const double v[3] = {w.vx, w.vy, w.vz};
      const double bc[3] = {w.bx, w.by, w.bz};
#pragma unroll
      for (int d = 0; d < 3; d++) {
        if (!b.act[d]) continue;
        const double cf = fast_speed(w.r, w.p, bc[d], bc[(d + 1) % 3], bc[(d + 2) % 3], b.gamma);
        const double l = (__builtin_fabs(v[d]) + cf) / b.dx[d];
        if (l > lmax) lmax = l;
      }
    }
    const double m = block_max(lmax);
    if (threadIdx.x == 0) b.lam[lt] = m;
  }
}

// One workgroup per box: max of the tile partials -> time step.  mode 0:
// step (clamp to t_stop, advance t); mode 1: query (dt of the current state
// into scal[3]).
__global__ __launch_bounds__(kTPB) void k_dt(const Box* boxes, int mode) {
  const Box& b = boxes[blockIdx.x];
  double m = 0.0;
  for (int t = threadIdx.x; t < b.ntile[kLAM]; t += kTPB) {
    const double v = b.lam[t];
    if (v > m) m = v;
  }
  m = block_max(m);
  if (threadIdx.x == 0) {
    double dt = b.cfl / m;
    if (mode == 1) {
      b.scal[3] = dt;
    } else {
      const double t = b.scal[1];
      const double ts = b.scal[2];
      if (ts > 0.0) {
        const double rem = ts - t;
        if (rem < dt) dt = rem;
        if (dt < 0.0) dt = 0.0;
      }
      b.scal[0] = dt;
      b.scal[1] = t + dt;
    }
  }
}

// Periodic-face check of a caller array in the boundary layout: sets *bad
// when face n differs from face 0 anywhere along axis d.
__global__ __launch_bounds__(kTPB) void k_check_periodic(const double* a, int d, int nx, int ny,
                                                         int nz, int* bad) {
  // boundary layout extents: n+1 along d
  const int ex = nx + (d == 0), ey = ny + (d == 1);
  long long P = (long long)(d == 0 ? 1 : nx) * (d == 1 ? 1 : ny) * (d == 2 ? 1 : nz);
  for (long long p = blockIdx.x * (long long)kTPB + threadIdx.x; p < P;
       p += (long long)gridDim.x * kTPB) {
    int ext0 = d == 0 ? 1 : nx, ext1 = d == 1 ? 1 : ny;
    int i = (int)(p % ext0), j = (int)((p / ext0) % ext1), k = (int)(p / ((long long)ext0 * ext1));
    int i2 = i, j2 = j, k2 = k;
    if (d == 0) i2 = nx; else if (d == 1) j2 = ny; else k2 = nz;
    const size_t a0 = ((size_t)k * ey + j) * ex + i;
    const size_t a1 = ((size_t)k2 * ey + j2) * ex + i2;
    if (a[a0] != a[a1]) atomicOr(bad, 1);
  }
}

}  // namespace mhd
