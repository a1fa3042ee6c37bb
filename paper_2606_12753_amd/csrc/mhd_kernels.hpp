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
//   * two- or three-stage SSP Runge-Kutta (Shu & Osher 1988) and the CFL time step from
//     the fast magnetosonic rate.
//
// Layout in HBM: structure of arrays, C order [z][y][x], x fastest; every
// wavefront's lanes run along x so that all global loads and stores are
// coalesced, whatever the sweep direction:
//   * the x sweep stages a row segment of primitives in LDS (one load and one
//     primitive recovery per cell) and computes one x face per lane;
//   * the y and z sweeps march each lane along its column: a window of two
//     cells and a limited slope (in registers or in a per-lane LDS column)
//     slides along the strided axis, so the strided access never reaches
//     HBM as strided; each new cell is one coalesced row load, issued two
//     faces ahead of its use.
// Periodic axes wrap cell indices and store n faces per axis (face n is face
// 0); outflow axes clamp cell indices (ghost = copy of the boundary cell) and
// store n+1 faces.  All offsets are 32-bit (a box holds at most 2^29 cells
// and 2^29 face or corner positions).
//
// Every kernel takes a tile table: tiles of all boxes of an ensemble are
// numbered consecutively and a workgroup finds its box by a binary search of
// the per-box tile offsets, so one launch covers uneven boxes; the grid may
// be smaller than the tile count (persistent grid-stride loop).
//
// The arithmetic type `real` is double (FP64 path) or float (mixed path:
// FP32 reconstruction, Riemann solver, face fluxes, EMFs and the stored
// stage residual; the state, the primitive recovery, the flux differences,
// the RK accumulation, the face-field curl and the time step stay FP64).  In
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
  double dx[3], idx[3];  // cell size and its reciprocal
  double gamma, igm1, cfl, pfloor;  // igm1 = 1/(gamma-1)
  double* U[3][kNQ];  // conserved state: [0] start of step, [1], [2] stage
                      // states ([2] only for the three-stage integrator)
  double* B[3][3];    // face field, same copies
  void* Ec[3];        // cell EMF  E = -v x B
  void* FX[kNQ];      // hydro flux on x faces
  void* EF[3][2];     // EMF (E_t1, E_t2) on the faces normal to each axis
  void* MF[3];        // mass flux for the CT upwinding, per face direction
  void* R[kNQ];       // residual of the x and y fluxes, from the y march to
                      // the z march: formed in FP64 from the face fluxes,
                      // stored in the arithmetic type of the path (the
                      // mixed path rounds it to FP32 once; the RK combine
                      // itself is FP64)
  void* ED[3];        // corner EMF along each axis
  void* SP[3][2];     // outer wave speeds S_L, S_R on the faces normal to
                      // each axis (upwind CT only; null otherwise)
  void* V[3];         // cell velocity, written by the x sweep (upwind CT
                      // only; null otherwise)
  double* lam;        // per-tile max CFL rate (length: max(x tiles, cell tiles))
  double* scal;       // [0] dt, [1] t, [2] t_stop, [3] dt of the current state
  unsigned long long* cnt;  // [0] floor hits, [1] HLL fallbacks, [2] bad cells
  int xft;            // x sweep: faces per tile
  int ctx;            // corner-EMF kernel: tile width along x (kTPB / ctx
                      // rows), 0 for flat order
  int czk;            // corner-EMF kernel: planes per lane (each lane walks
                      // czk consecutive planes of its column; 1 with ctx = 0)
  int emf;            // corner EMF: 0 contact-upwinded, 1 E0 (derivatives
                      // averaged), 2 mean of the four face EMFs, 3 upwind CT
  int lim;            // slope limiter (0 minmod, 1 MC, 2 van Leer), for the
                      // upwind-CT corner states
  int ysl, yseg;      // y march: cells per segment, segments
  int zsl, zseg;      // z march
  int ntile[6];       // tiles per kernel kind
};

enum Kind { kXS = 0, kYS = 1, kZS = 2, kCTE = 3, kCTF = 4, kLAM = 5 };

// The box descriptors and the tile table are written by the host only (never
// by a kernel), so kernels read them through the constant address space:
// the compiler may then load their fields with scalar loads once and keep
// them in scalar registers across the kernels' global stores, instead of
// re-reading them through the vector memory path after every store.
typedef const __attribute__((address_space(4))) Box CBox;
typedef const __attribute__((address_space(4))) int CInt;
__device__ __forceinline__ CBox& box_at(const Box* boxes, int i) { return ((CBox*)boxes)[i]; }
__device__ __forceinline__ CInt* table(const int* p) { return (CInt*)p; }

// Per-launch arguments.
struct Launch {
  const Box* boxes;
  const int* base;  // base[kind*(nboxes+1) + b]: first tile of box b
  int nboxes;
  int ntiles;       // tiles of this kind over all boxes
  int stage;        // state the stage sweeps (0: start of step, 1, 2: stage states)
  int dst;          // state the stage's combine writes
  int comb;         // stage combine (rk_combine)
  int lam;          // x sweep: also reduce the CFL rate of the owned cells
  int xcd;          // XCD-grouped tile order (see tile_of)
};

// Tile order.  The hardware deals the workgroups of a launch round-robin to
// the eight XCDs, each with its own L2.  With L.xcd set, slot v (of
// 8*ceil(ntiles/8) slots) takes tile (v mod 8)*C + v/8, C = ceil(ntiles/8):
// each XCD then works through one contiguous run of tiles, so the
// neighbouring rows and planes that a tile's stencil reads were mostly
// fetched into the same L2.  Slots past the last tile do nothing.
__device__ __forceinline__ int tile_slots(const Launch& L) {
  return L.xcd ? ((L.ntiles + 7) >> 3) << 3 : L.ntiles;
}
__device__ __forceinline__ int tile_of(const Launch& L, int v) {
  return L.xcd ? (v & 7) * ((L.ntiles + 7) >> 3) + (v >> 3) : v;
}

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ int find_box(CInt* base, int nb, int t) {
  int lo = 0, hi = nb - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (base[mid] <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// cell index along an axis for a position at most n outside the box
__device__ __forceinline__ int map_cell(int i, int n, int per) {
  if (per) return i < 0 ? i + n : (i >= n ? i - n : i);
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// upper face of cell i along an axis
__device__ __forceinline__ int face_up(int i, int n, int per) {
  int f = i + 1;
  return (per && f == n) ? 0 : f;
}

__device__ __forceinline__ int cidx(CBox& b, int i, int j, int k) {
  return (k * b.n[1] + j) * b.n[0] + i;
}

// element of the face array normal to axis d
__device__ __forceinline__ int fidx(CBox& b, int d, int i, int j, int k) {
  int ex = d == 0 ? b.nf[0] : b.n[0];
  int ey = d == 1 ? b.nf[1] : b.n[1];
  return (k * ey + j) * ex + i;
}

// element of the corner-EMF array along axis c: face extents on the two
// other axes, cell extent along c
__device__ __forceinline__ int eidx(CBox& b, int c, int i, int j, int k) {
  int ex = c == 0 ? b.n[0] : b.nf[0];
  int ey = c == 1 ? b.n[1] : b.nf[1];
  return (k * ey + j) * ex + i;
}

// element access through the global address space (the pointers in Box are
// generic; naming the address space gives global_load / global_store rather
// than flat accesses)
//
// The element offset is formed as a 32-bit byte offset (every array of a box
// is below 4 GiB: at most 2^29 elements of 8 bytes), so that the load takes
// the array base from scalar registers and one 32-bit lane offset, shared by
// all arrays indexed alike, instead of a 64-bit address per array and lane.
typedef const __attribute__((address_space(1))) char GChar;
typedef __attribute__((address_space(1))) char GCharW;
template <typename T>
__device__ __forceinline__ T ld(const void* p, int i) {
  const unsigned off = (unsigned)i * (unsigned)sizeof(T);
  return *(const __attribute__((address_space(1))) T*)((GChar*)p + off);
}
template <typename T>
__device__ __forceinline__ void st(void* p, int i, T v) {
  const unsigned off = (unsigned)i * (unsigned)sizeof(T);
  *(__attribute__((address_space(1))) T*)((GCharW*)p + off) = v;
}

// Reciprocal, quotient and square root of the sweeps.
// FP64: the hardware estimates (v_rcp_f64, v_rsq_f64) refined by Newton-Raphson
// steps with fused multiply-adds (Markstein 1990 for the reciprocal and the
// quotient's final correction; Goldschmidt's iteration for the square root),
// within about one ulp of the correctly rounded value for operands in the
// normal range, in 5 to 9 instructions instead of the IEEE sequences' 11 to
// 18 (scaling for denormal operands, special-case fix-ups).  Every operand
// here is a density, a wave speed, a squared speed or a sum of squares in
// the normal range; a zero or non-finite operand gives a non-finite result
// (a zero or negative density is reported as a non-physical cell).  The
// square root of zero is zero.
// FP32 (the mixed path): the hardware reciprocal and square root (about
// 1 ulp).  A quotient that shares its denominator with others is formed as
// one reciprocal and products.
__device__ __forceinline__ double rcp(double b) {
  double r = __builtin_amdgcn_rcp(b);
  double e = __builtin_fma(-b, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-b, r, 1.0);
  return __builtin_fma(r, e, r);
}
__device__ __forceinline__ float rcp(float b) { return __builtin_amdgcn_rcpf(b); }
// single quotient: the refined reciprocal, the product and one residual
// correction in FP64; reciprocal and product in FP32
__device__ __forceinline__ double quot(double a, double b) {
  const double r = rcp(b);
  const double q = a * r;
  return __builtin_fma(__builtin_fma(-b, q, a), r, q);
}
__device__ __forceinline__ float quot(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double sq(double x) {
  const double y = __builtin_amdgcn_rsq(x);  // estimate of 1/sqrt(x)
  double g = x * y, h = 0.5 * y;            // g ~ sqrt(x), h ~ 1/(2 sqrt(x))
  const double e = __builtin_fma(-g, h, 0.5);
  g = __builtin_fma(g, e, g);
  h = __builtin_fma(h, e, h);
  double d = __builtin_fma(-g, g, x);
  g = __builtin_fma(d, h, g);
  d = __builtin_fma(-g, g, x);
  g = __builtin_fma(d, h, g);
  return x > 0.0 ? g : x;
}
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
  double ir = rcp(u0);
  double vx = u1 * ir;
  double vy = u2 * ir;
  double vz = u3 * ir;
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

// Raw data of one cell: conserved variables and its six faces.
struct Raw {
  double u[kNQ];
  double bf[6];  // bx lo/hi, by lo/hi, bz lo/hi
};

// Offsets of mapped cell (i, j, k) and its six faces.
struct Addr {
  int c, bx0, bx1, by0, by1, bz0, bz1;
};

__device__ __forceinline__ Addr addr_of(CBox& b, int i, int j, int k) {
  Addr a;
  const int nx = b.n[0], ny = b.n[1];
  a.c = (k * ny + j) * nx + i;
  a.bx0 = (k * ny + j) * b.nf[0] + i;
  a.bx1 = (b.per[0] && i + 1 == nx) ? a.bx0 - i : a.bx0 + 1;
  a.by0 = (k * b.nf[1] + j) * nx + i;
  a.by1 = (b.per[1] && j + 1 == ny) ? a.by0 - j * nx : a.by0 + nx;
  a.bz0 = a.c;
  a.bz1 = (b.per[2] && k + 1 == b.n[2]) ? a.c - k * nx * ny : a.c + nx * ny;
  return a;
}

__device__ __forceinline__ Raw load_raw(CBox& b, int s, const Addr& a) {
  Raw r;
#pragma unroll
  for (int q = 0; q < kNQ; q++) r.u[q] = ld<double>(b.U[s][q], a.c);
  r.bf[0] = ld<double>(b.B[s][0], a.bx0);
  r.bf[1] = ld<double>(b.B[s][0], a.bx1);
  r.bf[2] = ld<double>(b.B[s][1], a.by0);
  r.bf[3] = ld<double>(b.B[s][1], a.by1);
  r.bf[4] = ld<double>(b.B[s][2], a.bz0);
  r.bf[5] = ld<double>(b.B[s][2], a.bz1);
  return r;
}

__device__ __forceinline__ int raw_to_prim(CBox& b, const Raw& r, PrimD& w) {
  double bx = 0.5 * (r.bf[0] + r.bf[1]);
  double by = 0.5 * (r.bf[2] + r.bf[3]);
  double bz = 0.5 * (r.bf[4] + r.bf[5]);
  return cons_to_prim(r.u[0], r.u[1], r.u[2], r.u[3], r.u[4], bx, by, bz, b.gamma, b.pfloor, w);
}

// primitives of mapped cell (i, j, k) of state s, with the face-averaged field
__device__ __forceinline__ int load_prim(CBox& b, int s, int i, int j, int k, PrimD& w) {
  return raw_to_prim(b, load_raw(b, s, addr_of(b, i, j, k)), w);
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

__device__ __forceinline__ double vmin(double a, double b) { return __builtin_fmin(a, b); }
__device__ __forceinline__ double vmax(double a, double b) { return __builtin_fmax(a, b); }
__device__ __forceinline__ float vmin(float a, float b) { return __builtin_fminf(a, b); }
__device__ __forceinline__ float vmax(float a, float b) { return __builtin_fmaxf(a, b); }

// minmod: the argument of smaller magnitude when both have the same sign,
// else zero; as max(min(a,b), min(max(a,b),0)), four min/max instructions
// and no branch (same value as the case-by-case definition; a zero result
// may carry either sign)
template <typename real>
__device__ __forceinline__ real minmod(real a, real b) {
  return vmax(vmin(a, b), vmin(vmax(a, b), (real)0));
}

// Slope limiter on the two one-sided differences a (left) and b (right):
// LIM 0 minmod, 1 monotonised central (the central difference bounded by
// twice each one-sided one; van Leer 1977), 2 van Leer's harmonic mean
// 2ab/(a + b) (van Leer 1974); zero where a and b differ in sign.
template <int LIM, typename real>
__device__ __forceinline__ real limit(real a, real b) {
  if constexpr (LIM == 0) {
    return minmod(a, b);
  } else if constexpr (LIM == 1) {
    const real c = (real)0.5 * (a + b);
    if (a > (real)0 && b > (real)0) return vmin(c, vmin((real)2 * a, (real)2 * b));
    if (a < (real)0 && b < (real)0) return vmax(c, vmax((real)2 * a, (real)2 * b));
    return (real)0;
  } else {
    if ((a > (real)0 && b > (real)0) || (a < (real)0 && b < (real)0))
      return quot((real)2 * a * b, a + b);
    return (real)0;
  }
}

// PLM interface values between cells c-1 and c from q(c-2), q(c-1), q(c),
// q(c+1)
template <typename real, int LIM = 0>
__device__ __forceinline__ void plm(real qm2, real qm1, real q0, real qp1, real& ql, real& qr) {
  real dm1 = limit<LIM>(qm1 - qm2, q0 - qm1);
  real d0 = limit<LIM>(q0 - qm1, qp1 - q0);
  ql = qm1 + (real)0.5 * dm1;
  qr = q0 - (real)0.5 * d0;
}

// Limited slope of a cell in the characteristic fields of its own state
// (face-frame primitives q0, normal field bn; neighbours qm, qp): the two
// one-sided differences are projected on the left eigenvectors of the
// primitive-variable MHD system, limited by minmod per field and projected
// back with the right eigenvectors (Roe & Balsara 1996 normalisation, waves
// u-c_f, u-c_a, u-c_s, u, u+c_s, u+c_a, u+c_f).  Where the slope would make
// the density or pressure at a face of the cell non-positive, the primitive
// minmod slope is used.  The eigenvector entries are formed in a fixed
// order and the projections are dense sums in index order, so FP64 results
// are reproducible bit for bit.
template <int LIM, typename real>
__device__ __forceinline__ St7<real> char_slope(const St7<real>& qm, const St7<real>& q0,
                                                const St7<real>& qp, real bn, real gamma) {
  real dm[7], dp[7];
#pragma unroll
  for (int v = 0; v < 7; v++) {
    dm[v] = q0.v[v] - qm.v[v];
    dp[v] = qp.v[v] - q0.v[v];
  }
  const real rho = q0.v[0], p = q0.v[4], by = q0.v[5], bz = q0.v[6];
  const real ir = rcp(rho);
  const real sr = sq(rho);
  const real a2 = gamma * p * ir;
  const real a = sq(a2);
  const real bn2 = bn * bn * ir;
  const real bt2 = (by * by + bz * bz) * ir;
  const real dd = a2 - bn2;
  const real disc = dd * dd + bt2 * ((real)2 * (a2 + bn2) + bt2);
  const real sqd = sq(disc);
  const real cf2 = (real)0.5 * (a2 + bn2 + bt2 + sqd);
  const real cs2 = quot(a2 * bn2, cf2);
  const real cf = sq(cf2), cs = sq(cs2);
  real af, as;
  if (sqd > (real)0) {
    // a^2 - c_s^2 and c_f^2 - a^2 without cancellation (the factor that
    // cancels is formed from the product of the two)
    const real g = bt2 * ((real)2 * (a2 + bn2) + bt2);
    real sp, sm;
    if (dd > (real)0) {
      sp = sqd + dd;
      sm = quot(g, sp);
    } else {
      sm = sqd - dd;
      sp = quot(g, sm);
    }
    real af2 = quot((real)0.5 * (sp - bt2), sqd);
    real as2 = quot((real)0.5 * (sm + bt2), sqd);
    af2 = af2 < (real)0 ? (real)0 : (af2 > (real)1 ? (real)1 : af2);
    as2 = as2 < (real)0 ? (real)0 : (as2 > (real)1 ? (real)1 : as2);
    af = sq(af2);
    as = sq(as2);
  } else {
    af = (real)1;
    as = (real)0;
  }
  const real bt = sq(by * by + bz * bz);
  real bey, bez;
  if (bt > (real)0) {
    bey = quot(by, bt);
    bez = quot(bz, bt);
  } else {
    bey = rcp(sq((real)2));
    bez = bey;
  }
  const real sg = bn < (real)0 ? (real)-1 : (real)1;
  const real qf = sg * af * cf, qs = sg * as * cs;
  const real Af = af * a * sr, As = as * a * sr;
  const real N = quot((real)0.5, a2);
  real L[7][7], R[7][7];
#pragma unroll
  for (int v = 0; v < 7; v++)
#pragma unroll
    for (int k = 0; k < 7; k++) L[v][k] = R[v][k] = (real)0;
  L[0][1] = -N * af * cf;  L[0][2] = N * qs * bey;  L[0][3] = N * qs * bez;
  L[0][4] = N * af * ir;  L[0][5] = N * As * bey * ir;  L[0][6] = N * As * bez * ir;
  L[6][1] = N * af * cf;  L[6][2] = -N * qs * bey;  L[6][3] = -N * qs * bez;
  L[6][4] = N * af * ir;  L[6][5] = N * As * bey * ir;  L[6][6] = N * As * bez * ir;
  L[1][2] = (real)-0.5 * bez;  L[1][3] = (real)0.5 * bey;
  L[1][5] = quot((real)-0.5 * sg * bez, sr);  L[1][6] = quot((real)0.5 * sg * bey, sr);
  L[5][2] = (real)-0.5 * bez;  L[5][3] = (real)0.5 * bey;
  L[5][5] = quot((real)0.5 * sg * bez, sr);  L[5][6] = quot((real)-0.5 * sg * bey, sr);
  L[2][1] = -N * as * cs;  L[2][2] = -N * qf * bey;  L[2][3] = -N * qf * bez;
  L[2][4] = N * as * ir;  L[2][5] = -N * Af * bey * ir;  L[2][6] = -N * Af * bez * ir;
  L[4][1] = N * as * cs;  L[4][2] = N * qf * bey;  L[4][3] = N * qf * bez;
  L[4][4] = N * as * ir;  L[4][5] = -N * Af * bey * ir;  L[4][6] = -N * Af * bez * ir;
  L[3][0] = (real)1;  L[3][4] = quot((real)-1, a2);
  real ch[7];
#pragma unroll
  for (int k = 0; k < 7; k++) {
    real cm = (real)0, cp = (real)0;
#pragma unroll
    for (int v = 0; v < 7; v++) {
      cm = cm + L[k][v] * dm[v];
      cp = cp + L[k][v] * dp[v];
    }
    ch[k] = limit<LIM>(cm, cp);
  }
  R[0][0] = rho * af;  R[1][0] = -af * cf;  R[2][0] = qs * bey;  R[3][0] = qs * bez;
  R[4][0] = rho * af * a2;  R[5][0] = As * bey;  R[6][0] = As * bez;
  R[0][6] = rho * af;  R[1][6] = af * cf;  R[2][6] = -qs * bey;  R[3][6] = -qs * bez;
  R[4][6] = rho * af * a2;  R[5][6] = As * bey;  R[6][6] = As * bez;
  R[2][1] = -bez;  R[3][1] = bey;  R[5][1] = -sg * sr * bez;  R[6][1] = sg * sr * bey;
  R[2][5] = -bez;  R[3][5] = bey;  R[5][5] = sg * sr * bez;  R[6][5] = -sg * sr * bey;
  R[0][2] = rho * as;  R[1][2] = -as * cs;  R[2][2] = -qf * bey;  R[3][2] = -qf * bez;
  R[4][2] = rho * as * a2;  R[5][2] = -Af * bey;  R[6][2] = -Af * bez;
  R[0][4] = rho * as;  R[1][4] = as * cs;  R[2][4] = qf * bey;  R[3][4] = qf * bez;
  R[4][4] = rho * as * a2;  R[5][4] = -Af * bey;  R[6][4] = -Af * bez;
  R[0][3] = (real)1;
  St7<real> d;
#pragma unroll
  for (int v = 0; v < 7; v++) {
    real s = (real)0;
#pragma unroll
    for (int k = 0; k < 7; k++) s = s + R[v][k] * ch[k];
    d.v[v] = s;
  }
  const bool ok = q0.v[0] + (real)0.5 * d.v[0] > (real)0 && q0.v[0] - (real)0.5 * d.v[0] > (real)0 &&
                  q0.v[4] + (real)0.5 * d.v[4] > (real)0 && q0.v[4] - (real)0.5 * d.v[4] > (real)0;
  if (!ok) {
#pragma unroll
    for (int v = 0; v < 7; v++) d.v[v] = limit<LIM>(dm[v], dp[v]);
  }
  return d;
}

// square of the fast magnetosonic speed along n
template <typename real>
__device__ __forceinline__ real fast_speed_sq(real rho, real p, real bn, real bt1, real bt2,
                                              real gamma) {
  real ir = rcp(rho);
  real a2 = gamma * p * ir;
  real b2 = (bn * bn + bt1 * bt1 + bt2 * bt2) * ir;
  real bn2 = bn * bn * ir;
  real s = a2 + b2;
  real disc = s * s - (real)4 * a2 * bn2;
  if (disc < (real)0) disc = (real)0;
  return (real)0.5 * (s + sq(disc));
}

template <typename real>
__device__ __forceinline__ real fast_speed(real rho, real p, real bn, real bt1, real bt2,
                                           real gamma) {
  return sq(fast_speed_sq(rho, p, bn, bt1, bt2, gamma));
}

// total energy of a face-frame state (igm1 = 1/(gamma-1))
template <typename real>
__device__ __forceinline__ real energy(const St7<real>& w, real bn, real igm1) {
  real bsq = bn * bn + w.v[5] * w.v[5] + w.v[6] * w.v[6];
  return w.v[4] * igm1 +
         (real)0.5 * w.v[0] * (w.v[1] * w.v[1] + w.v[2] * w.v[2] + w.v[3] * w.v[3]) +
         (real)0.5 * bsq;
}

// physical flux F and conserved vector U of a face-frame state whose total
// energy en and total pressure pt are known
template <typename real>
__device__ __forceinline__ void phys_flux_ep(const St7<real>& w, real bn, real en, real pt,
                                             real* f, real* u) {
  const real rho = w.v[0], vn = w.v[1], vt1 = w.v[2], vt2 = w.v[3];
  const real b1 = w.v[5], b2 = w.v[6];
  real vb = vn * bn + vt1 * b1 + vt2 * b2;
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

// physical flux F and conserved vector U of a face-frame state
template <typename real>
__device__ __forceinline__ void phys_flux(const St7<real>& w, real bn, real igm1, real* f,
                                          real* u) {
  const real p = w.v[4], b1 = w.v[5], b2 = w.v[6];
  const real rho = w.v[0], vn = w.v[1], vt1 = w.v[2], vt2 = w.v[3];
  real bsq = bn * bn + b1 * b1 + b2 * b2;
  real pt = p + (real)0.5 * bsq;
  real en = p * igm1 + (real)0.5 * rho * (vn * vn + vt1 * vt1 + vt2 * vt2) + (real)0.5 * bsq;
  phys_flux_ep(w, bn, en, pt, f, u);
}

// U_R - U_L of two face-frame states, formed from differences of the states
// (the total energies themselves are never subtracted: at low plasma beta
// they are dominated by the magnetic energy, and their difference would carry
// its rounding)
template <typename real>
__device__ __forceinline__ void state_jump(const St7<real>& wl, const St7<real>& wr, real igm1,
                                           real* du) {
  du[0] = wr.v[0] - wl.v[0];
  du[1] = wr.v[0] * wr.v[1] - wl.v[0] * wl.v[1];
  du[2] = wr.v[0] * wr.v[2] - wl.v[0] * wl.v[2];
  du[3] = wr.v[0] * wr.v[3] - wl.v[0] * wl.v[3];
  const real db1 = wr.v[5] - wl.v[5], db2 = wr.v[6] - wl.v[6];
  const real kr = wr.v[1] * wr.v[1] + wr.v[2] * wr.v[2] + wr.v[3] * wr.v[3];
  const real kl = wl.v[1] * wl.v[1] + wl.v[2] * wl.v[2] + wl.v[3] * wl.v[3];
  du[4] = (wr.v[4] - wl.v[4]) * igm1 + (real)0.5 * (wr.v[0] * kr - wl.v[0] * kl) +
          (real)0.5 * (db1 * (wr.v[5] + wl.v[5]) + db2 * (wr.v[6] + wl.v[6]));
  du[5] = db1;
  du[6] = db2;
}

// HLL flux with outer speeds sl < 0 < sr (or the upwind flux at the edges),
// as F_L + S_L (S_R (U_R - U_L) - (F_R - F_L)) / (S_R - S_L): the left flux
// plus a term proportional to the jump
template <typename real>
__device__ __forceinline__ void hll_flux(const St7<real>& wl, const St7<real>& wr, real bn,
                                         real igm1, real sl, real sr, real* f) {
  real uL[7], fL[7], uR[7], fR[7];
  phys_flux(wl, bn, igm1, fL, uL);
  phys_flux(wr, bn, igm1, fR, uR);
  if (sl >= (real)0) {
#pragma unroll
    for (int c = 0; c < 7; c++) f[c] = fL[c];
  } else if (sr <= (real)0) {
#pragma unroll
    for (int c = 0; c < 7; c++) f[c] = fR[c];
  } else {
    real du[7];
    state_jump(wl, wr, igm1, du);
    const real w = sl * rcp(sr - sl);
#pragma unroll
    for (int c = 0; c < 7; c++) f[c] = fL[c] + w * (sr * du[c] - (fR[c] - fL[c]));
  }
}

// HLLD single-star state of one side, kept as jumps from that side's state:
// drho = rho* - rho, dv = v*_t - v_t, db = B*_t - B_t, den = E* - E, and the
// thermal pressure p* that E* implies.  The HLLD relations (Miyoshi & Kusano
// 2005) rearranged so that each jump is a product with S_M - u (or the
// side's own differences), which vanishes for a state at rest against the
// contact: rho* - rho = rho (S_M - u)/(S - S_M); B*_t - B_t = B_t m (S_M - u)/D
// and v*_t - v_t = -B_n B_t (S_M - u)/D with m = rho (S - u), D = m (S - S_M)
// - B_n^2; p_T* - p_T = m (S_M - u); E* - E = [(S_M - u)(E + p_T - B_n^2) +
// (p_T* - p_T) S_M - B_n (v_t.dB + dv.B*_t)] / (S - S_M).
// Only the jumps are kept (the star values are the side's state plus its
// jump); the return value says whether p* > 0.
template <typename real>
struct StarD {
  real drho, dv1, dv2, db1, db2, den;
};

template <typename real>
__device__ __forceinline__ bool star_side(const St7<real>& w, real en, real pt, real sa, real sm,
                                          real pts, real bn, real gamma, StarD<real>& s) {
  const real sd = sa - w.v[1];
  const real isms = rcp(sa - sm);
  const real du = sm - w.v[1];
  s.drho = w.v[0] * du * isms;
  const real m = w.v[0] * sd;  // mass flux through the outer wave
  const real dd = m * (sa - sm) - bn * bn;
  if (ab(dd) <= Eps<real>::deg * pts) {
    // degenerate: tangential velocity and field pass through unchanged
    s.dv1 = s.dv2 = s.db1 = s.db2 = (real)0;
  } else {
    const real idd = rcp(dd);
    const real cv = -bn * du * idd;
    const real cb = m * du * idd;
    s.dv1 = w.v[5] * cv;
    s.dv2 = w.v[6] * cv;
    s.db1 = w.v[5] * cb;
    s.db2 = w.v[6] * cb;
  }
  const real v1 = w.v[2] + s.dv1, v2 = w.v[3] + s.dv2;
  const real b1 = w.v[5] + s.db1, b2 = w.v[6] + s.db2;
  const real dpt = m * du;
  s.den = (du * (en + pt - bn * bn) + dpt * sm -
           bn * (w.v[2] * s.db1 + w.v[3] * s.db2 + s.dv1 * b1 + s.dv2 * b2)) *
          isms;
  // p* = (gamma-1)(E* - rho*|v*|^2/2 - |B*|^2/2), as the side's pressure plus
  // the jumps of the energy, kinetic and magnetic terms
  const real dk = s.drho * (sm * sm + v1 * v1 + v2 * v2) +
                  w.v[0] * (du * (sm + w.v[1]) + s.dv1 * (w.v[2] + v1) + s.dv2 * (w.v[3] + v2));
  const real dm = s.db1 * (w.v[5] + b1) + s.db2 * (w.v[6] + b2);
  return w.v[4] + (gamma - (real)1) * (s.den - (real)0.5 * dk - (real)0.5 * dm) > (real)0;
}

template <typename real>
__device__ __forceinline__ real sel(bool c, real a, real b) {
  return c ? a : b;
}

// Riemann flux at one face.  RS = 0: HLLD, HLL when the HLLD star states are
// not physical; RS = 1: HLL at every face.  f[7] = (mass, mom n, mom t1,
// mom t2, energy, B_t1, B_t2); *fm is the mass flux handed to the CT
// upwinding (zero when zero up to rounding); sp = (S_L, S_R), the outer wave
// speeds (read by the upwind CT).  Returns 1 when HLLD fell back to HLL.
//
// The flux of the Riemann fan at x/t = 0 lies on the side of the contact
// given by sign(S_M): the solver computes both single-star states (both
// enter the double-star average and the positivity check), then selects the
// side once and assembles F* = F_a + S_a (U* - U_a), and F** = F* + S*_a
// (U** - U*) when the rotational wave of that side is left of (right of)
// x/t = 0, with selects instead of divergent branches.  Every U* - U_a and
// U** - U* is formed as a jump (star_side), never as a difference of two
// total energies: in FP32 at low plasma beta the rounding of E (mostly
// magnetic energy) would otherwise enter every flux, even between two states
// at rest.
template <typename real, int RS>
__device__ __forceinline__ int riemann(const St7<real>& wl, const St7<real>& wr, real bn,
                                       real gamma, real igm1, real* f, real* fm,
                                       real* sp) {
  // max(c_fL, c_fR) as the square root of the larger square: a square root
  // is monotone, so this is the same value with one square root fewer
  real cmax = sq(vmax(fast_speed_sq(wl.v[0], wl.v[4], bn, wl.v[5], wl.v[6], gamma),
                      fast_speed_sq(wr.v[0], wr.v[4], bn, wr.v[5], wr.v[6], gamma)));
  real umin = vmin(wl.v[1], wr.v[1]);
  real umax = vmax(wl.v[1], wr.v[1]);
  real sl = umin - cmax;
  real sr = umax + cmax;
  int used = 0;
  if (RS == 1) {
    hll_flux(wl, wr, bn, igm1, sl, sr, f);
  } else if (sl > (real)0 || sr < (real)0) {
    // supersonic: physical flux of the upwind state
    St7<real> w;
    const bool left = sl > (real)0;
#pragma unroll
    for (int v = 0; v < 7; v++) w.v[v] = sel(left, wl.v[v], wr.v[v]);
    real u[7];
    phys_flux(w, bn, igm1, f, u);
  } else {
    real ptl = wl.v[4] + (real)0.5 * (bn * bn + wl.v[5] * wl.v[5] + wl.v[6] * wl.v[6]);
    real ptr = wr.v[4] + (real)0.5 * (bn * bn + wr.v[5] * wr.v[5] + wr.v[6] * wr.v[6]);
    real sdl = sl - wl.v[1];
    real sdr = sr - wr.v[1];
    real iden = rcp(sdr * wr.v[0] - sdl * wl.v[0]);
    // S_M with p_T,R - p_T,L formed from the differences of the states
    const real dpt = (wr.v[4] - wl.v[4]) +
                     (real)0.5 * ((wr.v[5] - wl.v[5]) * (wr.v[5] + wl.v[5]) +
                                  (wr.v[6] - wl.v[6]) * (wr.v[6] + wl.v[6]));
    real sm = (sdr * wr.v[0] * wr.v[1] - sdl * wl.v[0] * wl.v[1] - dpt) * iden;
    real pts = (sdr * wr.v[0] * ptl - sdl * wl.v[0] * ptr +
                wl.v[0] * wr.v[0] * sdr * sdl * (wr.v[1] - wl.v[1])) *
               iden;
    bool ok = (sl < sm) && (sm < sr) && (pts > (real)0);
    if (ok) {
      const real enl = energy(wl, bn, igm1);
      const real enr = energy(wr, bn, igm1);
      StarD<real> stl, str;
      const bool posl = star_side(wl, enl, ptl, sl, sm, pts, bn, gamma, stl);
      const bool posr = star_side(wr, enr, ptr, sr, sm, pts, bn, gamma, str);
      if (!posl || !posr) ok = false;
      if (ok) {
        // side of the contact holding x/t = 0
        const bool left = sm > (real)0;
        St7<real> w;
#pragma unroll
        for (int v = 0; v < 7; v++) w.v[v] = sel(left, wl.v[v], wr.v[v]);
        StarD<real> sa;
        sa.drho = sel(left, stl.drho, str.drho);
        sa.dv1 = sel(left, stl.dv1, str.dv1);
        sa.dv2 = sel(left, stl.dv2, str.dv2);
        sa.db1 = sel(left, stl.db1, str.db1);
        sa.db2 = sel(left, stl.db2, str.db2);
        sa.den = sel(left, stl.den, str.den);
        // star values of the selected side: its state plus its jumps
        const real rhos = w.v[0] + sa.drho;
        const real v1s = w.v[2] + sa.dv1, v2s = w.v[3] + sa.dv2;
        const real b1s = w.v[5] + sa.db1, b2s = w.v[6] + sa.db2;
        const real s_out = sel(left, sl, sr);
        real fa[7], ua[7];
        // the side's total energy and pressure as already formed above
        phys_flux_ep(w, bn, sel(left, enl, enr), sel(left, ptl, ptr), fa, ua);
        // U* - U of the selected side
        real dus[7];
        dus[0] = sa.drho;
        dus[1] = sa.drho * sm + w.v[0] * (sm - w.v[1]);
        dus[2] = w.v[0] * sa.dv1 + sa.drho * v1s;
        dus[3] = w.v[0] * sa.dv2 + sa.drho * v2s;
        dus[4] = sa.den;
        dus[5] = sa.db1;
        dus[6] = sa.db2;
        real fs[7];
#pragma unroll
        for (int c = 0; c < 7; c++) fs[c] = fa[c] + s_out * dus[c];
        if ((real)0.5 * bn * bn <= Eps<real>::bsmall * pts) {
          // B_n ~ 0: the rotational waves merge with the contact
#pragma unroll
          for (int c = 0; c < 7; c++) f[c] = fs[c];
        } else {
          real sql = sq(wl.v[0] + stl.drho), sqr = sq(wr.v[0] + str.drho);
          real ssl = sm - quot(ab(bn), sql);
          real ssr = sm + quot(ab(bn), sqr);
          real sgn = bn > (real)0 ? (real)1 : (real)-1;
          real iss = rcp(sql + sqr);
          // jumps of the single-star states across the contact
          const real jv1 = (wr.v[2] - wl.v[2]) + (str.dv1 - stl.dv1);
          const real jv2 = (wr.v[3] - wl.v[3]) + (str.dv2 - stl.dv2);
          const real jb1 = (wr.v[5] - wl.v[5]) + (str.db1 - stl.db1);
          const real jb2 = (wr.v[6] - wl.v[6]) + (str.db2 - stl.db2);
          // double-star minus single-star values of the selected side:
          // v** - v*_L = [r_R jv + jb s]/(r_L + r_R), v** - v*_R = [-r_L jv + jb s]/(..);
          // B** - B*_L = [r_L jb + r_L r_R jv s]/(..), B** - B*_R = [-r_R jb + r_L r_R jv s]/(..)
          const real sgv = sel(left, (real)1, (real)-1);
          const real r_oth = sel(left, sqr, sql);
          const real r_own = sel(left, sql, sqr);
          const real dv1 = (sgv * r_oth * jv1 + jb1 * sgn) * iss;
          const real dv2 = (sgv * r_oth * jv2 + jb2 * sgn) * iss;
          const real db1 = (sgv * r_own * jb1 + sql * sqr * jv1 * sgn) * iss;
          const real db2 = (sgv * r_own * jb2 + sql * sqr * jv2 * sgn) * iss;
          // E** - E* = -+ sqrt(rho*) (v*.B* - v**.B**) sign(B_n), with
          // v*.B* - v**.B** = -(v*_t.dB + dv.B**_t)
          real t = r_own * (v1s * db1 + v2s * db2 + dv1 * (b1s + db1) + dv2 * (b2s + db2)) * sgn;
          t = sel(left, t, -t);
          // rotational wave of the selected side, and whether x/t = 0 lies
          // between it and the contact
          const real s_rot = sel(left, ssl, ssr);
          const bool inner = left ? !(ssl > (real)0) : !(ssr < (real)0);
          real duss[7];
          duss[0] = (real)0;
          duss[1] = (real)0;
          duss[2] = rhos * dv1;
          duss[3] = rhos * dv2;
          duss[4] = t;
          duss[5] = db1;
          duss[6] = db2;
#pragma unroll
          for (int c = 0; c < 7; c++) {
            const real fss = fs[c] + s_rot * duss[c];
            f[c] = inner ? fss : fs[c];
          }
        }
#pragma unroll
        for (int c = 0; c < 7; c++)
          if (!finite(f[c])) ok = false;
      }
    }
    if (!ok) {
      used = 1;
      hll_flux(wl, wr, bn, igm1, sl, sr, f);
    }
  }
  real thr = Eps<real>::mflux * (wl.v[0] + wr.v[0]) * (ab(sl) + ab(sr));
  *fm = ab(f[0]) <= thr ? (real)0 : f[0];
  sp[0] = sl;
  sp[1] = sr;
  return used;
}

// PLM on the seven face-frame variables of a four-cell stencil
template <int LIM, typename real>
__device__ __forceinline__ void plm_face(const St7<real>& q0, const St7<real>& q1,
                                         const St7<real>& q2, const St7<real>& q3,
                                         St7<real>& wl, St7<real>& wr) {
#pragma unroll
  for (int v = 0; v < 7; v++) plm<real, LIM>(q0.v[v], q1.v[v], q2.v[v], q3.v[v], wl.v[v], wr.v[v]);
}

__device__ __forceinline__ void count(unsigned long long* c, int fl) {
  if (fl & 1) atomicAdd(&c[0], 1ull);
  if (fl & 2) atomicAdd(&c[2], 1ull);
}

// CFL rate of a cell: max over active axes of (|v_d| + c_f,d) / dx_d
// (the box type B is a device box descriptor or a FlatBox kernel argument)
template <typename B>
__device__ __forceinline__ double cfl_rate(B& b, const PrimD& w) {
  const double v[3] = {w.vx, w.vy, w.vz};
  const double bc[3] = {w.bx, w.by, w.bz};
  double l = 0.0;
#pragma unroll
  for (int d = 0; d < 3; d++) {
    if (!b.act[d]) continue;
    const double cf = fast_speed(w.r, w.p, bc[d], bc[(d + 1) % 3], bc[(d + 2) % 3], b.gamma);
    const double x = (__builtin_fabs(v[d]) + cf) * b.idx[d];
    if (x > l) l = x;
  }
  return l;
}

// upwind choice of the CT average: flux > 0 -> lower side, < 0 -> upper,
// 0 -> mean
template <typename real>
__device__ __forceinline__ real upwind(real m, real lower, real upper) {
  if (m > (real)0) return lower;
  if (m < (real)0) return upper;
  return (real)0.5 * (lower + upper);
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    double w = __shfl_xor(v, o, 64);
    v = w > v ? w : v;
  }
  return v;
}

// block-wide max: wavefront butterfly, then across the TPB / 64 wavefronts
template <int TPB = kTPB>
__device__ __forceinline__ double block_max(double v) {
  __shared__ double part[TPB / 64];
  v = wave_max(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) part[wid] = v;
  __syncthreads();
  double m = part[0];
#pragma unroll
  for (int w = 1; w < TPB / 64; w++) m = part[w] > m ? part[w] : m;
  __syncthreads();
  return m;
}

// ---------------------------------------------------------------- kernels

// x-sweep tile: xft consecutive faces of the box's x faces numbered row by
// row (row = j + ny*k, face f, number row*nf + f).  The faces of one row
// within the tile form a piece; piece p is staged in LDS as its cells from
// two before its first face to one after its last (width + 3 slots), the
// pieces one after another.  A tile of 256 faces touches at most
// 2 + 255/nf rows, and the host keeps 256 + 3 pieces within the LDS capacity
// (for rows of fewer than 13 faces, where it cannot, a tile is whole rows),
// so every lane has a face in every tile but the box's last.
struct XTile {
  int nf, ny;
  int nF;          // faces in this tile
  int row0, fa;    // row and face of the tile's first face
  int W0;          // faces of the first piece
  int j0, k0;      // (j, k) of row0
};

__device__ __forceinline__ XTile x_tile(CBox& b, int lt) {
  XTile x;
  x.nf = b.nf[0];
  x.ny = b.n[1];
  const int F0 = lt * b.xft;
  x.nF = min(b.xft, b.n[1] * b.n[2] * x.nf - F0);
  x.row0 = F0 / x.nf;
  x.fa = F0 - x.row0 * x.nf;
  x.W0 = min(x.nf - x.fa, x.nF);
  x.j0 = x.row0 % x.ny;
  x.k0 = x.row0 / x.ny;
  return x;
}

// (j, k) of the tile's piece p
__device__ __forceinline__ void x_row(const XTile& x, int p, int& j, int& k) {
  j = x.j0;
  k = x.k0;
  if (p) {
    const int jj = x.j0 + p;
    k += jj / x.ny;
    j = jj - (jj / x.ny) * x.ny;
  }
}

// Staging slot s: piece p, cell index i in the row, offset c of the slot in
// its piece and the piece's face count w; the tile owns the cell when its
// index is one of the piece's faces (2 <= c < w + 2).
__device__ __forceinline__ void x_slot(const XTile& x, int s, int& p, int& i, int& c, int& w) {
  if (s < x.W0 + 3) {
    p = 0;
    c = s;
    w = x.W0;
    i = x.fa - 2 + c;
  } else {
    const int s2 = s - (x.W0 + 3);
    p = 1 + s2 / (x.nf + 3);
    c = s2 - (p - 1) * (x.nf + 3);
    w = min(x.nf, x.nF - x.W0 - (p - 1) * x.nf);
    i = c - 2;
  }
}

// Face t of the tile: piece p, face f in the row, and the slot o of the
// first of its four stencil cells (cells f-2 .. f+1).
__device__ __forceinline__ void x_face(const XTile& x, int t, int& p, int& f, int& o) {
  if (t < x.W0) {
    p = 0;
    f = x.fa + t;
    o = t;
  } else {
    const int t2 = t - x.W0;
    p = 1 + t2 / x.nf;
    f = t2 - (p - 1) * x.nf;
    o = x.W0 + 3 + (p - 1) * (x.nf + 3) + f;
  }
}

// x sweep: tiles of consecutive x faces staged in LDS; one x face per lane.
// Writes the hydro flux, the face EMFs (E_y, E_z), the CT mass flux and the
// cell EMF of every owned cell; with L.lam also the tile's max CFL rate
// (stage 1, the state at the start of the step).
// WPE: minimum resident wavefronts per SIMD the register allocation must
// allow (1 = unconstrained); one of the tunable launch variants.  RS: the
// Riemann solver (see riemann).  SL: slope kind, REC = SL & 1 and limiter
// LIM = SL >> 1 (see limit); REC = 1: slopes limited in characteristic
// fields (char_slope), computed once per staged cell into LDS rows 8-14
// after the staging pass (row 7 holds the cell's normal field).
template <typename real, int WPE, int RS, int SL>
__global__ __launch_bounds__(kTPB) __attribute__((amdgpu_waves_per_eu(WPE))) void k_sweep_x(
    Launch L) {
  constexpr int REC = SL & 1, LIM = SL >> 1;
  __shared__ real sw[REC ? 15 : 7][kLdsCells];
  const int s = L.stage;
  for (int v = blockIdx.x; v < tile_slots(L); v += gridDim.x) {
    const int tile = tile_of(L, v);
    if (tile >= L.ntiles) continue;
    const int bi = find_box(table(L.base) + kXS * (L.nboxes + 1), L.nboxes, tile);
    CBox& b = box_at(L.boxes, bi);
    const int lt = tile - table(L.base)[kXS * (L.nboxes + 1) + bi];
    const int nx = b.n[0];
    const XTile x = x_tile(b, lt);
    double lmax = 0.0;
    if (b.act[0]) {
      // the normal field of the lane's face (a tile has at most one face
      // per lane), loaded before the staging so that it has arrived when
      // the face is solved
      real bn_lane = (real)0;
      if ((int)threadIdx.x < x.nF) {
        int p, f, o, j, k;
        x_face(x, threadIdx.x, p, f, o);
        x_row(x, p, j, k);
        bn_lane = (real)ld<double>(b.B[s][0], fidx(b, 0, f, j, k));
      }
      const int npieces = 1 + (x.nF - x.W0 + x.nf - 1) / x.nf;
      const int ncell = x.nF + 3 * npieces;
      for (int sidx = threadIdx.x; sidx < ncell; sidx += kTPB) {
        int p, i, c, wd, j, k;
        x_slot(x, sidx, p, i, c, wd);
        const bool own = c >= 2 && c < wd + 2;
        x_row(x, p, j, k);
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
        if constexpr (REC) sw[7][sidx] = (real)w.bx;
        if (own && i >= 0 && i < nx) {
          const int c = cidx(b, i, j, k);
          st<real>(b.Ec[0], c, (real)(w.vz * w.by - w.vy * w.bz));
          st<real>(b.Ec[1], c, (real)(w.vx * w.bz - w.vz * w.bx));
          st<real>(b.Ec[2], c, (real)(w.vy * w.bx - w.vx * w.by));
          if (b.emf == 3) {
            st<real>(b.V[0], c, (real)w.vx);
            st<real>(b.V[1], c, (real)w.vy);
            st<real>(b.V[2], c, (real)w.vz);
          }
          if (fl) count(b.cnt, fl);
          if (L.lam) {
            const double l = cfl_rate(b, w);
            if (l > lmax) lmax = l;
          }
        }
      }
      __syncthreads();
      if constexpr (REC) {
        // slope of every cell next to a face of the tile (offsets 1..w+1
        // of its piece), from its two neighbours in the same piece
        for (int sidx = threadIdx.x; sidx < ncell; sidx += kTPB) {
          int p, i, c, wd;
          x_slot(x, sidx, p, i, c, wd);
          if (c >= 1 && c <= wd + 1) {
            St7<real> qm, q0, qp;
#pragma unroll
            for (int v = 0; v < 7; v++) {
              qm.v[v] = sw[v][sidx - 1];
              q0.v[v] = sw[v][sidx];
              qp.v[v] = sw[v][sidx + 1];
            }
            const St7<real> d = char_slope<LIM>(qm, q0, qp, sw[7][sidx], (real)b.gamma);
#pragma unroll
            for (int v = 0; v < 7; v++) sw[8 + v][sidx] = d.v[v];
          }
        }
        __syncthreads();
      }
      for (int t = threadIdx.x; t < x.nF; t += kTPB) {
        int p, f, o, j, k;
        x_face(x, t, p, f, o);
        x_row(x, p, j, k);
        St7<real> wl, wr;
        if constexpr (REC) {
#pragma unroll
          for (int v = 0; v < 7; v++) {
            wl.v[v] = sw[v][o + 1] + (real)0.5 * sw[8 + v][o + 1];
            wr.v[v] = sw[v][o + 2] - (real)0.5 * sw[8 + v][o + 2];
          }
        } else {
          St7<real> q[4];
#pragma unroll
          for (int m = 0; m < 4; m++)
#pragma unroll
            for (int v = 0; v < 7; v++) q[m].v[v] = sw[v][o + m];
          plm_face<LIM>(q[0], q[1], q[2], q[3], wl, wr);
        }
        const int fi = fidx(b, 0, f, j, k);
        const real bn = t == (int)threadIdx.x ? bn_lane : (real)ld<double>(b.B[s][0], fi);
        real F[7], fm, sp[2];
        const int used = riemann<real, RS>(wl, wr, bn, (real)b.gamma, (real)b.igm1, F, &fm, sp);
        if (b.emf == 3) {
          st<real>(b.SP[0][0], fi, sp[0]);
          st<real>(b.SP[0][1], fi, sp[1]);
        }
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
    } else {
      // inactive x: the face carries the cell's physical flux (no divergence)
      for (int t = threadIdx.x; t < x.nF; t += kTPB) {
        int p, f, o, j, k;
        x_face(x, t, p, f, o);
        x_row(x, p, j, k);
        const int im = map_cell(f, nx, b.per[0]);
        PrimD w;
        const int fl = load_prim(b, s, im, j, k, w);
        const double ecy = w.vx * w.bz - w.vz * w.bx;
        const double ecz = w.vy * w.bx - w.vx * w.by;
        const int fi = fidx(b, 0, f, j, k);
        st<real>(b.EF[0][0], fi, (real)ecy);
        st<real>(b.EF[0][1], fi, (real)ecz);
        st<real>(b.MF[0], fi, (real)ld<double>(b.U[s][1], cidx(b, im, j, k)));
        if (f == 0) {
          const int c = cidx(b, 0, j, k);
          st<real>(b.Ec[0], c, (real)(w.vz * w.by - w.vy * w.bz));
          st<real>(b.Ec[1], c, (real)ecy);
          st<real>(b.Ec[2], c, (real)ecz);
          if (b.emf == 3) {
            st<real>(b.V[0], c, (real)w.vx);
            st<real>(b.V[1], c, (real)w.vy);
            st<real>(b.V[2], c, (real)w.vz);
          }
          if (fl) count(b.cnt, fl);
          if (L.lam) {
            const double l = cfl_rate(b, w);
            if (l > lmax) lmax = l;
          }
        }
      }
    }
    if (L.lam) {
      const double m = block_max(lmax);
      if (threadIdx.x == 0) b.lam[lt] = m;
    } else {
      __syncthreads();  // the next tile reuses the LDS
    }
  }
}

// Stage combine of the strong-stability-preserving Runge-Kutta schemes
// (Shu & Osher 1988): uold is the state at the start of the step, usw the
// state the stage swept, dtl = dt times its residual.
//   0: first stage            usw + dtl
//   1: RK2 second stage       1/2 (uold + (usw + dtl))
//   2: RK3 second stage       3/4 uold + 1/4 (usw + dtl)
//   3: RK3 third stage        1/3 uold + 2/3 (usw + dtl)
// (the RK3 weights are the doubles nearest 3/4, 1/4, 1/3, 2/3; FP64 results
// are identical to the oracle's).
__device__ __forceinline__ double rk_combine(int kind, double uold, double usw, double dtl) {
  if (kind == 0) return usw + dtl;
  if (kind == 1) return 0.5 * (uold + (usw + dtl));
  if (kind == 2) return 0.75 * uold + 0.25 * (usw + dtl);
  return (1.0 / 3.0) * uold + (2.0 / 3.0) * (usw + dtl);
}

// Marching sweep along axis D (1 = y, 2 = z).  Each lane owns one column of
// cells along D (lanes run along x) and slides a register window (two cells,
// the limited slope of the older one and the incoming cell) down its
// segment; one Riemann solve per face; the raw data of the cell two faces
// ahead is loaded before the current face is solved.  Y: adds the x
// and y flux divergence and writes the residual.  Z: adds the z divergence
// to the residual and applies the SSP-RK2 stage combine.
// Window of the march: cells f-1 and f and the limited slope of cell f-1.
// LW = 0 keeps it in registers; LW = 1 keeps it in a per-lane LDS column
// (three slots of seven values, no sharing between lanes, so no barrier):
// fewer registers live across the Riemann solve.
// Register window (LW = 0) for any slope kind SL (REC = SL & 1, LIM =
// SL >> 1): with REC = 1 the slopes are limited in characteristic fields
// and the window also keeps the normal field of its newer cell, whose
// slope the next face computes.  The LDS window (LW = 1) serves SL = 0.
template <typename real, int LW, int SL>
struct Window;

template <typename real, int SL>
struct Window<real, 0, SL> {
  static constexpr int REC = SL & 1, LIM = SL >> 1;
  St7<real> q1, q2, dm1;
  real bn2;
  __device__ __forceinline__ void init(const St7<real>& a, const St7<real>& b, const St7<real>& d,
                                       real bnb) {
    q1 = a;
    q2 = b;
    dm1 = d;
    bn2 = bnb;
  }
  // PLM states of the face between the window's cells given the next cell
  // q3 (normal field bn3); then slides the window by one cell
  __device__ __forceinline__ void face_and_slide(const St7<real>& q3, real bn3, real gamma,
                                                 St7<real>& wl, St7<real>& wr) {
    if constexpr (REC) {
      const St7<real> d0 = char_slope<LIM>(q1, q2, q3, bn2, gamma);
#pragma unroll
      for (int v = 0; v < 7; v++) {
        wl.v[v] = q1.v[v] + (real)0.5 * dm1.v[v];
        wr.v[v] = q2.v[v] - (real)0.5 * d0.v[v];
      }
      dm1 = d0;
      bn2 = bn3;
    } else {
#pragma unroll
      for (int v = 0; v < 7; v++) {
        const real d0 = limit<LIM>(q2.v[v] - q1.v[v], q3.v[v] - q2.v[v]);
        wl.v[v] = q1.v[v] + (real)0.5 * dm1.v[v];
        wr.v[v] = q2.v[v] - (real)0.5 * d0;
        dm1.v[v] = d0;
      }
    }
    q1 = q2;
    q2 = q3;
  }
};

template <typename real>
struct Window<real, 1, 0> {
  real (*lds)[kTPB];  // [21][kTPB]: slots 0-6 and 7-13 cells, 14-20 slope
  int t, a;           // lane, offset of the slot holding cell f-1
  __device__ __forceinline__ void init(const St7<real>& q1, const St7<real>& q2, const St7<real>& d,
                                       real) {
    a = 0;
#pragma unroll
    for (int v = 0; v < 7; v++) {
      lds[v][t] = q1.v[v];
      lds[7 + v][t] = q2.v[v];
      lds[14 + v][t] = d.v[v];
    }
  }
  __device__ __forceinline__ void face_and_slide(const St7<real>& q3, real, real, St7<real>& wl,
                                                 St7<real>& wr) {
    const int bo = 7 - a;
#pragma unroll
    for (int v = 0; v < 7; v++) {
      const real x1 = lds[a + v][t];
      const real x2 = lds[bo + v][t];
      const real dm = lds[14 + v][t];
      const real d0 = minmod(x2 - x1, q3.v[v] - x2);
      wl.v[v] = x1 + (real)0.5 * dm;
      wr.v[v] = x2 - (real)0.5 * d0;
      lds[a + v][t] = q3.v[v];  // cell f+1 takes the slot of cell f-1
      lds[14 + v][t] = d0;
    }
    a = bo;
  }
};

// CU (z march only): the swept state of the last three cells loaded is kept
// in a per-lane LDS ring (no sharing between lanes, so no barrier).  It is
// the state the RK combine reads (U^n in stage 1, U* in stage 2), three
// faces after the sweep loaded it, when it has usually left L2; the ring
// saves that second fetch.
template <typename real, int D, int PF, int LW, int CU, int RS, int FZ, int SL>
__device__ __forceinline__ void march_column(CBox& b, int s, int dst, int comb, int i, int tr,
                                             int j0, int j1, real (*lds)[kTPB],
                                             double (*ring)[kTPB]) {
  constexpr bool kRing = CU && D == 2;
  const int lane = threadIdx.x;
  // (i, tr): x index and the index along the remaining axis (z for D=1, y
  // for D=2); cells [j0, j1) along D, faces j0..j1
  const int n = b.n[D];
  const int per = b.per[D];
  auto addr_at = [&](int a) {
    const int am = map_cell(a, n, per);
    return D == 1 ? addr_of(b, i, am, tr) : addr_of(b, i, tr, am);
  };
  constexpr int REC = SL & 1, LIM = SL >> 1;
  Window<real, LW, SL> win;
  const real gam = (real)b.gamma;
  // cell-centred normal field of a primitive state (characteristic slopes)
  auto bnorm = [&](const PrimD& w) { return (real)(D == 1 ? w.by : w.bz); };
  if constexpr (LW) {
    win.lds = lds;
    win.t = threadIdx.x;
  }
  {
    PrimD w;
    raw_to_prim(b, load_raw(b, s, addr_at(j0 - 2)), w);
    const St7<real> q0 = rotate<real>(w, D);
    raw_to_prim(b, load_raw(b, s, addr_at(j0 - 1)), w);
    const St7<real> q1 = rotate<real>(w, D);
    const real bn1 = bnorm(w);
    const Raw r2 = load_raw(b, s, addr_at(j0));
    raw_to_prim(b, r2, w);
    const St7<real> q2 = rotate<real>(w, D);
    const real bn2 = bnorm(w);
    if constexpr (kRing) {
      const int slot = j0 % 3;
#pragma unroll
      for (int q = 0; q < kNQ; q++) ring[slot * kNQ + q][lane] = r2.u[q];
    }
    St7<real> dm1;
    if constexpr (REC) {
      dm1 = char_slope<LIM>(q0, q1, q2, bn1, gam);
    } else {
#pragma unroll
      for (int v = 0; v < 7; v++) dm1.v[v] = limit<LIM>(q1.v[v] - q0.v[v], q2.v[v] - q1.v[v]);
    }
    win.init(q1, q2, dm1, bn2);
  }
  Raw next = load_raw(b, s, addr_at(j0 + 1));
  real fprev[kNQ];
  const bool extra = (j1 == n) && (b.nf[D] == n + 1);
  // face offsets along D: face f of this column
  const int fstride = D == 1 ? b.n[0] : b.n[0] * b.n[1];
  const int fbase = D == 1 ? (tr * b.nf[1]) * b.n[0] + i : tr * b.n[0] + i;
  // face f along D is in [0, n]; periodic face n is face 0
  auto face_at = [&](int f) { return fbase + ((per && f == n) ? 0 : f) * fstride; };
  const int cstride = fstride;
  const int cbase = D == 1 ? (tr * b.n[1]) * b.n[0] + i : tr * b.n[0] + i;
  constexpr bool kFin = D == 2 || FZ;  // this march applies the RK combine
  const double dt = kFin ? b.scal[0] : 0.0;
  int cw = (j0 + 1) % 3;  // ring slot of cell f+1 at face f
  for (int f = j0; f <= j1; ++f) {
    // the face's normal field first: a load completes only after every
    // earlier one, so loaded after the next cell's prefetch its solve would
    // wait for that prefetch too
    const real bn = (real)ld<double>(b.B[s][D], face_at(f));
    PrimD w;
    raw_to_prim(b, next, w);
    const St7<real> q3 = rotate<real>(w, D);
    if constexpr (kRing) {
#pragma unroll
      for (int q = 0; q < kNQ; q++) ring[cw * kNQ + q][lane] = next.u[q];
    }
    if (f < j1) next = load_raw(b, s, addr_at(f + 2));
    // inputs of the cell update: issued before the solve (PF) or after it
    const int cprev = cbase + (f - 1) * cstride;
    double racc[kNQ];
    double usw[kNQ], uold[kNQ];  // swept state of cell f-1; U^n in stage 2
    auto load_update_inputs = [&]() {
      if (D == 1) {
        const int f0 = (tr * b.n[1] + (f - 1)) * b.nf[0] + i;
        const int f1 = (b.per[0] && i + 1 == b.n[0]) ? f0 - i : f0 + 1;
#pragma unroll
        for (int q = 0; q < kNQ; q++) {
          double r = 0.0;
          if (b.act[0])
            r = r - ((double)ld<real>(b.FX[q], f1) - (double)ld<real>(b.FX[q], f0)) * b.idx[0];
          racc[q] = r;
          if constexpr (FZ) {
            usw[q] = ld<double>(b.U[s][q], cprev);
            uold[q] = comb ? ld<double>(b.U[0][q], cprev) : 0.0;
          }
        }
      } else {
        const int cr = cw == 2 ? 0 : cw + 1;  // ring slot of cell f-1
#pragma unroll
        for (int q = 0; q < kNQ; q++) {
          racc[q] = (double)ld<real>(b.R[q], cprev);
          if constexpr (kRing)
            usw[q] = ring[cr * kNQ + q][lane];
          else
            usw[q] = ld<double>(b.U[s][q], cprev);
          uold[q] = comb ? ld<double>(b.U[0][q], cprev) : 0.0;
        }
      }
    };
    if (PF && f > j0) load_update_inputs();
    St7<real> wl, wr;
    win.face_and_slide(q3, bnorm(w), gam, wl, wr);
    const int fi = face_at(f);
    real F[7], fm, sp[2];
    const int used = riemann<real, RS>(wl, wr, bn, (real)b.gamma, (real)b.igm1, F, &fm, sp);
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
      if (b.emf == 3) {
        st<real>(b.SP[D][0], fi, sp[0]);
        st<real>(b.SP[D][1], fi, sp[1]);
      }
      if (used) atomicAdd(&b.cnt[1], 1ull);
    }
    if (f > j0) {
      // cell f-1 is complete
      if (!PF) load_update_inputs();
      const double idxD = b.idx[D];
#pragma unroll
      for (int q = 0; q < kNQ; q++) {
        const double r = racc[q] - ((double)fl[q] - (double)fprev[q]) * idxD;
        if (kFin)
          st<double>(b.U[dst][q], cprev, rk_combine(comb, uold[q], usw[q], dt * r));
        else
          st<real>(b.R[q], cprev, (real)r);
      }
      if constexpr (FZ) {
        // z faces of the cell (one cell along z: no z flux divergence): the
        // face EMFs are the cell EMF and the mass flux is the momentum
        const real ex = ld<real>(b.Ec[0], cprev), ey = ld<real>(b.Ec[1], cprev);
        const real mz = (real)ld<double>(b.U[s][3], cprev);
        const int nxy = b.n[0] * b.n[1];
        for (int kf = 0; kf < b.nf[2]; ++kf) {
          const int fz = kf * nxy + (f - 1) * b.n[0] + i;
          st<real>(b.EF[2][0], fz, ex);
          st<real>(b.EF[2][1], fz, ey);
          st<real>(b.MF[2], fz, mz);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < kNQ; q++) fprev[q] = fl[q];
    cw = cw == 2 ? 0 : cw + 1;
  }
}

// ---------------------------------------------------------------- fused x+y march
//
// The y march with the x faces of its own rows computed in the same kernel:
// the lanes of a workgroup hold consecutive columns (i, k) of the box, so
// at every step of the march the row of cells they load is also a row
// segment along x.  Each lane writes the x-frame primitives of the cell it
// loads into a three-row LDS ring; two steps later, when that row's cells
// are completed, every lane computes the x face below its cell from the
// four cells i-2..i+1 of the ring (cells beyond the workgroup's piece of
// the row are loaded directly), the x-face fluxes are exchanged through LDS
// (the face above a cell is its right neighbour's face below, or computed
// by the last lane of a piece), and the x and y flux differences complete
// the cell's residual together.  The x sweep, its second read of the state
// and the x-face hydro flux array it hands to the y march are then not
// needed; the march also writes what the x sweep wrote for the corner EMFs
// (cell EMF, x-face EMFs and mass flux), counts floor hits and non-physical
// cells and, in the first stage, reduces the CFL rate of its cells.  Every
// x-face flux is the same function of the same values as in the x sweep.
// Used for boxes whose three axes are active, with primitive slopes.
template <typename real, int TPB>
struct XRing {
  real q[3][7][TPB];     // x-frame primitives of three rows, per lane
  real f[2][kNQ][TPB];   // x-face hydro fluxes of the row being completed,
                         // alternating between two buffers row by row
};

// x-frame primitives of cell (i, j, k) of state s
template <typename real>
__device__ __forceinline__ St7<real> xprim_of(CBox& b, int s, int i, int j, int k) {
  PrimD w;
  load_prim(b, s, map_cell(i, b.n[0], b.per[0]), j, k, w);
  return rotate<real>(w, 0);
}

// the x-frame primitives of the cell at x offset d from lane t's column
// (i, row j, k): from the ring when that cell's column belongs to a live
// lane of this workgroup in the same row, else loaded
template <typename real, int TPB>
__device__ __forceinline__ St7<real> xneighbour(CBox& b, int s, XRing<real, TPB>& xr, int slot,
                                                int t, int col, int ncols, int i, int j, int k,
                                                int d) {
  const int ii = map_cell(i + d, b.n[0], b.per[0]);
  const int tt = t + (ii - i);
  St7<real> q;
  if (tt >= 0 && tt < TPB && col + (ii - i) < ncols) {
#pragma unroll
    for (int v = 0; v < 7; v++) q.v[v] = xr.q[slot][v][tt];
  } else {
    q = xprim_of<real>(b, s, ii, j, k);
  }
  return q;
}

// x-face index of the lower face of cell (i + d) of row (j, k): face i + d
// (face n of an outflow axis; periodic face n is face 0)
__device__ __forceinline__ int xface_idx(CBox& b, int i, int j, int k, int d) {
  const int f = i + d;
  return fidx(b, 0, (b.per[0] && f == b.n[0]) ? 0 : f, j, k);
}

// x-face flux at the lower face of cell (i + d) of row (j, k) from its four
// stencil cells and the face's normal field bn; writes the face data the
// corner EMFs read when `store`
template <typename real, int RS, int TPB>
__device__ __forceinline__ void xface(CBox& b, XRing<real, TPB>& xr, int s, int slot, int t,
                                      int col, int ncols, int i, int j, int k, int d, real bn,
                                      bool store, real* fl, int* used) {
  St7<real> q[4], wl, wr;
#pragma unroll
  for (int m = 0; m < 4; m++)
    q[m] = xneighbour<real, TPB>(b, s, xr, slot, t, col, ncols, i, j, k, d + m - 2);
  plm_face<0>(q[0], q[1], q[2], q[3], wl, wr);
  const int fi = xface_idx(b, i, j, k, d);
  real F[7], fm, sp[2];
  *used = riemann<real, RS>(wl, wr, bn, (real)b.gamma, (real)b.igm1, F, &fm, sp);
#pragma unroll
  for (int q2 = 0; q2 < kNQ; q2++) fl[q2] = F[q2];
  if (store) {
    st<real>(b.EF[0][0], fi, F[6]);
    st<real>(b.EF[0][1], fi, -F[5]);
    st<real>(b.MF[0], fi, fm);
  }
}

template <typename real, int LW, int RS, int TPB>
__device__ __forceinline__ void march_column_xy(CBox& b, int s, int i, int tr, int col, int ncols,
                                                bool live, int j0, int j1, real (*lds)[kTPB],
                                                XRing<real, TPB>& xr, int lam, double& lmax) {
  const int t = threadIdx.x;
  const int n = b.n[1];
  const int per = b.per[1];
  auto addr_at = [&](int a) { return addr_of(b, i, map_cell(a, n, per), tr); };
  // an own cell of the march: its x-frame primitives into the ring; the
  // x sweep's per-cell work (cell EMF, counters, CFL rate)
  auto own_cell = [&](int j, const PrimD& w, int fl) {
    const St7<real> qx = rotate<real>(w, 0);
#pragma unroll
    for (int v = 0; v < 7; v++) xr.q[j % 3][v][t] = qx.v[v];
    if (live) {
      const int c = cidx(b, i, j, tr);
      st<real>(b.Ec[0], c, (real)(w.vz * w.by - w.vy * w.bz));
      st<real>(b.Ec[1], c, (real)(w.vx * w.bz - w.vz * w.bx));
      st<real>(b.Ec[2], c, (real)(w.vy * w.bx - w.vx * w.by));
      if (fl) count(b.cnt, fl);
      if (lam) {
        const double l = cfl_rate(b, w);
        if (l > lmax) lmax = l;
      }
    }
  };
  Window<real, LW, 0> win;
  if constexpr (LW) {
    win.lds = lds;
    win.t = t;
  }
  {
    PrimD w;
    raw_to_prim(b, load_raw(b, s, addr_at(j0 - 2)), w);
    const St7<real> q0 = rotate<real>(w, 1);
    raw_to_prim(b, load_raw(b, s, addr_at(j0 - 1)), w);
    const St7<real> q1 = rotate<real>(w, 1);
    const int fl = raw_to_prim(b, load_raw(b, s, addr_at(j0)), w);
    const St7<real> q2 = rotate<real>(w, 1);
    own_cell(j0, w, fl);
    St7<real> dm1;
#pragma unroll
    for (int v = 0; v < 7; v++) dm1.v[v] = limit<0>(q1.v[v] - q0.v[v], q2.v[v] - q1.v[v]);
    win.init(q1, q2, dm1, (real)w.by);
  }
  Raw next = load_raw(b, s, addr_at(j0 + 1));
  real fprev[kNQ];
  const bool extra = (j1 == n) && (b.nf[1] == n + 1);
  const int fstride = b.n[0];
  const int fbase = (tr * b.nf[1]) * b.n[0] + i;
  const int cbase = (tr * b.n[1]) * b.n[0] + i;
  // y face f in [0, n]; periodic face n is face 0
  auto face_at = [&](int f) { return fbase + ((per && f == n) ? 0 : f) * fstride; };
  // FP64: normal fields loaded ahead of their solves (a load completes only
  // after every load issued before it, so a field loaded just before its
  // solve waits for the next cell's prefetch): the y face one step ahead,
  // the x face of the row being completed first thing in its step.  In the
  // mixed path, whose waves wait less, the extra registers cost more than
  // the waits (measured), and the fields are loaded at their solves.
  constexpr bool kAhead = sizeof(real) == 8;
  real bny_cur = kAhead ? (real)ld<double>(b.B[s][1], face_at(j0)) : (real)0;
  // the lane that holds the face above this lane's cell: its right
  // neighbour in the same row piece, else this lane computes that face
  const int iu = map_cell(i + 1, b.n[0], b.per[0]);
  const bool up_in_ring = (i + 1 < b.n[0] || b.per[0]) && t + (iu - i) >= 0 &&
                          t + (iu - i) < TPB && col + (iu - i) < ncols;
  for (int f = j0; f <= j1; ++f) {
    const real bnx =
        kAhead && f > j0 ? (real)ld<double>(b.B[s][0], xface_idx(b, i, f - 1, tr, 0)) : (real)0;
    PrimD w;
    const int fl = raw_to_prim(b, next, w);
    const St7<real> q3 = rotate<real>(w, 1);
    // Ring slot (f + 1) % 3 was last read by the x faces of row f - 2 in
    // the previous step, before that step's flux-exchange barrier, which
    // also made the rows written since visible; the first two steps, with
    // no exchange behind them, wait here instead.
    if (f <= j0 + 1) __syncthreads();
    if (f + 1 < j1) own_cell(f + 1, w, fl);
    if (f < j1) next = load_raw(b, s, addr_at(f + 2));
    real bny_nxt = bny_cur;
    if (kAhead && f < j1) bny_nxt = (real)ld<double>(b.B[s][1], face_at(f + 1));
    St7<real> wl, wr;
    win.face_and_slide(q3, (real)w.by, (real)b.gamma, wl, wr);
    const int fi = face_at(f);
    const real bn = kAhead ? bny_cur : (real)ld<double>(b.B[s][1], fi);
    bny_cur = bny_nxt;
    real F[7], fm, sp[2];
    const int used = riemann<real, RS>(wl, wr, bn, (real)b.gamma, (real)b.igm1, F, &fm, sp);
    real fy[kNQ];
    fy[0] = F[0];
    fy[4] = F[4];
    fy[2] = F[1];
    fy[3] = F[2];
    fy[1] = F[3];
    if (live && (f < j1 || (f == n && extra))) {
      st<real>(b.EF[1][0], fi, F[6]);
      st<real>(b.EF[1][1], fi, -F[5]);
      st<real>(b.MF[1], fi, fm);
      if (used) atomicAdd(&b.cnt[1], 1ull);
    }
    if (f > j0) {
      // row f - 1 is complete along y: its x faces
      const int c = f - 1;
      const int slot = c % 3;
      real flo[kNQ], fup[kNQ];
      int ux = 0, uu = 0;
      const bool up_boundary = !b.per[0] && i + 1 == b.n[0];  // face n of an outflow axis
      // the face below the cell, then (lanes whose face above is not in the
      // ring) the face above: one call site, so one copy of the solver
#pragma unroll 1
      for (int d = 0; d < 2; d++) {
        if (d == 1 && up_in_ring) break;
        real fx[kNQ];
        int u = 0;
        const real bnd = kAhead && d == 0 ? bnx : (real)ld<double>(b.B[s][0], xface_idx(b, i, c, tr, d));
        xface<real, RS, TPB>(b, xr, s, slot, t, col, ncols, i, c, tr, d, bnd,
                             d == 0 ? live : (live && up_boundary), fx, &u);
#pragma unroll
        for (int q = 0; q < kNQ; q++) {
          if (d == 0) flo[q] = fx[q]; else fup[q] = fx[q];
        }
        if (d == 0) ux = u; else uu = u;
      }
      // flux exchange: a buffer is written again two rows later, after
      // the next row's barrier, which every reader of this row has passed
      const int fb = c & 1;
#pragma unroll
      for (int q = 0; q < kNQ; q++) xr.f[fb][q][t] = flo[q];
      __syncthreads();
      if (up_in_ring) {
#pragma unroll
        for (int q = 0; q < kNQ; q++) fup[q] = xr.f[fb][q][t + (iu - i)];
      }
      if (live) {
        if (ux) atomicAdd(&b.cnt[1], 1ull);
        if (uu && up_boundary) atomicAdd(&b.cnt[1], 1ull);
        const int cprev = cbase + c * fstride;
        const double idx0 = b.idx[0], idx1 = b.idx[1];
#pragma unroll
        for (int q = 0; q < kNQ; q++) {
          double r = 0.0;
          r = r - ((double)fup[q] - (double)flo[q]) * idx0;
          r = r - ((double)fy[q] - (double)fprev[q]) * idx1;
          st<real>(b.R[q], cprev, (real)r);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < kNQ; q++) fprev[q] = fy[q];
  }
}

// lanes (columns) per workgroup of the y march with the x faces when its
// window is in registers
constexpr int kYXW = 2 * kTPB;

// TPB lanes per workgroup: 256, or 512 with the window in registers, so
// that a periodic row of up to 512 cells lies in one workgroup and every
// x face above a lane's cell is a face another lane computes (with rows
// split between workgroups, the last lane of a piece solves one more face
// and its wavefront runs the solver twice).
template <typename real, int LW, int RS, int TPB>
__global__ __launch_bounds__(TPB) void k_sweep_march_xy(Launch L) {
  static_assert(TPB == kTPB || (TPB == 2 * kTPB && LW == 0), "LDS window: 256 lanes only");
  __shared__ real lds[LW ? 21 : 1][kTPB];
  __shared__ XRing<real, TPB> xr;
  for (int v = blockIdx.x; v < tile_slots(L); v += gridDim.x) {
    const int tile = tile_of(L, v);
    if (tile >= L.ntiles) continue;
    const int bi = find_box(table(L.base) + kYS * (L.nboxes + 1), L.nboxes, tile);
    CBox& b = box_at(L.boxes, bi);
    const int lt = tile - table(L.base)[kYS * (L.nboxes + 1) + bi];
    const int seg = lt % b.yseg;
    const int ct = lt / b.yseg;
    const int ncols = b.n[0] * b.n[2];
    const int col0 = ct * TPB + (int)threadIdx.x;
    // lanes past the last column take part in the barriers on a copy of
    // the last column and store nothing
    const bool live = col0 < ncols;
    const int col = live ? col0 : ncols - 1;
    const int i = col % b.n[0];
    const int tr = col / b.n[0];
    const int j0 = seg * b.ysl;
    const int j1 = min(j0 + b.ysl, b.n[1]);
    double lmax = 0.0;
    march_column_xy<real, LW, RS, TPB>(b, L.stage, i, tr, col0 < ncols ? col0 : col, ncols, live,
                                       j0, j1, lds, xr, L.lam, lmax);
    if (L.lam) {
      const double m = block_max<TPB>(lmax);
      if (threadIdx.x == 0) b.lam[lt] = m;
    } else {
      __syncthreads();  // the next tile reuses the LDS
    }
  }
}

// inactive axis D: residual from the earlier axes only, face data from the
// cell (EMF = cell EMF, mass flux = momentum)
template <typename real, int D>
__device__ __forceinline__ void inactive_column(CBox& b, int s, int dst, int comb, int i,
                                                int tr) {
  auto pos = [&](int a, int& ii, int& jj, int& kk) {
    ii = i;
    if (D == 1) { jj = a; kk = tr; } else { jj = tr; kk = a; }
  };
  const int t1 = (D + 1) % 3, t2 = (D + 2) % 3;
  for (int f = 0; f < b.nf[D]; ++f) {
    int ii, jj, kk;
    pos(map_cell(f, b.n[D], b.per[D]), ii, jj, kk);
    const int c = cidx(b, ii, jj, kk);
    int fi_, fj_, fk_;
    pos(f, fi_, fj_, fk_);
    const int fi = fidx(b, D, fi_, fj_, fk_);
    st<real>(b.EF[D][0], fi, ld<real>(b.Ec[t1], c));
    st<real>(b.EF[D][1], fi, ld<real>(b.Ec[t2], c));
    st<real>(b.MF[D], fi, (real)ld<double>(b.U[s][1 + D], c));
  }
  int ci, cj, ck;
  pos(0, ci, cj, ck);
  const int c = cidx(b, ci, cj, ck);
  if (D == 1) {
    const int f0 = fidx(b, 0, ci, cj, ck);
    const int f1 = fidx(b, 0, face_up(ci, b.n[0], b.per[0]), cj, ck);
#pragma unroll
    for (int q = 0; q < kNQ; q++) {
      double r = 0.0;
      if (b.act[0])
        r = r - ((double)ld<real>(b.FX[q], f1) - (double)ld<real>(b.FX[q], f0)) * b.idx[0];
      st<real>(b.R[q], c, (real)r);
    }
  } else {
    const double dt = b.scal[0];
#pragma unroll
    for (int q = 0; q < kNQ; q++) {
      double r = (double)ld<real>(b.R[q], c);
      const double uold = comb ? ld<double>(b.U[0][q], c) : 0.0;
      st<double>(b.U[dst][q], c, rk_combine(comb, uold, ld<double>(b.U[s][q], c), dt * r));
    }
  }
}

// PF: prefetch the inputs of the cell update ahead of the Riemann solve
// (latency hidden, more registers live across the solve); RS: the Riemann
// solver (see riemann); FZ (y march only, every box with one cell along z
// and more than one along y): the y march completes the stage, RK combine
// and z-face data included, and no z march runs.  SL: slope kind (see
// Window); kinds other than 0 use the register window.
template <typename real, int D, int WPE, int PF, int LW, int CU, int RS, int FZ, int SL>
__global__ __launch_bounds__(kTPB) __attribute__((amdgpu_waves_per_eu(WPE))) void k_sweep_march(
    Launch L) {
  __shared__ real lds[LW ? 21 : 1][kTPB];
  __shared__ double ring[CU ? 3 * kNQ : 1][kTPB];
  const int kind = D == 1 ? kYS : kZS;
  for (int v = blockIdx.x; v < tile_slots(L); v += gridDim.x) {
    const int tile = tile_of(L, v);
    if (tile >= L.ntiles) continue;
    const int bi = find_box(table(L.base) + kind * (L.nboxes + 1), L.nboxes, tile);
    CBox& b = box_at(L.boxes, bi);
    const int lt = tile - table(L.base)[kind * (L.nboxes + 1) + bi];
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
      march_column<real, D, PF, LW, CU, RS, FZ, SL>(b, L.stage, L.dst, L.comb, i, tr, j0, j1, lds, ring);
    } else {
      inactive_column<real, D>(b, L.stage, L.dst, L.comb, i, tr);
    }
  }
}

// decompose a flat position over extents (e0, e1, e2)
__device__ __forceinline__ void unflatten(int p, int e0, int e1, int pos[3]) {
  const int q = p / e0;
  pos[0] = p - q * e0;
  pos[2] = q / e1;
  pos[1] = q - pos[2] * e1;
}

// Position of a lane in the corner-EMF kernel: tiles of ctx x (kTPB / ctx)
// positions of a patch of the xy plane, so that the row below a lane's row,
// whose face values and cell EMFs the lane reads, is mostly fetched by the
// same workgroup; each lane then walks czk planes of its column from plane
// pos[2] (tiles: patches fastest, then blocks of czk planes).  ctx = 0:
// flat order over all positions, one plane per lane.  Returns false for
// lanes past the edge.
__device__ __forceinline__ bool ct_pos(CBox& b, int lt, int pos[3]) {
  const int cx = b.ctx;
  if (cx == 0) {
    const int p = lt * kTPB + (int)threadIdx.x;
    if (p >= b.nf[0] * b.nf[1] * b.nf[2]) return false;
    unflatten(p, b.nf[0], b.nf[1], pos);
    return true;
  }
  const int cy = kTPB / cx;
  const int nbx = (b.nf[0] + cx - 1) / cx;
  const int nby = (b.nf[1] + cy - 1) / cy;
  const int np = nbx * nby;
  const int kb = lt / np;
  const int patch = lt - kb * np;
  const int by = patch / nbx;
  const int bx = patch - by * nbx;
  pos[0] = bx * cx + (int)threadIdx.x % cx;
  pos[1] = by * cy + (int)threadIdx.x / cx;
  pos[2] = kb * b.czk;
  return pos[0] < b.nf[0] && pos[1] < b.nf[1];
}

// planes a lane of the corner-EMF kernel walks from its first plane k0
__device__ __forceinline__ int ct_planes(CBox& b, int k0) {
  return b.ctx == 0 ? 1 : min(b.czk, b.nf[2] - k0);
}

// Slope limiter chosen at run time (the upwind-CT corner states).
template <typename real>
__device__ __forceinline__ real limit_rt(int lim, real a, real b) {
  if (lim == 1) return limit<1>(a, b);
  if (lim == 2) return limit<2>(a, b);
  return limit<0>(a, b);
}

// Value q0 of a cell carried half a cell towards a corner: up (side 0, the
// cell lies below the corner) or down (side 1), with its limited slope
// between the neighbours qm and qp; no slope along an inactive axis.
template <typename real>
__device__ __forceinline__ real to_corner(int lim, int act, int side, real qm, real q0, real qp) {
  const real d = act ? limit_rt(lim, q0 - qm, qp - q0) : (real)0;
  return side == 0 ? q0 + (real)0.5 * d : q0 - (real)0.5 * d;
}

// Largest right-going (left = 0) or left-going (left = 1) signal speed of
// two faces' outer wave speeds, at least zero.
template <typename real>
__device__ __forceinline__ real speed_bound(real s0, real s1, int left) {
  if (left) {
    const real m = s0 < s1 ? s0 : s1;
    return m < (real)0 ? -m : (real)0;
  }
  const real m = s0 > s1 ? s0 : s1;
  return m > (real)0 ? m : (real)0;
}

// Upwind-CT corner EMF along c (Londrillo & Del Zanna 2004, HLL form) at
// corner position pos (a-face index pos[a], b-face index pos[b], (a, b, c)
// cyclic) of state s.  The four cells around the edge give four corner
// states: their velocities along a and b carried to the corner with the
// limited slopes along a, then b.  The a-face field of the two a-faces at
// the corner is carried along b, the b-face field along a.  Speed bounds:
// the outer wave speeds of the same faces.  The corner EMF is the HLL flux
// of the four states along both axes, E_c = v_b B_a - v_a B_b of each
// weighted by the bound towards it, plus the HLL diffusion of B_a along b and
// of B_b along a.  An inactive axis has equal states on both sides and
// weights 1.
template <typename real>
__device__ __forceinline__ real uct_corner(CBox& b, int s, int c, const int pos[3]) {
  const int a = (c + 1) % 3, bb = (c + 2) % 3;
  const int lim = b.lim;
  // mapped indices pos - 2 .. pos + 1 along a and b (map_cell wraps a
  // periodic axis by one period only, which covers two cells when n >= 2;
  // an axis of one cell maps everything to cell 0)
  int ma[4], mb[4];
#pragma unroll
  for (int o = 0; o < 4; o++) {
    ma[o] = b.n[a] == 1 ? 0 : map_cell(pos[a] - 2 + o, b.n[a], b.per[a]);
    mb[o] = b.n[bb] == 1 ? 0 : map_cell(pos[bb] - 2 + o, b.n[bb], b.per[bb]);
  }
  real al[4] = {(real)1, (real)1, (real)1, (real)1};
  int q[3];
  q[c] = pos[c];
  if (b.act[a]) {  // a-faces (ia; ib-1), (ia; ib)
    q[a] = pos[a];
    q[bb] = mb[1];
    const int f0 = fidx(b, a, q[0], q[1], q[2]);
    q[bb] = mb[2];
    const int f1 = fidx(b, a, q[0], q[1], q[2]);
    al[0] = speed_bound(ld<real>(b.SP[a][1], f0), ld<real>(b.SP[a][1], f1), 0);
    al[1] = speed_bound(ld<real>(b.SP[a][0], f0), ld<real>(b.SP[a][0], f1), 1);
  }
  if (b.act[bb]) {  // b-faces (ib; ia-1), (ib; ia)
    q[bb] = pos[bb];
    q[a] = ma[1];
    const int f0 = fidx(b, bb, q[0], q[1], q[2]);
    q[a] = ma[2];
    const int f1 = fidx(b, bb, q[0], q[1], q[2]);
    al[2] = speed_bound(ld<real>(b.SP[bb][1], f0), ld<real>(b.SP[bb][1], f1), 0);
    al[3] = speed_bound(ld<real>(b.SP[bb][0], f0), ld<real>(b.SP[bb][0], f1), 1);
  }
  // velocities along a and b of the cells (ma[oa], mb[ob]), as the x sweep
  // recovered them; the corners of the 4 x 4 block are not needed
  real va[4][4], vb[4][4];
#pragma unroll
  for (int oa = 0; oa < 4; oa++)
#pragma unroll
    for (int ob = 0; ob < 4; ob++) {
      va[oa][ob] = vb[oa][ob] = (real)0;
      if ((oa == 0 || oa == 3) && (ob == 0 || ob == 3)) continue;
      q[a] = ma[oa];
      q[bb] = mb[ob];
      const int ci = cidx(b, q[0], q[1], q[2]);
      va[oa][ob] = ld<real>(b.V[a], ci);
      vb[oa][ob] = ld<real>(b.V[bb], ci);
    }
  real cva[4], cvb[4];
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const int sa = k & 1, sb = k >> 1, oa = 1 + sa, ob = 1 + sb;
#pragma unroll
    for (int e = 0; e < 2; e++) {
      real (*v)[4] = e == 0 ? va : vb;
      const real v0 = v[oa][ob];
      real x = to_corner(lim, b.act[a], sa, v[oa - 1][ob], v0, v[oa + 1][ob]);
      const real db = b.act[bb] ? limit_rt(lim, v0 - v[oa][ob - 1], v[oa][ob + 1] - v0) : (real)0;
      x = sb == 0 ? x + (real)0.5 * db : x - (real)0.5 * db;
      if (e == 0)
        cva[k] = x;
      else
        cvb[k] = x;
    }
  }
  real fa[2], fb[2];
#pragma unroll
  for (int s2 = 0; s2 < 2; s2++) {
    q[c] = pos[c];
    q[a] = pos[a];  // a-face (ia; ib-1+s2), carried along b
    real g[3];
#pragma unroll
    for (int o = 0; o < 3; o++) {
      q[bb] = mb[s2 + o];
      g[o] = (real)ld<double>(b.B[s][a], fidx(b, a, q[0], q[1], q[2]));
    }
    fa[s2] = to_corner(lim, b.act[bb], s2, g[0], g[1], g[2]);
    q[bb] = pos[bb];  // b-face (ib; ia-1+s2), carried along a
#pragma unroll
    for (int o = 0; o < 3; o++) {
      q[a] = ma[s2 + o];
      g[o] = (real)ld<double>(b.B[s][bb], fidx(b, bb, q[0], q[1], q[2]));
    }
    fb[s2] = to_corner(lim, b.act[a], s2, g[0], g[1], g[2]);
  }
  real e[4];
#pragma unroll
  for (int k = 0; k < 4; k++) e[k] = cvb[k] * fa[k >> 1] - cva[k] * fb[k & 1];
  const real num = al[0] * al[2] * e[0] + al[1] * al[2] * e[1] + al[0] * al[3] * e[2] +
                   al[1] * al[3] * e[3];
  const real sa = al[0] + al[1], sb = al[2] + al[3];
  return num / (sa * sb) - al[2] * al[3] / sb * (fa[1] - fa[0]) +
         al[0] * al[1] / sa * (fb[1] - fb[0]);
}

// Upwind-CT corner EMFs (b.emf = 3), tiled like k_ct_edge: a kernel of its
// own, so that the heavier gather of the upwind states does not raise the
// register count of the face-EMF averages.
template <typename real>
__global__ __launch_bounds__(kTPB) void k_ct_uct(Launch L) {
  for (int v = blockIdx.x; v < tile_slots(L); v += gridDim.x) {
    const int tile = tile_of(L, v);
    if (tile >= L.ntiles) continue;
    const int bi = find_box(table(L.base) + kCTE * (L.nboxes + 1), L.nboxes, tile);
    CBox& b = box_at(L.boxes, bi);
    const int lt = tile - table(L.base)[kCTE * (L.nboxes + 1) + bi];
    int pos[3];
    if (!ct_pos(b, lt, pos)) continue;
    const int nk = ct_planes(b, pos[2]);
    for (int kk = 0; kk < nk; ++kk, ++pos[2]) {
#pragma unroll
      for (int c = 0; c < 3; c++) {
        if (pos[c] >= b.n[c]) continue;
        st<real>(b.ED[c], eidx(b, c, pos[0], pos[1], pos[2]), uct_corner<real>(b, L.stage, c, pos));
      }
    }
  }
}

// The corner EMF from its four face EMFs (fa1, fa0 on the a-faces at b-cell
// index ib and ib - 1, fb1, fb0 on the b-faces at a-cell index ia and
// ia - 1), the cell EMFs of the four cells around the edge ((ia-1, ib-1),
// (ia, ib-1), (ia-1, ib), (ia, ib)) and the mass fluxes of the four faces,
// for the averages of k_ct_edge.
template <typename real>
__device__ __forceinline__ real corner_avg(int emf, real fa1, real fa0, real fb1, real fb0,
                                           const real ec[4], real m_a1, real m_a0, real m_b1,
                                           real m_b0) {
  if (emf == 2) return (real)0.25 * (fa1 + fa0 + fb1 + fb0);
  const real dbp = upwind(m_a1, ec[2] - fb0, ec[3] - fb1);
  const real dbm = upwind(m_a0, fb0 - ec[0], fb1 - ec[1]);
  const real dap = upwind(m_b1, ec[1] - fa0, ec[3] - fa1);
  const real dam = upwind(m_b0, fa0 - ec[0], fa1 - ec[2]);
  return (real)0.25 * (fa1 + fa0 + fb1 + fb0) + (real)0.25 * (dbm - dbp) +
         (real)0.25 * (dam - dap);
}

// Corner EMFs: for every corner position one lane computes the EMF along
// each axis c whose range contains it: the contact-upwinded average of
// Gardiner & Stone (2005) (EMF = 0), their E0 average with every
// face-to-corner derivative taken as the mean of its two sides (1), or the
// mean of the four face EMFs (2, Balsara & Spicer 1999; no cell EMF or mass
// flux is read).  A lane walks ct_planes planes of its column: the EMFs
// along x and y at plane k read the plane below (z-cell k - 1) for the
// y-face and x-face EMFs, mass fluxes and cell EMFs that the lane loaded
// itself at plane k - 1, so those come from registers (loaded once before
// the walk for its first plane; the same values, so the same results).
// Every load of a plane is issued before any of its EMFs is formed; a
// position outside an axis's range loads a clamped, valid index and
// stores nothing for that axis.
template <typename real, int EMF>
__global__ __launch_bounds__(kTPB) void k_ct_edge(Launch L) {
  constexpr bool cm = EMF != 2;   // cell EMFs read
  constexpr bool mf = EMF == 0;   // mass fluxes read
  for (int v = blockIdx.x; v < tile_slots(L); v += gridDim.x) {
    const int tile = tile_of(L, v);
    if (tile >= L.ntiles) continue;
    const int bi = find_box(table(L.base) + kCTE * (L.nboxes + 1), L.nboxes, tile);
    CBox& b = box_at(L.boxes, bi);
    const int lt = tile - table(L.base)[kCTE * (L.nboxes + 1) + bi];
    int pos[3];
    if (!ct_pos(b, lt, pos)) continue;
    const int nk = ct_planes(b, pos[2]);
    const int i = pos[0], j = pos[1];
    // mapped cell indices of the positions and of the positions - 1 in x, y
    const int m1x = map_cell(i, b.n[0], b.per[0]), m0x = map_cell(i - 1, b.n[0], b.per[0]);
    const int m1y = map_cell(j, b.n[1], b.per[1]), m0y = map_cell(j - 1, b.n[1], b.per[1]);
    const bool ex_on = i < b.n[0], ey_on = j < b.n[1];
    const int ic = ex_on ? i : b.n[0] - 1;   // x-cell index of the EMF along x
    const int jc = ey_on ? j : b.n[1] - 1;   // y-cell index of the EMF along y
    // plane-below values of the EMFs along x (y-face EMF and mass flux at
    // (ic, j), cell EMFs (ic, m0y) and (ic, m1y)) and along y (x-face EMF
    // and mass flux at (i, jc), cell EMFs (m0x, jc) and (m1x, jc))
    real xa, xma = 0, xe0 = 0, xe1 = 0, ya, yma = 0, ye0 = 0, ye1 = 0;
    {
      const int m0z = map_cell(pos[2] - 1, b.n[2], b.per[2]);
      xa = ld<real>(b.EF[1][1], fidx(b, 1, ic, j, m0z));
      ya = ld<real>(b.EF[0][0], fidx(b, 0, i, jc, m0z));
      if (mf) {
        xma = ld<real>(b.MF[1], fidx(b, 1, ic, j, m0z));
        yma = ld<real>(b.MF[0], fidx(b, 0, i, jc, m0z));
      }
      if (cm) {
        xe0 = ld<real>(b.Ec[0], cidx(b, ic, m0y, m0z));
        xe1 = ld<real>(b.Ec[0], cidx(b, ic, m1y, m0z));
        ye0 = ld<real>(b.Ec[1], cidx(b, m0x, jc, m0z));
        ye1 = ld<real>(b.Ec[1], cidx(b, m1x, jc, m0z));
      }
    }
    for (int kk = 0; kk < nk; ++kk) {
      const int k = pos[2] + kk;
      const int m1z = map_cell(k, b.n[2], b.per[2]);
      const bool ez_on = k < b.n[2];
      const int kc = ez_on ? k : b.n[2] - 1;   // z-cell index of the EMF along z
      // loads of the plane
      // along z: a = x-faces (i; m1y), (i; m0y), b = y-faces (j; m1x), (j; m0x)
      const int za1 = fidx(b, 0, i, m1y, kc), za0 = fidx(b, 0, i, m0y, kc);
      const int zb1 = fidx(b, 1, m1x, j, kc), zb0 = fidx(b, 1, m0x, j, kc);
      const real zfa1 = ld<real>(b.EF[0][1], za1), zfa0 = ld<real>(b.EF[0][1], za0);
      const real zfb1 = ld<real>(b.EF[1][0], zb1), zfb0 = ld<real>(b.EF[1][0], zb0);
      real zec[4] = {0, 0, 0, 0}, zm[4] = {0, 0, 0, 0};
      if (cm) {
        zec[0] = ld<real>(b.Ec[2], cidx(b, m0x, m0y, kc));
        zec[1] = ld<real>(b.Ec[2], cidx(b, m1x, m0y, kc));
        zec[2] = ld<real>(b.Ec[2], cidx(b, m0x, m1y, kc));
        zec[3] = ld<real>(b.Ec[2], cidx(b, m1x, m1y, kc));
      }
      if (mf) {
        zm[0] = ld<real>(b.MF[0], za1);
        zm[1] = ld<real>(b.MF[0], za0);
        zm[2] = ld<real>(b.MF[1], zb1);
        zm[3] = ld<real>(b.MF[1], zb0);
      }
      // along x: a = y-faces (j; m1z), (j; m0z), b = z-faces (k; m1y), (k; m0y)
      const int xa1 = fidx(b, 1, ic, j, m1z);
      const int xb1 = fidx(b, 2, ic, m1y, k), xb0 = fidx(b, 2, ic, m0y, k);
      const real xfa1 = ld<real>(b.EF[1][1], xa1);
      const real xfb1 = ld<real>(b.EF[2][0], xb1), xfb0 = ld<real>(b.EF[2][0], xb0);
      real xec2 = 0, xec3 = 0, xm1 = 0, xmb1 = 0, xmb0 = 0;
      if (cm) {
        xec2 = ld<real>(b.Ec[0], cidx(b, ic, m0y, m1z));
        xec3 = ld<real>(b.Ec[0], cidx(b, ic, m1y, m1z));
      }
      if (mf) {
        xm1 = ld<real>(b.MF[1], xa1);
        xmb1 = ld<real>(b.MF[2], xb1);
        xmb0 = ld<real>(b.MF[2], xb0);
      }
      // along y: a = z-faces (k; m1x), (k; m0x), b = x-faces (i; m1z), (i; m0z)
      const int ya1 = fidx(b, 2, m1x, jc, k), ya0 = fidx(b, 2, m0x, jc, k);
      const int yb1 = fidx(b, 0, i, jc, m1z);
      const real yfa1 = ld<real>(b.EF[2][1], ya1), yfa0 = ld<real>(b.EF[2][1], ya0);
      const real yfb1 = ld<real>(b.EF[0][0], yb1);
      real yec1 = 0, yec3 = 0, yma1 = 0, yma0 = 0, ymb1 = 0;
      if (cm) {
        yec1 = ld<real>(b.Ec[1], cidx(b, m0x, jc, m1z));
        yec3 = ld<real>(b.Ec[1], cidx(b, m1x, jc, m1z));
      }
      if (mf) {
        yma1 = ld<real>(b.MF[2], ya1);
        yma0 = ld<real>(b.MF[2], ya0);
        ymb1 = ld<real>(b.MF[0], yb1);
      }
      // the EMFs of the plane
      if (ez_on)
        st<real>(b.ED[2], eidx(b, 2, i, j, k),
                 corner_avg<real>(EMF, zfa1, zfa0, zfb1, zfb0, zec, zm[0], zm[1], zm[2], zm[3]));
      if (ex_on) {
        const real ec[4] = {xe0, xe1, xec2, xec3};
        st<real>(b.ED[0], eidx(b, 0, i, j, k),
                 corner_avg<real>(EMF, xfa1, xa, xfb1, xfb0, ec, xm1, xma, xmb1, xmb0));
      }
      if (ey_on) {
        const real ec[4] = {ye0, yec1, ye1, yec3};
        st<real>(b.ED[1], eidx(b, 1, i, j, k),
                 corner_avg<real>(EMF, yfa1, yfa0, yfb1, ya, ec, yma1, yma0, ymb1, yma));
      }
      // this plane's values are the next plane's plane-below values
      xa = xfa1;
      xma = xm1;
      xe0 = xec2;
      xe1 = xec3;
      ya = yfb1;
      yma = ymb1;
      ye0 = yec1;
      ye1 = yec3;
    }
  }
}

// Face update: dB_d/dt = -[(E_f(e+1/2) - E_f(e-1/2))/dx_e
//                          - (E_e(f+1/2) - E_e(f-1/2))/dx_f], (d, e, f)
// cyclic, formed in FP64, then the Runge-Kutta stage combine.  Every input
// of the lane's three faces is loaded before any is used (an index that a
// face does not need points at a valid element, mostly one the lane reads
// anyway, and its value is not used), so that the loads overlap instead of
// waiting one after another behind the conditions on the axes and the
// combine.
template <typename real>
__global__ __launch_bounds__(kTPB) void k_ct_face(Launch L) {
  for (int v = blockIdx.x; v < tile_slots(L); v += gridDim.x) {
    const int tile = tile_of(L, v);
    if (tile >= L.ntiles) continue;
    const int bi = find_box(table(L.base) + kCTF * (L.nboxes + 1), L.nboxes, tile);
    CBox& b = box_at(L.boxes, bi);
    const int lt = tile - table(L.base)[kCTF * (L.nboxes + 1) + bi];
    const int p = lt * kTPB + (int)threadIdx.x;
    if (p >= b.nf[0] * b.nf[1] * b.nf[2]) continue;
    int pos[3];
    unflatten(p, b.nf[0], b.nf[1], pos);
    const double dt = b.scal[0];
    bool ok[3];
    int fi[3], i1h[3], i1l[3], i2h[3], i2l[3];
    real e1h[3], e1l[3], e2h[3], e2l[3];
    double bs[3], bo[3];
#pragma unroll
    for (int d = 0; d < 3; d++) {
      const int e = (d + 1) % 3, f = (d + 2) % 3;
      ok[d] = pos[e] < b.n[e] && pos[f] < b.n[f];
      // a face that does not exist reads its lane's first face instead
      int q0[3] = {pos[0], pos[1], pos[2]};
      if (!ok[d]) q0[e] = q0[f] = 0;
      const int lo_f = eidx(b, f, q0[0], q0[1], q0[2]);
      const int lo_e = eidx(b, e, q0[0], q0[1], q0[2]);
      int q[3] = {q0[0], q0[1], q0[2]};
      if (b.act[e]) q[e] = face_up(q0[e], b.n[e], b.per[e]);
      i1h[d] = b.act[e] ? eidx(b, f, q[0], q[1], q[2]) : lo_f;
      i1l[d] = lo_f;
      q[e] = q0[e];
      if (b.act[f]) q[f] = face_up(q0[f], b.n[f], b.per[f]);
      i2h[d] = b.act[f] ? eidx(b, e, q[0], q[1], q[2]) : lo_e;
      i2l[d] = lo_e;
      fi[d] = fidx(b, d, q0[0], q0[1], q0[2]);
    }
#pragma unroll
    for (int d = 0; d < 3; d++) {
      const int e = (d + 1) % 3, f = (d + 2) % 3;
      e1h[d] = ld<real>(b.ED[f], i1h[d]);
      e1l[d] = ld<real>(b.ED[f], i1l[d]);
      e2h[d] = ld<real>(b.ED[e], i2h[d]);
      e2l[d] = ld<real>(b.ED[e], i2l[d]);
      bs[d] = ld<double>(b.B[L.stage][d], fi[d]);
      // the start-of-step field for the combine; without a combine the same
      // element as bs again (no extra traffic), its value unused
      bo[d] = ld<double>(b.B[L.comb ? 0 : L.stage][d], fi[d]);
    }
#pragma unroll
    for (int d = 0; d < 3; d++) {
      const int e = (d + 1) % 3, f = (d + 2) % 3;
      if (!ok[d]) continue;
      double t1 = 0.0, t2 = 0.0;
      if (b.act[e]) t1 = ((double)e1h[d] - (double)e1l[d]) * b.idx[e];
      if (b.act[f]) t2 = ((double)e2h[d] - (double)e2l[d]) * b.idx[f];
      const double rate = -(t1 - t2);
      const double bold = L.comb ? bo[d] : 0.0;
      st<double>(b.B[L.dst][d], fi[d], rk_combine(L.comb, bold, bs[d], dt * rate));
    }
  }
}

// CFL rate of every cell of state s, reduced to one max per tile
static __global__ __launch_bounds__(kTPB) void k_lambda(Launch L) {
  for (int v = blockIdx.x; v < tile_slots(L); v += gridDim.x) {
    const int tile = tile_of(L, v);
    if (tile >= L.ntiles) continue;
    const int bi = find_box(table(L.base) + kLAM * (L.nboxes + 1), L.nboxes, tile);
    CBox& b = box_at(L.boxes, bi);
    const int lt = tile - table(L.base)[kLAM * (L.nboxes + 1) + bi];
    const int p = lt * kTPB + (int)threadIdx.x;
    const int N = b.n[0] * b.n[1] * b.n[2];
    double lmax = 0.0;
    if (p < N) {
      int pos[3];
      unflatten(p, b.n[0], b.n[1], pos);
      PrimD w;
      load_prim(b, L.stage, pos[0], pos[1], pos[2], w);
      lmax = cfl_rate(b, w);
    }
    const double m = block_max(lmax);
    if (threadIdx.x == 0) b.lam[lt] = m;
  }
}

// One workgroup per box: max of the tile partials -> time step.  mode 0:
// step (clamp to t_stop, advance t); mode 1: query (dt of the current state
// into scal[3]).  npart: kind whose tiles wrote the partials.
static __global__ __launch_bounds__(kTPB) void k_dt(const Box* boxes, int mode, int kind) {
  CBox& b = box_at(boxes, blockIdx.x);
  const int n = b.ntile[kind];
  // 32 independent loads in flight per lane (a 256^3 box has 65536
  // partials: 256 per lane, so eight round trips)
  double mm[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int t0 = threadIdx.x; t0 < n; t0 += 32 * kTPB) {
    double v[32];
#pragma unroll
    for (int u = 0; u < 32; u++) {
      const int t = t0 + u * kTPB;
      v[u] = t < n ? b.lam[t] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 32; u++)
      if (v[u] > mm[u & 7]) mm[u & 7] = v[u];
  }
  double m = 0.0;
#pragma unroll
  for (int u = 0; u < 8; u++)
    if (mm[u] > m) m = mm[u];
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

// CFL time step of one box whose state the caller holds in the boundary
// layout (five cell arrays, three face arrays with both bounding faces),
// described by value in the kernel arguments, for the allocation-free entry
// point: k_lambda_flat writes one max rate per tile of kTPB cells into the
// caller-provided partials, k_dt_flat reduces them into dt = cfl / max.  A
// non-physical cell makes its rate infinite, so the step is zero.
struct FlatBox {
  const double* U[kNQ];
  const double* B[3];
  int n[3];
  int act[3];
  double idx[3];
  double gamma, pfloor, cfl;
  int ntiles;
};

static __global__ __launch_bounds__(kTPB) void k_lambda_flat(FlatBox f, double* part) {
  const int tile = blockIdx.x;
  const int p = tile * kTPB + (int)threadIdx.x;
  const int nx = f.n[0], ny = f.n[1];
  double lmax = 0.0;
  if (p < nx * ny * f.n[2]) {
    int pos[3];
    unflatten(p, nx, ny, pos);
    const int i = pos[0], j = pos[1], k = pos[2];
    const int fx = (k * ny + j) * (nx + 1) + i;
    const int fy = (k * (ny + 1) + j) * nx + i;
    const double bx = 0.5 * (ld<double>(f.B[0], fx) + ld<double>(f.B[0], fx + 1));
    const double by = 0.5 * (ld<double>(f.B[1], fy) + ld<double>(f.B[1], fy + nx));
    const double bz = 0.5 * (ld<double>(f.B[2], p) + ld<double>(f.B[2], p + nx * ny));
    PrimD w;
    const int fl = cons_to_prim(ld<double>(f.U[0], p), ld<double>(f.U[1], p), ld<double>(f.U[2], p),
                                ld<double>(f.U[3], p), ld<double>(f.U[4], p), bx, by, bz, f.gamma,
                                f.pfloor, w);
    lmax = (fl & 2) ? __builtin_inf() : cfl_rate(f, w);
  }
  const double m = block_max(lmax);
  if (threadIdx.x == 0) part[tile] = m;
}

static __global__ __launch_bounds__(kTPB) void k_dt_flat(const double* part, int ntiles, double cfl,
                                                         double* dt_out) {
  double m = 0.0;
  for (int t = threadIdx.x; t < ntiles; t += kTPB) {
    const double v = part[t];
    if (v > m) m = v;
  }
  m = block_max(m);
  if (threadIdx.x == 0) dt_out[0] = cfl / m;
}

// Periodic-face check of a caller array in the boundary layout: sets *bad
// when face n differs from face 0 anywhere along axis d.
static __global__ __launch_bounds__(kTPB) void k_check_periodic(const double* a, int d, int nx, int ny,
                                                         int nz, int* bad) {
  // boundary layout extents: n+1 along d
  const int ex = nx + (d == 0), ey = ny + (d == 1);
  const int ext0 = d == 0 ? 1 : nx, ext1 = d == 1 ? 1 : ny;
  const int P = ext0 * ext1 * (d == 2 ? 1 : nz);
  for (int p = blockIdx.x * kTPB + threadIdx.x; p < P; p += gridDim.x * kTPB) {
    int pos[3];
    unflatten(p, ext0, ext1, pos);
    int i2 = pos[0], j2 = pos[1], k2 = pos[2];
    if (d == 0) i2 = nx; else if (d == 1) j2 = ny; else k2 = nz;
    const size_t a0 = ((size_t)pos[2] * ey + pos[1]) * ex + pos[0];
    const size_t a1 = ((size_t)k2 * ey + j2) * ex + i2;
    if (a[a0] != a[a1]) atomicOr(bad, 1);
  }
}

}  // namespace mhd
