/*
 * mhd_oracle.c -- plain serial FP64 oracle of the ideal-MHD update.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark.  The GPU library never links, calls or
 * includes anything from here.  Built with -ffp-contract=off (no fused
 * multiply-add), IEEE division and square root.
 *
 * What it computes (arXiv 2606.12753 §2.2.3, "main cycle"): a finite-volume
 * Godunov update of the ideal-MHD conservation laws that, per direction,
 * reconstructs primitive variables, solves a Riemann problem at each interface
 * and applies the conservative flux difference; constrained transport (CT)
 * evolves the face-centred magnetic field; Runge-Kutta integrates in time.
 * The paper names these stages but prints none of their formulas, so each
 * stage below follows the published algorithm it is named after:
 *   - reconstruction: piecewise-linear primitive variables, minmod limiter;
 *   - Riemann solver: HLLD of Miyoshi & Kusano (2005, J. Comput. Phys. 208),
 *     falling back to HLL (Harten, Lax & van Leer 1983) on unphysical stars;
 *   - CT corner EMF: contact-upwinded average of Gardiner & Stone (2005,
 *     J. Comput. Phys. 205), face update as the discrete curl;
 *   - time stepping: two- or three-stage SSP Runge-Kutta (Shu & Osher 1988;
 *     the paper runs the third-order scheme by default);
 *   - time step: CFL condition on the fast magnetosonic speed.
 *
 * Readings of points the paper leaves open (all shared with the GPU library,
 * which writes them independently):
 *   gamma-law gas, magnetic pressure |B|^2/2; seven reconstructed primitives
 *   per direction (rho, v_n, v_t1, v_t2, p, B_t1, B_t2) in the cyclic frame
 *   (n, t1, t2) = (d, d+1, d+2) mod 3, the normal field taken from the face;
 *   wave speeds S_L = min(u_L,u_R) - max(cf_L,cf_R), S_R = max(u_L,u_R) +
 *   max(cf_L,cf_R); HLLD degeneracy thresholds 1e-12 (relative to the star
 *   total pressure); HLL used at a face when S_M is not strictly inside
 *   (S_L, S_R), the star total pressure or a star thermal pressure is not
 *   positive, or the HLLD flux is not finite; the CT upwinding treats a
 *   mass flux below 1e-12 (rho_L + rho_R)(|S_L| + |S_R|) as zero; primitive pressure floor (total energy untouched); an inactive
 *   axis (one cell) carries the physical flux of the cell, so no divergence
 *   and face EMFs equal to the cell EMF; outflow ghosts copy the boundary
 *   cell's cell-centred state and the tangential faces; the CFL rate of a cell
 *   is the max over active axes of (|v_d| + c_f,d)/dx_d.
 *
 * Floating-point evaluation: every quotient is an IEEE division written as
 * the formula writes it (m/rho, p/(gamma-1), flux differences over dx, the
 * HLLD and HLL quotients), with no fused multiply-add.  The oracle's
 * rounding is its own: it is not arranged to follow any other
 * implementation, so agreement with one is agreement to rounding, not bit
 * for bit.
 *
 * Parity pins live in tests/ (consistency, exact contact and rotational
 * discontinuities, conservation, div B, uniform state, symmetry, second-order
 * convergence on the circularly polarised Alfven wave).
 */
#include "mhd_oracle.h"

#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NG 3            /* ghost width of the padded work arrays */
#define NQ 5            /* hydro conserved variables */
#define EPS_DEG 1.0e-12 /* HLLD degenerate-denominator threshold */
#define EPS_B 1.0e-12   /* HLLD "B_n ~ 0" threshold: skip double-star states */
#define EPS_M 1.0e-12   /* CT upwinding: mass flux zero up to rounding */

struct orc_box {
  int n[3];
  int bc[3];
  int active[3];
  int rk;               /* Runge-Kutta stages: 2 (SSP-RK2) or 3 (SSP-RK3) */
  int solver;           /* Riemann solver: ORC_HLLD (HLL fallback) or ORC_HLL */
  int rec;              /* reconstruction: ORC_REC_PRIM or ORC_REC_CHAR */
  int emf;              /* corner EMF: ORC_EMF_CONTACT, ORC_EMF_E0, ORC_EMF_ARITH */
  int lim;              /* slope limiter: ORC_LIM_MINMOD, ORC_LIM_MC, ORC_LIM_VANLEER */
  double dx[3];         /* cell size */
  double gamma, cfl, pfloor;
  int sx, sy, sz;      /* padded extents: n + 2 NG + 1 (one extra face) */
  size_t np;           /* elements per padded array */
  double *U[NQ], *B[3];    /* state */
  double *U0[NQ], *B0[3];  /* state at the start of the step */
  double *Bc[3];           /* cell-centred field */
  double *W[8];            /* primitives */
  double *Ec[3];           /* cell EMF  E = -v x B */
  double *FH[3][NQ];       /* hydro flux on d-faces (lab frame) */
  double *EF[3][3];        /* EMF component c on d-faces (c != d used) */
  double *FM[3];           /* mass flux on d-faces */
  double *R[NQ];           /* cell residual */
  double *ED[3];           /* corner EMF along axis c */
  double *RB[3];           /* face rate */
  double *SP[3][2];        /* outer wave speeds S_L, S_R on d-faces (read by
                              the upwind-CT corner EMF only) */
  double t;
  long long nfloor, nhll, nbad;
};

static inline size_t IX(const orc_box *b, int i, int j, int k) {
  return ((size_t)(k + NG) * (size_t)b->sy + (size_t)(j + NG)) * (size_t)b->sx +
         (size_t)(i + NG);
}

/* index of (a,b,c) triple given axis roles: pos[axis] */
static inline size_t IXp(const orc_box *b, const int pos[3]) {
  return IX(b, pos[0], pos[1], pos[2]);
}

/* ------------------------------------------------------------------ */
/* point physics                                                       */
/* ------------------------------------------------------------------ */

double orc_minmod(double a, double b) {
  if (a > 0.0 && b > 0.0) return a < b ? a : b;
  if (a < 0.0 && b < 0.0) return a > b ? a : b;
  return 0.0;
}

/* Monotonised central limiter (van Leer 1977): the central difference
 * (a + b)/2, bounded by twice each one-sided difference; 0 at an extremum. */
double orc_mc(double a, double b) {
  if (a > 0.0 && b > 0.0) {
    double c = 0.5 * (a + b);
    double m = 2.0 * a < 2.0 * b ? 2.0 * a : 2.0 * b;
    return c < m ? c : m;
  }
  if (a < 0.0 && b < 0.0) {
    double c = 0.5 * (a + b);
    double m = 2.0 * a > 2.0 * b ? 2.0 * a : 2.0 * b;
    return c > m ? c : m;
  }
  return 0.0;
}

/* van Leer's harmonic limiter (van Leer 1974): 2ab/(a + b) where a and b
 * have the same sign, else 0. */
double orc_vanleer(double a, double b) {
  if ((a > 0.0 && b > 0.0) || (a < 0.0 && b < 0.0)) return 2.0 * a * b / (a + b);
  return 0.0;
}

/* limited slope from the two one-sided differences */
double orc_limit(int lim, double a, double b) {
  if (lim == ORC_LIM_MC) return orc_mc(a, b);
  if (lim == ORC_LIM_VANLEER) return orc_vanleer(a, b);
  return orc_minmod(a, b);
}

int orc_cons_to_prim(const double u[5], const double bc[3], double gamma,
                     double pfloor, double w[8]) {
  double rho = u[0];
  double vx = u[1] / rho;
  double vy = u[2] / rho;
  double vz = u[3] / rho;
  double ek = 0.5 * rho * (vx * vx + vy * vy + vz * vz);
  double em = 0.5 * (bc[0] * bc[0] + bc[1] * bc[1] + bc[2] * bc[2]);
  double p = (gamma - 1.0) * (u[4] - ek - em);
  int fl = 0;
  if (p < pfloor) {
    p = pfloor;
    fl |= 1;
  }
  if (!(rho > 0.0) || !isfinite(rho) || !isfinite(vx) || !isfinite(vy) ||
      !isfinite(vz) || !isfinite(p))
    fl |= 2;
  w[0] = rho;
  w[1] = vx;
  w[2] = vy;
  w[3] = vz;
  w[4] = p;
  w[5] = bc[0];
  w[6] = bc[1];
  w[7] = bc[2];
  return fl;
}

/* PLM face values of the interface between cells c-1 and c from the cell
 * values q(c-2), q(c-1), q(c), q(c+1): left = q(c-1) + slope(c-1)/2,
 * right = q(c) - slope(c)/2 with minmod slopes. */
void orc_plm_face(double qm2, double qm1, double q0, double qp1, double *ql,
                  double *qr) {
  double dm1 = orc_minmod(qm1 - qm2, q0 - qm1);
  double d0 = orc_minmod(q0 - qm1, qp1 - q0);
  *ql = qm1 + 0.5 * dm1;
  *qr = q0 - 0.5 * d0;
}

/* Eigen-decomposition of the primitive-variable ideal-MHD system along one
 * axis, w = (rho, v_n, v_t1, v_t2, p, B_t1, B_t2), B_n = bn: the seven
 * waves in the order u-c_f, u-c_a, u-c_s, u, u+c_s, u+c_a, u+c_f; R[v][k]
 * = component v of right eigenvector k, L[k][v] = component v of left
 * eigenvector k, L = R^-1.  Normalisation of Roe & Balsara (1996):
 * alpha_f^2 = (a^2 - c_s^2)/(c_f^2 - c_s^2), alpha_s^2 = (c_f^2 - a^2)/
 * (c_f^2 - c_s^2) (alpha_f = 1, alpha_s = 0 where c_f = c_s), beta = B_t/|B_t|
 * (both 1/sqrt 2 where B_t = 0), S = sign(B_n) (+1 for B_n = 0).
 * c_f^2 - c_s^2 is the square root of the discriminant, written as
 * (a^2 - b_n^2)^2 + b_t^2 (2 (a^2 + b_n^2) + b_t^2) so that it is a sum of
 * non-negative terms; c_s^2 = a^2 b_n^2 / c_f^2 (the product of the roots).
 * Vectors derived from the linearised equations (the components of each
 * wave follow from the continuity, normal momentum, pressure and induction
 * equations; the left rows follow from the identities c_f^2 + c_s^2 =
 * a^2 + b^2 and c_f^2 c_s^2 = a^2 b_n^2). */
void orc_prim_eigen(const double w[7], double bn, double gamma, double lam[7],
                    double R[7][7], double L[7][7]) {
  double rho = w[0], u = w[1], p = w[4], by = w[5], bz = w[6];
  double sr = sqrt(rho);
  double a2 = gamma * p / rho;
  double a = sqrt(a2);
  double bn2 = bn * bn / rho;
  double bt2 = (by * by + bz * bz) / rho;
  double dd = a2 - bn2;
  double disc = dd * dd + bt2 * (2.0 * (a2 + bn2) + bt2);
  double sq = sqrt(disc);
  double cf2 = 0.5 * (a2 + bn2 + bt2 + sq);
  double cs2 = a2 * bn2 / cf2;
  double cf = sqrt(cf2), cs = sqrt(cs2), ca = sqrt(bn2);
  /* a^2 - c_s^2 = (sq + dd - b_t^2)/2 and c_f^2 - a^2 = (sq - dd + b_t^2)/2
   * with sq = c_f^2 - c_s^2, dd = a^2 - b_n^2.  Of sq + dd and sq - dd the
   * one that cancels is formed from their product, (sq + dd)(sq - dd) =
   * b_t^2 (2 (a^2 + b_n^2) + b_t^2), so alpha_s keeps its accuracy for a
   * small transverse field (alpha_s ~ |B_t| when a > c_A). */
  double af, as;
  if (sq > 0.0) {
    double g = bt2 * (2.0 * (a2 + bn2) + bt2);
    double sp, sm;
    if (dd > 0.0) {
      sp = sq + dd;
      sm = g / sp;
    } else {
      sm = sq - dd;
      sp = g / sm;
    }
    double af2 = 0.5 * (sp - bt2) / sq;
    double as2 = 0.5 * (sm + bt2) / sq;
    af2 = af2 < 0.0 ? 0.0 : (af2 > 1.0 ? 1.0 : af2);
    as2 = as2 < 0.0 ? 0.0 : (as2 > 1.0 ? 1.0 : as2);
    af = sqrt(af2);
    as = sqrt(as2);
  } else {
    af = 1.0;
    as = 0.0;
  }
  double bt = sqrt(by * by + bz * bz);
  double bey, bez;
  if (bt > 0.0) {
    bey = by / bt;
    bez = bz / bt;
  } else {
    bey = 1.0 / sqrt(2.0);
    bez = bey;
  }
  double sg = bn < 0.0 ? -1.0 : 1.0;
  double qf = sg * af * cf, qs = sg * as * cs;  /* S alpha c */
  double Af = af * a * sr, As = as * a * sr;    /* alpha a sqrt(rho) */
  double N = 0.5 / a2;
  int v, k;
  for (v = 0; v < 7; v++)
    for (k = 0; k < 7; k++) R[v][k] = L[k][v] = 0.0;
  lam[0] = u - cf;
  lam[1] = u - ca;
  lam[2] = u - cs;
  lam[3] = u;
  lam[4] = u + cs;
  lam[5] = u + ca;
  lam[6] = u + cf;
  /* fast, u -/+ c_f */
  R[0][0] = rho * af;  R[1][0] = -af * cf;  R[2][0] = qs * bey;  R[3][0] = qs * bez;
  R[4][0] = rho * af * a2;  R[5][0] = As * bey;  R[6][0] = As * bez;
  R[0][6] = rho * af;  R[1][6] = af * cf;  R[2][6] = -qs * bey;  R[3][6] = -qs * bez;
  R[4][6] = rho * af * a2;  R[5][6] = As * bey;  R[6][6] = As * bez;
  /* Alfven, u -/+ c_a */
  R[2][1] = -bez;  R[3][1] = bey;  R[5][1] = -sg * sr * bez;  R[6][1] = sg * sr * bey;
  R[2][5] = -bez;  R[3][5] = bey;  R[5][5] = sg * sr * bez;  R[6][5] = -sg * sr * bey;
  /* slow, u -/+ c_s */
  R[0][2] = rho * as;  R[1][2] = -as * cs;  R[2][2] = -qf * bey;  R[3][2] = -qf * bez;
  R[4][2] = rho * as * a2;  R[5][2] = -Af * bey;  R[6][2] = -Af * bez;
  R[0][4] = rho * as;  R[1][4] = as * cs;  R[2][4] = qf * bey;  R[3][4] = qf * bez;
  R[4][4] = rho * as * a2;  R[5][4] = -Af * bey;  R[6][4] = -Af * bez;
  /* entropy, u */
  R[0][3] = 1.0;
  /* left rows */
  L[0][1] = -N * af * cf;  L[0][2] = N * qs * bey;  L[0][3] = N * qs * bez;
  L[0][4] = N * af / rho;  L[0][5] = N * As * bey / rho;  L[0][6] = N * As * bez / rho;
  L[6][1] = N * af * cf;  L[6][2] = -N * qs * bey;  L[6][3] = -N * qs * bez;
  L[6][4] = N * af / rho;  L[6][5] = N * As * bey / rho;  L[6][6] = N * As * bez / rho;
  L[1][2] = -0.5 * bez;  L[1][3] = 0.5 * bey;
  L[1][5] = -0.5 * sg * bez / sr;  L[1][6] = 0.5 * sg * bey / sr;
  L[5][2] = -0.5 * bez;  L[5][3] = 0.5 * bey;
  L[5][5] = 0.5 * sg * bez / sr;  L[5][6] = -0.5 * sg * bey / sr;
  L[2][1] = -N * as * cs;  L[2][2] = -N * qf * bey;  L[2][3] = -N * qf * bez;
  L[2][4] = N * as / rho;  L[2][5] = -N * Af * bey / rho;  L[2][6] = -N * Af * bez / rho;
  L[4][1] = N * as * cs;  L[4][2] = N * qf * bey;  L[4][3] = N * qf * bez;
  L[4][4] = N * as / rho;  L[4][5] = -N * Af * bey / rho;  L[4][6] = -N * Af * bez / rho;
  L[3][0] = 1.0;  L[3][4] = -1.0 / a2;
}

/* Limited slope of cell 0 from its neighbours qm, qp (seven face-frame
 * primitives each), with limiter lim (orc_limit).  rec = ORC_REC_PRIM: the
 * limiter on the two one-sided differences per variable.  ORC_REC_CHAR: the
 * differences are projected on the left eigenvectors of the cell's own
 * state (B_n = bn, its cell-centred normal field), limited per
 * characteristic field and projected back with the right eigenvectors;
 * where that slope would make the density or pressure at either face of the
 * cell non-positive, the cell takes the primitive slope instead. */
void orc_slope(const double qm[7], const double q0[7], const double qp[7], double bn,
               double gamma, int rec, int lim, double d[7]) {
  double dm[7], dp[7];
  int v, k;
  for (v = 0; v < 7; v++) {
    dm[v] = q0[v] - qm[v];
    dp[v] = qp[v] - q0[v];
  }
  if (rec == ORC_REC_CHAR) {
    double lam[7], R[7][7], L[7][7], ch[7];
    orc_prim_eigen(q0, bn, gamma, lam, R, L);
    for (k = 0; k < 7; k++) {
      double cm = 0.0, cp = 0.0;
      for (v = 0; v < 7; v++) {
        cm = cm + L[k][v] * dm[v];
        cp = cp + L[k][v] * dp[v];
      }
      ch[k] = orc_limit(lim, cm, cp);
    }
    for (v = 0; v < 7; v++) {
      double s = 0.0;
      for (k = 0; k < 7; k++) s = s + R[v][k] * ch[k];
      d[v] = s;
    }
    if (q0[0] + 0.5 * d[0] > 0.0 && q0[0] - 0.5 * d[0] > 0.0 &&
        q0[4] + 0.5 * d[4] > 0.0 && q0[4] - 0.5 * d[4] > 0.0)
      return;
  }
  for (v = 0; v < 7; v++) d[v] = orc_limit(lim, dm[v], dp[v]);
}

/* fast magnetosonic speed along the normal of (bn, bt1, bt2) */
double orc_fast_speed(double rho, double p, double bn, double bt1, double bt2,
                      double gamma) {
  double a2 = gamma * p / rho;
  double b2 = (bn * bn + bt1 * bt1 + bt2 * bt2) / rho;
  double bn2 = bn * bn / rho;
  double s = a2 + b2;
  double disc = s * s - 4.0 * a2 * bn2;
  if (disc < 0.0) disc = 0.0;
  return sqrt(0.5 * (s + sqrt(disc)));
}

/* physical flux and conserved state of a face-frame primitive state */
void orc_phys_flux(const double w[7], double bn, double gamma, double f[7],
                   double u[7]) {
  double rho = w[0], vn = w[1], vt1 = w[2], vt2 = w[3], p = w[4];
  double b1 = w[5], b2 = w[6];
  double bsq = bn * bn + b1 * b1 + b2 * b2;
  double pt = p + 0.5 * bsq;
  double vb = vn * bn + vt1 * b1 + vt2 * b2;
  double en = p / (gamma - 1.0) + 0.5 * rho * (vn * vn + vt1 * vt1 + vt2 * vt2) +
              0.5 * bsq;
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

static double total_pressure(const double w[7], double bn) {
  return w[4] + 0.5 * (bn * bn + w[5] * w[5] + w[6] * w[6]);
}

/* HLL flux with the same wave-speed estimate as HLLD */
static void hll_with(const double uL[7], const double fL[7], const double uR[7],
                     const double fR[7], double sl, double sr, double f[7]) {
  int c;
  if (sl >= 0.0) {
    for (c = 0; c < 7; c++) f[c] = fL[c];
    return;
  }
  if (sr <= 0.0) {
    for (c = 0; c < 7; c++) f[c] = fR[c];
    return;
  }
  for (c = 0; c < 7; c++)
    f[c] = (sr * fL[c] - sl * fR[c] + sl * sr * (uR[c] - uL[c])) / (sr - sl);
}

static void wave_speeds(const double wl[7], const double wr[7], double bn,
                        double gamma, double *sl, double *sr) {
  double cfl = orc_fast_speed(wl[0], wl[4], bn, wl[5], wl[6], gamma);
  double cfr = orc_fast_speed(wr[0], wr[4], bn, wr[5], wr[6], gamma);
  double cmax = cfl > cfr ? cfl : cfr;
  double umin = wl[1] < wr[1] ? wl[1] : wr[1];
  double umax = wl[1] > wr[1] ? wl[1] : wr[1];
  *sl = umin - cmax;
  *sr = umax + cmax;
}

void orc_hll(const double wl[7], const double wr[7], double bn, double gamma,
             double f[7]) {
  double uL[7], fL[7], uR[7], fR[7], sl, sr;
  orc_phys_flux(wl, bn, gamma, fL, uL);
  orc_phys_flux(wr, bn, gamma, fR, uR);
  wave_speeds(wl, wr, bn, gamma, &sl, &sr);
  hll_with(uL, fL, uR, fR, sl, sr, f);
}

/* HLLD single-star state of one side (Miyoshi & Kusano 2005, §3-4).
 * w: face-frame prims, u: conserved, pt: total pressure, sa: outer wave
 * speed, sm: contact speed, pts: star total pressure.  Outputs the star
 * conserved vector us[7], tangential velocity/field and v*.B*. */
typedef struct {
  double rho, vt1, vt2, bt1, bt2, en, vb;
  double u[7];
} star_t;

static void star_side(const double w[7], const double u[7], double pt,
                      double sa, double sm, double pts, double bn, star_t *s) {
  double sd = sa - w[1];
  double sms = sa - sm;
  double rs = w[0] * sd / sms;
  double dd = w[0] * sd * sms - bn * bn;
  double vt1s, vt2s, bt1s, bt2s;
  if (fabs(dd) <= EPS_DEG * pts) {
    /* degenerate: tangential velocity and field pass through unchanged */
    vt1s = w[2];
    vt2s = w[3];
    bt1s = w[5];
    bt2s = w[6];
  } else {
    vt1s = w[2] - bn * w[5] * (sm - w[1]) / dd;
    vt2s = w[3] - bn * w[6] * (sm - w[1]) / dd;
    bt1s = w[5] * (w[0] * sd * sd - bn * bn) / dd;
    bt2s = w[6] * (w[0] * sd * sd - bn * bn) / dd;
  }
  double vb = w[1] * bn + w[2] * w[5] + w[3] * w[6];
  double vbs = sm * bn + vt1s * bt1s + vt2s * bt2s;
  double ens = (sd * u[4] - pt * w[1] + pts * sm + bn * (vb - vbs)) / sms;
  s->rho = rs;
  s->vt1 = vt1s;
  s->vt2 = vt2s;
  s->bt1 = bt1s;
  s->bt2 = bt2s;
  s->en = ens;
  s->vb = vbs;
  s->u[0] = rs;
  s->u[1] = rs * sm;
  s->u[2] = rs * vt1s;
  s->u[3] = rs * vt2s;
  s->u[4] = ens;
  s->u[5] = bt1s;
  s->u[6] = bt2s;
}

static double star_pressure(const star_t *s, double sm, double bn,
                            double gamma) {
  return (gamma - 1.0) *
         (s->en - 0.5 * s->rho * (sm * sm + s->vt1 * s->vt1 + s->vt2 * s->vt2) -
          0.5 * (bn * bn + s->bt1 * s->bt1 + s->bt2 * s->bt2));
}

/* Mass flux handed to the CT upwinding: a flux that is zero up to rounding
 * (|F| <= EPS_M (rho_L + rho_R)(|S_L| + |S_R|)) counts as exactly zero, so
 * that a flux that vanishes by symmetry selects the symmetric average
 * rather than a side picked by the sign of rounding noise. */
static double ct_mass_flux(double f0, const double wl[7], const double wr[7],
                           double sl, double sr) {
  double thr = EPS_M * (wl[0] + wr[0]) * (fabs(sl) + fabs(sr));
  return fabs(f0) <= thr ? 0.0 : f0;
}

static int riemann(const double wl[7], const double wr[7], double bn,
                   double gamma, double f[7], double *fm_ct);
static int riemann_flux(const double wl[7], const double wr[7], double bn,
                        double gamma, double f[7]);

int orc_hlld(const double wl[7], const double wr[7], double bn, double gamma,
             double f[7]) {
  double fm;
  return riemann(wl, wr, bn, gamma, f, &fm);
}

double orc_ct_mass_flux(const double wl[7], const double wr[7], double bn,
                        double gamma) {
  double f[7], fm;
  riemann(wl, wr, bn, gamma, f, &fm);
  return fm;
}

static int riemann(const double wl[7], const double wr[7], double bn,
                   double gamma, double f[7], double *fm_ct) {
  int used = riemann_flux(wl, wr, bn, gamma, f);
  double sl, sr;
  wave_speeds(wl, wr, bn, gamma, &sl, &sr);
  *fm_ct = ct_mass_flux(f[0], wl, wr, sl, sr);
  return used;
}

static int riemann_flux(const double wl[7], const double wr[7], double bn,
                        double gamma, double f[7]) {
  double uL[7], fL[7], uR[7], fR[7], sl, sr;
  int c;
  orc_phys_flux(wl, bn, gamma, fL, uL);
  orc_phys_flux(wr, bn, gamma, fR, uR);
  wave_speeds(wl, wr, bn, gamma, &sl, &sr);
  if (sl > 0.0) {
    for (c = 0; c < 7; c++) f[c] = fL[c];
    return 0;
  }
  if (sr < 0.0) {
    for (c = 0; c < 7; c++) f[c] = fR[c];
    return 0;
  }
  double ptl = total_pressure(wl, bn);
  double ptr = total_pressure(wr, bn);
  double sdl = sl - wl[1];
  double sdr = sr - wr[1];
  /* contact speed and star total pressure */
  double sm = (sdr * wr[0] * wr[1] - sdl * wl[0] * wl[1] - ptr + ptl) /
              (sdr * wr[0] - sdl * wl[0]);
  double pts = (sdr * wr[0] * ptl - sdl * wl[0] * ptr +
                wl[0] * wr[0] * sdr * sdl * (wr[1] - wl[1])) /
               (sdr * wr[0] - sdl * wl[0]);
  int ok = (sl < sm) && (sm < sr) && (pts > 0.0);
  double fo[7];
  if (ok) {
    star_t stl, str;
    star_side(wl, uL, ptl, sl, sm, pts, bn, &stl);
    star_side(wr, uR, ptr, sr, sm, pts, bn, &str);
    if (!(star_pressure(&stl, sm, bn, gamma) > 0.0) ||
        !(star_pressure(&str, sm, bn, gamma) > 0.0))
      ok = 0;
    if (ok) {
      if (0.5 * bn * bn <= EPS_B * pts) {
        /* B_n ~ 0: the rotational waves merge with the contact */
        if (sm > 0.0)
          for (c = 0; c < 7; c++) fo[c] = fL[c] + sl * (stl.u[c] - uL[c]);
        else
          for (c = 0; c < 7; c++) fo[c] = fR[c] + sr * (str.u[c] - uR[c]);
      } else {
        double sql = sqrt(stl.rho), sqr = sqrt(str.rho);
        double ssl = sm - fabs(bn) / sql;
        double ssr = sm + fabs(bn) / sqr;
        double sgn = bn > 0.0 ? 1.0 : -1.0;
        double vt1ss = (sql * stl.vt1 + sqr * str.vt1 + (str.bt1 - stl.bt1) * sgn) / (sql + sqr);
        double vt2ss = (sql * stl.vt2 + sqr * str.vt2 + (str.bt2 - stl.bt2) * sgn) / (sql + sqr);
        double bt1ss =
            (sql * str.bt1 + sqr * stl.bt1 + sql * sqr * (str.vt1 - stl.vt1) * sgn) / (sql + sqr);
        double bt2ss =
            (sql * str.bt2 + sqr * stl.bt2 + sql * sqr * (str.vt2 - stl.vt2) * sgn) / (sql + sqr);
        double vbss = sm * bn + vt1ss * bt1ss + vt2ss * bt2ss;
        if (sm > 0.0) {
          double fs[7], uss[7];
          for (c = 0; c < 7; c++) fs[c] = fL[c] + sl * (stl.u[c] - uL[c]);
          if (ssl > 0.0) {
            for (c = 0; c < 7; c++) fo[c] = fs[c];
          } else {
            uss[0] = stl.rho;
            uss[1] = stl.rho * sm;
            uss[2] = stl.rho * vt1ss;
            uss[3] = stl.rho * vt2ss;
            uss[4] = stl.en - sql * (stl.vb - vbss) * sgn;
            uss[5] = bt1ss;
            uss[6] = bt2ss;
            for (c = 0; c < 7; c++) fo[c] = fs[c] + ssl * (uss[c] - stl.u[c]);
          }
        } else {
          double fs[7], uss[7];
          for (c = 0; c < 7; c++) fs[c] = fR[c] + sr * (str.u[c] - uR[c]);
          if (ssr < 0.0) {
            for (c = 0; c < 7; c++) fo[c] = fs[c];
          } else {
            uss[0] = str.rho;
            uss[1] = str.rho * sm;
            uss[2] = str.rho * vt1ss;
            uss[3] = str.rho * vt2ss;
            uss[4] = str.en + sqr * (str.vb - vbss) * sgn;
            uss[5] = bt1ss;
            uss[6] = bt2ss;
            for (c = 0; c < 7; c++) fo[c] = fs[c] + ssr * (uss[c] - str.u[c]);
          }
        }
      }
      for (c = 0; c < 7; c++)
        if (!isfinite(fo[c])) ok = 0;
    }
  }
  if (!ok) {
    hll_with(uL, fL, uR, fR, sl, sr, f);
    return 1;
  }
  for (c = 0; c < 7; c++) f[c] = fo[c];
  return 0;
}

/* upwind selector of the contact-upwinded CT average: flux > 0 picks the
 * lower-side value, < 0 the upper-side value, 0 their mean */
static double upwind(double mflux, double lower, double upper) {
  if (mflux > 0.0) return lower;
  if (mflux < 0.0) return upper;
  return 0.5 * (lower + upper);
}

/* Corner EMF along axis c from the two a-faces and two b-faces around the
 * corner, (a, b, c) cyclic.  Each face value is carried to the corner by half
 * a cell of the transverse derivative, taken on the upwind side of the mass
 * flux through that face (Gardiner & Stone 2005, contact-upwinded average).
 * The four estimates are averaged, which for a plane-parallel grid-aligned
 * flow returns the face value itself. */
double orc_ct_corner(double fa1, double fa0, double fb1, double fb0,
                     const double ec[4], double ma1, double ma0, double mb1,
                     double mb0) {
  /* ec[2*ob + oa]: oa = 0 -> cell ia-1, 1 -> cell ia; ob likewise for b */
  /* d_b at (a-1/2, b-1/4): cell (., ib) minus b-face (., ib-1/2), side by ma1 */
  double dbp = upwind(ma1, ec[2] - fb0, ec[3] - fb1);
  /* d_b at (a-1/2, b-3/4): b-face minus cell (., ib-1), side by ma0 */
  double dbm = upwind(ma0, fb0 - ec[0], fb1 - ec[1]);
  /* d_a at (a-1/4, b-1/2): cell (ia, .) minus a-face, side by mb1 */
  double dap = upwind(mb1, ec[1] - fa0, ec[3] - fa1);
  /* d_a at (a-3/4, b-1/2): a-face minus cell (ia-1, .), side by mb0 */
  double dam = upwind(mb0, fa0 - ec[0], fa1 - ec[2]);
  return 0.25 * (fa1 + fa0 + fb1 + fb0) + 0.25 * (dbm - dbp) +
         0.25 * (dam - dap);
}

/* Corner EMF of the chosen kind: ORC_EMF_CONTACT as orc_ct_corner;
 * ORC_EMF_E0, Gardiner & Stone's E0 average, the same formula with both
 * sides of every derivative averaged (no upwinding); ORC_EMF_ARITH, the
 * mean of the four face EMFs (Balsara & Spicer 1999). */
double orc_ct_corner_kind(int kind, double fa1, double fa0, double fb1, double fb0,
                          const double ec[4], double ma1, double ma0, double mb1,
                          double mb0) {
  if (kind == ORC_EMF_ARITH) return 0.25 * (fa1 + fa0 + fb1 + fb0);
  if (kind == ORC_EMF_E0) return orc_ct_corner(fa1, fa0, fb1, fb0, ec, 0.0, 0.0, 0.0, 0.0);
  return orc_ct_corner(fa1, fa0, fb1, fb0, ec, ma1, ma0, mb1, mb0);
}

/* ------------------------------------------------------------------ */
/* box                                                                 */
/* ------------------------------------------------------------------ */

static double *alloc_arr(size_t np) {
  double *p = (double *)malloc(np * sizeof(double));
  if (p) memset(p, 0, np * sizeof(double));
  return p;
}

#define FOR_ALL_ARRAYS(X)                                   \
  do {                                                      \
    int q_, d_, c_;                                         \
    for (q_ = 0; q_ < NQ; q_++) {                           \
      X(b->U[q_]);                                          \
      X(b->U0[q_]);                                         \
      X(b->R[q_]);                                          \
    }                                                       \
    for (d_ = 0; d_ < 3; d_++) {                            \
      X(b->B[d_]);                                          \
      X(b->B0[d_]);                                         \
      X(b->Bc[d_]);                                         \
      X(b->Ec[d_]);                                         \
      X(b->FM[d_]);                                         \
      X(b->ED[d_]);                                         \
      X(b->RB[d_]);                                         \
      for (q_ = 0; q_ < NQ; q_++) X(b->FH[d_][q_]);         \
      for (c_ = 0; c_ < 3; c_++) X(b->EF[d_][c_]);          \
      for (c_ = 0; c_ < 2; c_++) X(b->SP[d_][c_]);          \
    }                                                       \
    for (q_ = 0; q_ < 8; q_++) X(b->W[q_]);                 \
  } while (0)

orc_box *orc_box_new(const int n[3], const double lo[3], const double hi[3],
                     const int bc[3], double gamma, double cfl, double pfloor) {
  int d;
  for (d = 0; d < 3; d++) {
    if (n[d] < 1 || !(hi[d] > lo[d])) return NULL;
    if (bc[d] != ORC_BC_PERIODIC && bc[d] != ORC_BC_OUTFLOW) return NULL;
  }
  if (!(gamma > 1.0) || !(cfl > 0.0)) return NULL;
  /* a box with no axis of more than one cell has no wave speed, so the CFL
     step is undefined: rejected */
  if (n[0] == 1 && n[1] == 1 && n[2] == 1) return NULL;
  orc_box *b = (orc_box *)calloc(1, sizeof(orc_box));
  if (!b) return NULL;
  for (d = 0; d < 3; d++) {
    b->n[d] = n[d];
    b->bc[d] = bc[d];
    b->active[d] = n[d] > 1;
    b->rk = 2;
    b->solver = ORC_HLLD;
    b->rec = ORC_REC_PRIM;
    b->emf = ORC_EMF_CONTACT;
    b->lim = ORC_LIM_MINMOD;
    b->dx[d] = (hi[d] - lo[d]) / (double)n[d];
  }
  b->gamma = gamma;
  b->cfl = cfl;
  b->pfloor = pfloor > 0.0 ? pfloor : 1.0e-10;
  b->sx = n[0] + 2 * NG + 1;
  b->sy = n[1] + 2 * NG + 1;
  b->sz = n[2] + 2 * NG + 1;
  b->np = (size_t)b->sx * (size_t)b->sy * (size_t)b->sz;
  int fail = 0;
#define ALLOC_ONE(p)                  \
  do {                                \
    (p) = alloc_arr(b->np);           \
    if (!(p)) fail = 1;               \
  } while (0)
  FOR_ALL_ARRAYS(ALLOC_ONE);
#undef ALLOC_ONE
  if (fail) {
    orc_box_free(b);
    return NULL;
  }
  return b;
}

void orc_box_free(orc_box *b) {
  if (!b) return;
#define FREE_ONE(p) free(p)
  FOR_ALL_ARRAYS(FREE_ONE);
#undef FREE_ONE
  free(b);
}

/* boundary-layout strides */
static size_t cell_off(const orc_box *b, int i, int j, int k) {
  return ((size_t)k * b->n[1] + j) * b->n[0] + i;
}
static size_t face_off(const orc_box *b, int d, int i, int j, int k) {
  int nx = b->n[0] + (d == 0), ny = b->n[1] + (d == 1);
  return ((size_t)k * ny + j) * nx + i;
}

int orc_set_state(orc_box *b, const double *const cons[5],
                  const double *const bface[3], double t) {
  int i, j, k, q, d;
  for (d = 0; d < 3; d++) {
    if (b->bc[d] != ORC_BC_PERIODIC) continue;
    /* last face must equal the first on periodic axes */
    int ext[3] = {b->n[0], b->n[1], b->n[2]};
    ext[d] = 1;
    for (k = 0; k < ext[2]; k++)
      for (j = 0; j < ext[1]; j++)
        for (i = 0; i < ext[0]; i++) {
          int p0[3] = {i, j, k}, p1[3] = {i, j, k};
          p1[d] = b->n[d];
          if (bface[d][face_off(b, d, p0[0], p0[1], p0[2])] !=
              bface[d][face_off(b, d, p1[0], p1[1], p1[2])])
            return -1;
        }
  }
  for (k = 0; k < b->n[2]; k++)
    for (j = 0; j < b->n[1]; j++)
      for (i = 0; i < b->n[0]; i++)
        for (q = 0; q < NQ; q++) b->U[q][IX(b, i, j, k)] = cons[q][cell_off(b, i, j, k)];
  for (d = 0; d < 3; d++) {
    int ex = b->n[0] + (d == 0), ey = b->n[1] + (d == 1), ez = b->n[2] + (d == 2);
    for (k = 0; k < ez; k++)
      for (j = 0; j < ey; j++)
        for (i = 0; i < ex; i++) b->B[d][IX(b, i, j, k)] = bface[d][face_off(b, d, i, j, k)];
  }
  b->t = t;
  b->nfloor = b->nhll = b->nbad = 0;
  return 0;
}

void orc_get_state(const orc_box *b, double *const cons[5],
                   double *const bface[3], double *t) {
  int i, j, k, q, d;
  for (k = 0; k < b->n[2]; k++)
    for (j = 0; j < b->n[1]; j++)
      for (i = 0; i < b->n[0]; i++)
        for (q = 0; q < NQ; q++) cons[q][cell_off(b, i, j, k)] = b->U[q][IX(b, i, j, k)];
  for (d = 0; d < 3; d++) {
    int ex = b->n[0] + (d == 0), ey = b->n[1] + (d == 1), ez = b->n[2] + (d == 2);
    for (k = 0; k < ez; k++)
      for (j = 0; j < ey; j++)
        for (i = 0; i < ex; i++) bface[d][face_off(b, d, i, j, k)] = b->B[d][IX(b, i, j, k)];
  }
  if (t) *t = b->t;
}

void orc_counters(const orc_box *b, long long counters[3]) {
  counters[0] = b->nfloor;
  counters[1] = b->nhll;
  counters[2] = b->nbad;
}

/* ------------------------------------------------------------------ */
/* boundary conditions (ghost fill)                                    */
/* ------------------------------------------------------------------ */

/* source index along an axis for a ghost cell position */
static int ghost_src(const orc_box *b, int a, int i) {
  int n = b->n[a];
  if (b->bc[a] == ORC_BC_PERIODIC) {
    while (i < 0) i += n;
    while (i >= n) i -= n;
    return i;
  }
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

/* Fill ghost layers of a cell-centred (or tangentially placed face) array
 * along axis a, over the full padded extent of the other axes.  nmax is the
 * number of interior positions along a (n_a for cells). */
static void fill_cells_axis(orc_box *b, double *arr, int a) {
  int lo[3], hi[3], d;
  for (d = 0; d < 3; d++) {
    lo[d] = -NG;
    hi[d] = b->n[d] + NG; /* exclusive; includes the extra face slot */
  }
#pragma omp parallel for schedule(static)
  for (int k = lo[2]; k < hi[2]; k++) {
    int pos[3];
    pos[2] = k;
    for (pos[1] = lo[1]; pos[1] < hi[1]; pos[1]++)
      for (pos[0] = lo[0]; pos[0] < hi[0]; pos[0]++) {
        int p = pos[a];
        if (p >= 0 && p < b->n[a]) continue;
        int src[3] = {pos[0], pos[1], pos[2]};
        src[a] = ghost_src(b, a, p);
        arr[IXp(b, pos)] = arr[IXp(b, src)];
      }
  }
}

/* Fill ghost faces of the normal field B_a along its own axis: periodic wrap
 * (face n == face 0); outflow ghosts are never read and are set to NaN so
 * that any use shows in the tests. */
static void fill_faces_normal(orc_box *b, double *arr, int a) {
  int lo[3], hi[3], d;
  for (d = 0; d < 3; d++) {
    lo[d] = -NG;
    hi[d] = b->n[d] + NG;
  }
  hi[a] = b->n[a] + NG + 1;
  int n = b->n[a];
#pragma omp parallel for schedule(static)
  for (int k = lo[2]; k < hi[2]; k++) {
    int pos[3];
    pos[2] = k;
    for (pos[1] = lo[1]; pos[1] < hi[1]; pos[1]++)
      for (pos[0] = lo[0]; pos[0] < hi[0]; pos[0]++) {
        int p = pos[a];
        if (p >= 0 && p <= n) continue;
        if (b->bc[a] == ORC_BC_PERIODIC) {
          int src[3] = {pos[0], pos[1], pos[2]};
          int s = p;
          while (s < 0) s += n;
          while (s > n) s -= n;
          src[a] = s;
          arr[IXp(b, pos)] = arr[IXp(b, src)];
        } else {
          arr[IXp(b, pos)] = NAN;
        }
      }
  }
}

/* Stage-start preparation: cell-centred field, ghost cells, primitives and
 * cell EMFs over the whole padded domain. */
static void prepare(orc_box *b) {
  int q, a, d;
#pragma omp parallel for schedule(static)
  for (int k = 0; k < b->n[2]; k++)
    for (int j = 0; j < b->n[1]; j++)
      for (int i = 0; i < b->n[0]; i++) {
        size_t c = IX(b, i, j, k);
        b->Bc[0][c] = 0.5 * (b->B[0][c] + b->B[0][IX(b, i + 1, j, k)]);
        b->Bc[1][c] = 0.5 * (b->B[1][c] + b->B[1][IX(b, i, j + 1, k)]);
        b->Bc[2][c] = 0.5 * (b->B[2][c] + b->B[2][IX(b, i, j, k + 1)]);
      }
  for (a = 0; a < 3; a++) {
    for (q = 0; q < NQ; q++) fill_cells_axis(b, b->U[q], a);
    for (d = 0; d < 3; d++) fill_cells_axis(b, b->Bc[d], a);
    for (d = 0; d < 3; d++) {
      if (d == a)
        fill_faces_normal(b, b->B[d], a);
      else
        fill_cells_axis(b, b->B[d], a);
    }
  }
  /* primitives and cell EMF everywhere (ghosts hold copies, so their
   * primitives equal those of their source cells); counters on interior
   * cells only */
  long long nfloor = 0, nbad = 0;
#pragma omp parallel for schedule(static) reduction(+ : nfloor, nbad)
  for (int k = -NG; k < b->n[2] + NG; k++)
    for (int j = -NG; j < b->n[1] + NG; j++)
      for (int i = -NG; i < b->n[0] + NG; i++) {
        size_t c = IX(b, i, j, k);
        double u[5], bcv[3], w[8];
        for (int m = 0; m < NQ; m++) u[m] = b->U[m][c];
        for (int e = 0; e < 3; e++) bcv[e] = b->Bc[e][c];
        int fl = orc_cons_to_prim(u, bcv, b->gamma, b->pfloor, w);
        if (i >= 0 && i < b->n[0] && j >= 0 && j < b->n[1] && k >= 0 && k < b->n[2]) {
          if (fl & 1) nfloor++;
          if (fl & 2) nbad++;
        }
        for (int m = 0; m < 8; m++) b->W[m][c] = w[m];
        /* E = -v x B */
        b->Ec[0][c] = w[3] * w[6] - w[2] * w[7];
        b->Ec[1][c] = w[1] * w[7] - w[3] * w[5];
        b->Ec[2][c] = w[2] * w[5] - w[1] * w[6];
      }
  b->nfloor += nfloor;
  b->nbad += nbad;
}

/* Face fluxes along direction d for faces 0..n_d and transverse cells
 * -1..n_t.  Active axis: PLM-minmod + HLLD.  Inactive axis: physical flux of
 * the cell, i.e. EMFs = cell EMF and mass flux = momentum. */
static void sweep(orc_box *b, int d) {
  int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
  /* face-frame primitive slots in W: rho, v_n, v_t1, v_t2, p, B_t1, B_t2 */
  int slot[7] = {0, 1 + d, 1 + t1, 1 + t2, 4, 5 + t1, 5 + t2};
  int lo[3], hi[3], a;
  for (a = 0; a < 3; a++) {
    lo[a] = -1;
    hi[a] = b->n[a] + 1; /* exclusive: -1..n */
  }
  lo[d] = 0;
  hi[d] = b->n[d] + 1; /* faces 0..n_d */
  long long nhll = 0;
#pragma omp parallel for schedule(static) reduction(+ : nhll)
  for (int k = lo[2]; k < hi[2]; k++) {
    int pos[3];
    pos[2] = k;
    for (pos[1] = lo[1]; pos[1] < hi[1]; pos[1]++)
      for (pos[0] = lo[0]; pos[0] < hi[0]; pos[0]++) {
        size_t fidx = IXp(b, pos);
        if (!b->active[d]) {
          /* cell "pos" (its ghost copy for pos[d] == n_d) */
          b->EF[d][t1][fidx] = b->Ec[t1][fidx];
          b->EF[d][t2][fidx] = b->Ec[t2][fidx];
          b->FM[d][fidx] = b->U[1 + d][fidx];
          for (int q = 0; q < NQ; q++) b->FH[d][q][fidx] = 0.0;
          continue;
        }
        /* stencil cells c-2, c-1, c, c+1 along d, face = lower face of c */
        size_t cs[4];
        for (int s = 0; s < 4; s++) {
          int p2[3] = {pos[0], pos[1], pos[2]};
          p2[d] += s - 2;
          cs[s] = IXp(b, p2);
        }
        double wl[7], wr[7];
        if (b->rec == ORC_REC_PRIM && b->lim == ORC_LIM_MINMOD) {
          for (int v = 0; v < 7; v++) {
            double *q = b->W[slot[v]];
            orc_plm_face(q[cs[0]], q[cs[1]], q[cs[2]], q[cs[3]], &wl[v], &wr[v]);
          }
        } else {
          /* slopes of the two cells next to the face (in the characteristic
           * fields of each cell's own state for ORC_REC_CHAR) */
          double qs[4][7], s1[7], s2[7];
          for (int m = 0; m < 4; m++)
            for (int v = 0; v < 7; v++) qs[m][v] = b->W[slot[v]][cs[m]];
          orc_slope(qs[0], qs[1], qs[2], b->W[5 + d][cs[1]], b->gamma, b->rec, b->lim, s1);
          orc_slope(qs[1], qs[2], qs[3], b->W[5 + d][cs[2]], b->gamma, b->rec, b->lim, s2);
          for (int v = 0; v < 7; v++) {
            wl[v] = qs[1][v] + 0.5 * s1[v];
            wr[v] = qs[2][v] - 0.5 * s2[v];
          }
        }
        double bn = b->B[d][fidx];
        double f[7], fm;
        int used_hll;
        if (b->solver == ORC_HLL) {
          /* HLL at every face (the paper's 2D Riemann runs use it) */
          double sl, sr;
          orc_hll(wl, wr, bn, b->gamma, f);
          wave_speeds(wl, wr, bn, b->gamma, &sl, &sr);
          fm = ct_mass_flux(f[0], wl, wr, sl, sr);
          used_hll = 0;
        } else {
          used_hll = riemann(wl, wr, bn, b->gamma, f, &fm);
        }
        /* count each distinct interior face once */
        int interior = 1;
        for (int e = 0; e < 3; e++) {
          if (e == d) {
            int nf = b->bc[d] == ORC_BC_PERIODIC ? b->n[d] : b->n[d] + 1;
            if (pos[e] >= nf) interior = 0;
          } else if (pos[e] < 0 || pos[e] >= b->n[e]) {
            interior = 0;
          }
        }
        if (used_hll && interior) nhll++;
        b->FH[d][0][fidx] = f[0];
        b->FH[d][1 + d][fidx] = f[1];
        b->FH[d][1 + t1][fidx] = f[2];
        b->FH[d][1 + t2][fidx] = f[3];
        b->FH[d][4][fidx] = f[4];
        /* flux of B_t1 = -E_t2, flux of B_t2 = +E_t1 */
        b->EF[d][t1][fidx] = f[6];
        b->EF[d][t2][fidx] = -f[5];
        b->FM[d][fidx] = fm;
        if (b->emf == ORC_EMF_UCT_HLL) {
          double sl, sr;
          wave_speeds(wl, wr, bn, b->gamma, &sl, &sr);
          b->SP[d][0][fidx] = sl;
          b->SP[d][1][fidx] = sr;
        }
      }
  }
  b->nhll += nhll;
}

/* Value of q at the side of a cell facing the corner: the cell value q0
 * carried half a cell up (side 0, the cell lies below the corner) or down
 * (side 1) with the limited slope of q0 between its neighbours qm and qp;
 * no slope along an inactive axis. */
static double to_corner(const orc_box *b, int active, int side, double qm, double q0,
                        double qp) {
  double d = active ? orc_limit(b->lim, q0 - qm, qp - q0) : 0.0;
  return side == 0 ? q0 + 0.5 * d : q0 - 0.5 * d;
}

/* Upper bound of the right-going (left-going when left != 0) signal speed
 * at a corner from the outer wave speeds of its two faces, at least 0 */
static double speed_bound(double s0, double s1, int left) {
  if (left) {
    double m = s0 < s1 ? s0 : s1;
    return m < 0.0 ? -m : 0.0;
  }
  double m = s0 > s1 ? s0 : s1;
  return m > 0.0 ? m : 0.0;
}

double orc_uct_hll(const double va[4], const double vb[4], const double ba[2],
                   const double bb[2], const double alpha[4]) {
  double apa = alpha[0], ama = alpha[1], apb = alpha[2], amb = alpha[3];
  double e[4];
  int k;
  /* E_c = v_b B_a - v_a B_b of each corner state */
  for (k = 0; k < 4; k++) e[k] = vb[k] * ba[k >> 1] - va[k] * bb[k & 1];
  /* HLL along both axes: the lower state of an axis is weighted by the
   * right-going bound, the upper state by the left-going one; each axis adds
   * the HLL diffusion of the field component it carries (the flux of B_a
   * along b is E_c, the flux of B_b along a is -E_c) */
  double num = apa * apb * e[0] + ama * apb * e[1] + apa * amb * e[2] + ama * amb * e[3];
  double sa = apa + ama, sb = apb + amb;
  return num / (sa * sb) - apb * amb / sb * (ba[1] - ba[0]) +
         apa * ama / sa * (bb[1] - bb[0]);
}

/* Upwind-CT corner EMF along c at corner position pos (a-face index ia =
 * pos[a], b-face index ib = pos[b]): the four cells around the edge give
 * the corner states (velocities carried to the corner with their limited
 * slopes along a and b), the a-faces (ia; ib-1), (ia; ib) and the b-faces
 * (ib; ia-1), (ib; ia) give the field carried along the other axis and the
 * speed bounds.  An inactive axis has equal states on both sides; its
 * weights are 1. */
static double uct_corner(const orc_box *b, int c, const int pos[3]) {
  int a = (c + 1) % 3, bb = (c + 2) % 3;
  int ax[2] = {a, bb};
  double alpha[4] = {1.0, 1.0, 1.0, 1.0};
  for (int e = 0; e < 2; e++) {
    int d = ax[e], t = ax[1 - e];
    if (!b->active[d]) continue;
    int p0[3] = {pos[0], pos[1], pos[2]};
    p0[t] -= 1;
    size_t i0 = IXp(b, p0), i1 = IXp(b, pos);
    alpha[2 * e] = speed_bound(b->SP[d][1][i0], b->SP[d][1][i1], 0);
    alpha[2 * e + 1] = speed_bound(b->SP[d][0][i0], b->SP[d][0][i1], 1);
  }
  double va[4], vb[4], fa[2], fb[2];
  for (int k = 0; k < 4; k++) {
    int sa = k & 1, sb = k >> 1;
    int pc[3] = {pos[0], pos[1], pos[2]}; /* cell (ia-1+sa, ib-1+sb) */
    pc[a] += sa - 1;
    pc[bb] += sb - 1;
    int am[3] = {pc[0], pc[1], pc[2]}, ap[3] = {pc[0], pc[1], pc[2]};
    int bm[3] = {pc[0], pc[1], pc[2]}, bp[3] = {pc[0], pc[1], pc[2]};
    am[a] -= 1;
    ap[a] += 1;
    bm[bb] -= 1;
    bp[bb] += 1;
    for (int e = 0; e < 2; e++) {
      const double *q = b->W[1 + ax[e]];
      double q0 = q[IXp(b, pc)];
      /* half the a slope, then half the b slope of the same cell */
      double x = to_corner(b, b->active[a], sa, q[IXp(b, am)], q0, q[IXp(b, ap)]);
      double db = b->active[bb] ? orc_limit(b->lim, q0 - q[IXp(b, bm)], q[IXp(b, bp)] - q0) : 0.0;
      x = sb == 0 ? x + 0.5 * db : x - 0.5 * db;
      if (e == 0)
        va[k] = x;
      else
        vb[k] = x;
    }
  }
  for (int s2 = 0; s2 < 2; s2++) {
    /* a-face field at (ia; ib-1+s2), carried along b */
    int pf[3] = {pos[0], pos[1], pos[2]};
    pf[bb] += s2 - 1;
    int fm[3] = {pf[0], pf[1], pf[2]}, fp[3] = {pf[0], pf[1], pf[2]};
    fm[bb] -= 1;
    fp[bb] += 1;
    const double *qa = b->B[a];
    fa[s2] = to_corner(b, b->active[bb], s2, qa[IXp(b, fm)], qa[IXp(b, pf)], qa[IXp(b, fp)]);
    /* b-face field at (ib; ia-1+s2), carried along a */
    int pg[3] = {pos[0], pos[1], pos[2]};
    pg[a] += s2 - 1;
    int gm[3] = {pg[0], pg[1], pg[2]}, gp[3] = {pg[0], pg[1], pg[2]};
    gm[a] -= 1;
    gp[a] += 1;
    const double *qb = b->B[bb];
    fb[s2] = to_corner(b, b->active[a], s2, qb[IXp(b, gm)], qb[IXp(b, pg)], qb[IXp(b, gp)]);
  }
  return orc_uct_hll(va, vb, fa, fb, alpha);
}

/* corner EMFs along c at a-faces 0..n_a, b-faces 0..n_b, c cells 0..n_c-1 */
static void corner_emfs(orc_box *b, int c) {
  int a = (c + 1) % 3, bb = (c + 2) % 3;
  int lo[3] = {0, 0, 0}, hi[3];
  hi[a] = b->n[a] + 1;
  hi[bb] = b->n[bb] + 1;
  hi[c] = b->n[c];
#pragma omp parallel for schedule(static)
  for (int k = lo[2]; k < hi[2]; k++) {
    int pos[3];
    pos[2] = k;
    for (pos[1] = lo[1]; pos[1] < hi[1]; pos[1]++)
      for (pos[0] = lo[0]; pos[0] < hi[0]; pos[0]++) {
        int pa[3] = {pos[0], pos[1], pos[2]}; /* a-face (ia, ib-1) */
        pa[bb] -= 1;
        int pb[3] = {pos[0], pos[1], pos[2]}; /* b-face (ib, ia-1) */
        pb[a] -= 1;
        int pab[3] = {pos[0], pos[1], pos[2]}; /* cell (ia-1, ib-1) */
        pab[a] -= 1;
        pab[bb] -= 1;
        size_t i11 = IXp(b, pos), ia0 = IXp(b, pa), ib0 = IXp(b, pb), i00 = IXp(b, pab);
        if (b->emf == ORC_EMF_UCT_HLL) {
          b->ED[c][i11] = uct_corner(b, c, pos);
          continue;
        }
        double fa1 = b->EF[a][c][i11], fa0 = b->EF[a][c][ia0];
        double fb1 = b->EF[bb][c][i11], fb0 = b->EF[bb][c][ib0];
        /* cells: oa = 0 -> ia-1, ob = 0 -> ib-1 */
        double ec[4];
        ec[0] = b->Ec[c][i00]; /* (ia-1, ib-1) */
        ec[1] = b->Ec[c][ia0]; /* (ia, ib-1)   */
        ec[2] = b->Ec[c][ib0]; /* (ia-1, ib)   */
        ec[3] = b->Ec[c][i11]; /* (ia, ib)     */
        b->ED[c][i11] = orc_ct_corner_kind(b->emf, fa1, fa0, fb1, fb0, ec, b->FM[a][i11],
                                           b->FM[a][ia0], b->FM[bb][i11], b->FM[bb][ib0]);
      }
  }
}

/* Stage operator: R (interior cells) and RB (faces). */
static void stage_operator(orc_box *b) {
  int d;
  prepare(b);
  for (d = 0; d < 3; d++) sweep(b, d);
#pragma omp parallel for schedule(static)
  for (int k = 0; k < b->n[2]; k++)
    for (int j = 0; j < b->n[1]; j++)
      for (int i = 0; i < b->n[0]; i++) {
        size_t c = IX(b, i, j, k);
        size_t up[3] = {IX(b, i + 1, j, k), IX(b, i, j + 1, k), IX(b, i, j, k + 1)};
        for (int m = 0; m < NQ; m++) {
          double r = 0.0;
          for (int e = 0; e < 3; e++) {
            if (!b->active[e]) continue;
            r = r - (b->FH[e][m][up[e]] - b->FH[e][m][c]) / b->dx[e];
          }
          b->R[m][c] = r;
        }
      }
  for (d = 0; d < 3; d++) corner_emfs(b, d);
  /* face rate: dB_d/dt = -[(E_f(e+1/2)-E_f(e-1/2))/dx_e - (E_e(f+1/2)-E_e(f-1/2))/dx_f] */
  for (d = 0; d < 3; d++) {
    int e = (d + 1) % 3, f = (d + 2) % 3;
    int hi[3] = {b->n[0], b->n[1], b->n[2]};
    hi[d] = b->n[d] + 1;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < hi[2]; k++) {
      int pos[3];
      pos[2] = k;
      for (pos[1] = 0; pos[1] < hi[1]; pos[1]++)
        for (pos[0] = 0; pos[0] < hi[0]; pos[0]++) {
          int pe[3] = {pos[0], pos[1], pos[2]};
          pe[e] += 1;
          int pf[3] = {pos[0], pos[1], pos[2]};
          pf[f] += 1;
          size_t c0 = IXp(b, pos);
          double t1 = 0.0, t2 = 0.0;
          if (b->active[e]) t1 = (b->ED[f][IXp(b, pe)] - b->ED[f][c0]) / b->dx[e];
          if (b->active[f]) t2 = (b->ED[e][IXp(b, pf)] - b->ED[e][c0]) / b->dx[f];
          b->RB[d][c0] = -(t1 - t2);
        }
    }
  }
}

double orc_dt(orc_box *b) {
  double lmax = 0.0;
  /* the maximum is independent of the order of the cells */
#pragma omp parallel for schedule(static) reduction(max : lmax)
  for (int k = 0; k < b->n[2]; k++)
    for (int j = 0; j < b->n[1]; j++)
      for (int i = 0; i < b->n[0]; i++) {
        size_t c = IX(b, i, j, k);
        double u[5], bcv[3], w[8];
        for (int q = 0; q < NQ; q++) u[q] = b->U[q][c];
        bcv[0] = 0.5 * (b->B[0][c] + b->B[0][IX(b, i + 1, j, k)]);
        bcv[1] = 0.5 * (b->B[1][c] + b->B[1][IX(b, i, j + 1, k)]);
        bcv[2] = 0.5 * (b->B[2][c] + b->B[2][IX(b, i, j, k + 1)]);
        orc_cons_to_prim(u, bcv, b->gamma, b->pfloor, w);
        for (int d = 0; d < 3; d++) {
          if (!b->active[d]) continue;
          int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
          double cf = orc_fast_speed(w[0], w[4], w[5 + d], w[5 + t1], w[5 + t2], b->gamma);
          double l = (fabs(w[1 + d]) + cf) / b->dx[d];
          if (l > lmax) lmax = l;
        }
      }
  return b->cfl / lmax;
}

/* Stage combine of the strong-stability-preserving Runge-Kutta schemes of
 * Shu & Osher (1988), with L the stage operator just evaluated and U0 the
 * state at the start of the step:
 *   first stage (both):   U = U0 + dt L
 *   RK2, second stage:    U = 1/2 (U0 + (U + dt L))
 *   RK3, second stage:    U = 3/4 U0 + 1/4 (U + dt L)
 *   RK3, third stage:     U = 1/3 U0 + 2/3 (U + dt L)
 * (kind 0, 1, 2, 3 below; the RK3 weights are the double nearest 3/4, 1/4,
 * 1/3, 2/3, in the form a U0 + b (U + dt L)). */
static double combine(int kind, double u0, double u, double dtl) {
  switch (kind) {
    case 0: return u0 + dtl;
    case 1: return 0.5 * (u0 + (u + dtl));
    case 2: return 0.75 * u0 + 0.25 * (u + dtl);
    default: return (1.0 / 3.0) * u0 + (2.0 / 3.0) * (u + dtl);
  }
}

static void stage_update(orc_box *b, double dt, int kind) {
  int d;
#pragma omp parallel for schedule(static)
  for (int k = 0; k < b->n[2]; k++)
    for (int j = 0; j < b->n[1]; j++)
      for (int i = 0; i < b->n[0]; i++) {
        size_t c = IX(b, i, j, k);
        for (int q = 0; q < NQ; q++)
          b->U[q][c] = combine(kind, b->U0[q][c], b->U[q][c], dt * b->R[q][c]);
      }
  for (d = 0; d < 3; d++) {
    int ex = b->n[0] + (d == 0), ey = b->n[1] + (d == 1), ez = b->n[2] + (d == 2);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < ez; k++)
      for (int j = 0; j < ey; j++)
        for (int i = 0; i < ex; i++) {
          size_t c = IX(b, i, j, k);
          b->B[d][c] = combine(kind, b->B0[d][c], b->B[d][c], dt * b->RB[d][c]);
        }
  }
}

static void save_start(orc_box *b) {
  int q, d;
  for (q = 0; q < NQ; q++) memcpy(b->U0[q], b->U[q], b->np * sizeof(double));
  for (d = 0; d < 3; d++) memcpy(b->B0[d], b->B[d], b->np * sizeof(double));
}

void orc_step_fixed_dt(orc_box *b, double dt) {
  save_start(b);
  stage_operator(b);
  stage_update(b, dt, 0);
  if (b->rk == 3) {
    stage_operator(b);
    stage_update(b, dt, 2);
    stage_operator(b);
    stage_update(b, dt, 3);
  } else {
    stage_operator(b);
    stage_update(b, dt, 1);
  }
  b->t = b->t + dt;
}

int orc_set_rk(orc_box *b, int stages) {
  if (stages != 2 && stages != 3) return -1;
  b->rk = stages;
  return 0;
}

int orc_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

int orc_set_limiter(orc_box *b, int lim) {
  if (lim != ORC_LIM_MINMOD && lim != ORC_LIM_MC && lim != ORC_LIM_VANLEER) return -1;
  b->lim = lim;
  return 0;
}

int orc_set_emf(orc_box *b, int emf) {
  if (emf != ORC_EMF_CONTACT && emf != ORC_EMF_E0 && emf != ORC_EMF_ARITH &&
      emf != ORC_EMF_UCT_HLL)
    return -1;
  b->emf = emf;
  return 0;
}

int orc_set_recon(orc_box *b, int rec) {
  if (rec != ORC_REC_PRIM && rec != ORC_REC_CHAR) return -1;
  b->rec = rec;
  return 0;
}

int orc_set_solver(orc_box *b, int solver) {
  if (solver != ORC_HLLD && solver != ORC_HLL) return -1;
  b->solver = solver;
  return 0;
}

void orc_step(orc_box *b, int nsteps, double t_stop) {
  int s;
  for (s = 0; s < nsteps; s++) {
    double dt = orc_dt(b);
    if (t_stop > 0.0) {
      double rem = t_stop - b->t;
      if (rem < dt) dt = rem;
      if (dt < 0.0) dt = 0.0;
    }
    orc_step_fixed_dt(b, dt);
  }
}

void orc_rhs(orc_box *b, double *const R[5], double *const rB[3]) {
  int i, j, k, q, d;
  stage_operator(b);
  for (k = 0; k < b->n[2]; k++)
    for (j = 0; j < b->n[1]; j++)
      for (i = 0; i < b->n[0]; i++)
        for (q = 0; q < NQ; q++) R[q][cell_off(b, i, j, k)] = b->R[q][IX(b, i, j, k)];
  for (d = 0; d < 3; d++) {
    int ex = b->n[0] + (d == 0), ey = b->n[1] + (d == 1), ez = b->n[2] + (d == 2);
    for (k = 0; k < ez; k++)
      for (j = 0; j < ey; j++)
        for (i = 0; i < ex; i++) rB[d][face_off(b, d, i, j, k)] = b->RB[d][IX(b, i, j, k)];
  }
}

double orc_divb_max(const orc_box *b) {
  double m = 0.0;
#pragma omp parallel for schedule(static) reduction(max : m)
  for (int k = 0; k < b->n[2]; k++)
    for (int j = 0; j < b->n[1]; j++)
      for (int i = 0; i < b->n[0]; i++) {
        size_t c = IX(b, i, j, k);
        double dv = (b->B[0][IX(b, i + 1, j, k)] - b->B[0][c]) / b->dx[0] +
                    (b->B[1][IX(b, i, j + 1, k)] - b->B[1][c]) / b->dx[1] +
                    (b->B[2][IX(b, i, j, k + 1)] - b->B[2][c]) / b->dx[2];
        if (fabs(dv) > m) m = fabs(dv);
      }
  return m;
}
