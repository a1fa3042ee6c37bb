/*
 * mhd_oracle.h -- interface of the CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, serial, FP64 C implementation
 * of the ideal-MHD finite-volume update that the GPU library is checked
 * against.  Only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark load it.  It shares no code, header, table or constant
 * generator with the GPU library.
 *
 * The scheme is the main cycle of arXiv 2606.12753 §2.2.3: per-direction
 * reconstruction of primitive variables, a Riemann solve at every interface,
 * a flux-conservative update, constrained transport for the magnetic field and
 * Runge-Kutta time stepping (here the two-stage SSP form).  The component
 * algorithms are the published ones named in mhd_oracle.c.
 *
 * Array layout at this interface (the "boundary layout"): C order [z][y][x],
 * x fastest.  Cell arrays hold nz*ny*nx doubles.  Face arrays hold both
 * bounding faces of every cell: Bx nz*ny*(nx+1), By nz*(ny+1)*nx,
 * Bz (nz+1)*ny*nx.  On periodic axes the last face must equal the first.
 */
#ifndef MHD_ORACLE_H
#define MHD_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_BC_PERIODIC 0
#define ORC_BC_OUTFLOW 1

typedef struct orc_box orc_box;

/* n[3] cells per axis (n==1: inactive axis; at least one axis active), lo/hi
 * domain corners, bc[3] per axis (both sides alike), gamma, CFL number,
 * pressure floor.  NULL on bad arguments or out of memory. */
orc_box *orc_box_new(const int n[3], const double lo[3], const double hi[3],
                     const int bc[3], double gamma, double cfl, double pfloor);
void orc_box_free(orc_box *b);

/* Copies the state in/out (boundary layout).  set returns 0, or -1 when a
 * periodic axis has last face != first face. */
int orc_set_state(orc_box *b, const double *const cons[5],
                  const double *const bface[3], double t);
void orc_get_state(const orc_box *b, double *const cons[5],
                   double *const bface[3], double *t);

/* Advances nsteps full Runge-Kutta steps (SSP-RK2 unless orc_set_rk chose
 * SSP-RK3) with the CFL time step of each step's starting state (clamped to
 * t_stop - t when t_stop > 0). */
void orc_step(orc_box *b, int nsteps, double t_stop);
/* Threads of the cell and face loops (OpenMP; each output element is
 * computed by one thread in the serial order of its own terms, counters are
 * integer sums and the time step a maximum, so results are identical for any
 * count).  n > 0 sets the count; returns the count in use (1 without
 * OpenMP). */
int orc_threads(int n);
/* Integrator: 2 (SSP-RK2, the default) or 3 (SSP-RK3) stages; -1 otherwise. */
int orc_set_rk(orc_box *b, int stages);
/* Riemann solver of every face: ORC_HLLD (the default; HLL where the HLLD
 * star states are not physical) or ORC_HLL (HLL everywhere); -1 otherwise. */
#define ORC_HLLD 0
#define ORC_HLL 1
int orc_set_solver(orc_box *b, int solver);
/* Variables the PLM slopes are limited in: ORC_REC_PRIM (the default,
 * primitive variables) or ORC_REC_CHAR (characteristic fields of each
 * cell's state, see orc_slope); -1 otherwise. */
#define ORC_REC_PRIM 0
#define ORC_REC_CHAR 1
int orc_set_recon(orc_box *b, int rec);
/* Corner EMF of the constrained transport: ORC_EMF_CONTACT (the default,
 * contact-upwinded average, see orc_ct_corner), ORC_EMF_E0 (the same
 * average with both sides of every derivative averaged), ORC_EMF_ARITH
 * (mean of the four face EMFs) or ORC_EMF_UCT_HLL (upwind CT: the
 * two-dimensional HLL flux of the four reconstructed corner states, see
 * orc_uct_hll); -1 otherwise. */
#define ORC_EMF_CONTACT 0
#define ORC_EMF_E0 1
#define ORC_EMF_ARITH 2
#define ORC_EMF_UCT_HLL 3
int orc_set_emf(orc_box *b, int emf);
double orc_ct_corner_kind(int kind, double fa1, double fa0, double fb1, double fb0,
                          const double ec[4], double ma1, double ma0, double mb1,
                          double mb0);
/* Point functions of the characteristic reconstruction (pinned by tests). */
void orc_prim_eigen(const double w[7], double bn, double gamma, double lam[7],
                    double R[7][7], double L[7][7]);
void orc_slope(const double qm[7], const double q0[7], const double qp[7], double bn,
               double gamma, int rec, int lim, double d[7]);
/* Slope limiter of the PLM reconstruction: ORC_LIM_MINMOD (the default),
 * ORC_LIM_MC (monotonised central) or ORC_LIM_VANLEER (harmonic); -1
 * otherwise.  orc_limit is the limiter as a point function. */
#define ORC_LIM_MINMOD 0
#define ORC_LIM_MC 1
#define ORC_LIM_VANLEER 2
int orc_set_limiter(orc_box *b, int lim);
double orc_limit(int lim, double a, double b);
/* One step with a caller-given dt (used for sampled parity on sub-boxes). */
void orc_step_fixed_dt(orc_box *b, double dt);
/* CFL time step of the current state (no t_stop clamp). */
double orc_dt(orc_box *b);
/* Stage operator L(U,B) of the current state: cell residual R[5] (cell
 * layout) and face rates rB[3] (boundary face layout). */
void orc_rhs(orc_box *b, double *const R[5], double *const rB[3]);
/* counters[0] = pressure-floor hits, [1] = HLL fallbacks, [2] = bad cells
 * (rho <= 0 or non-finite), accumulated since creation / last set_state. */
void orc_counters(const orc_box *b, long long counters[3]);
/* max over cells of |div B| (face differences / dx). */
double orc_divb_max(const orc_box *b);

/* ---- point functions (for the pins) ---- */
/* cons (rho, mx, my, mz, E) + cell-centred B -> prims (rho, vx, vy, vz, p,
 * bx, by, bz); returns bit0 = floor hit, bit1 = bad. */
int orc_cons_to_prim(const double u[5], const double bc[3], double gamma,
                     double pfloor, double w[8]);
double orc_fast_speed(double rho, double p, double bn, double bt1, double bt2,
                      double gamma);
double orc_minmod(double a, double b);
/* PLM interface values between cells c-1 and c from q(c-2..c+1) */
void orc_plm_face(double qm2, double qm1, double q0, double qp1, double *ql,
                  double *qr);
/* states in the face frame: (rho, vn, vt1, vt2, p, bt1, bt2), normal field bn.
 * flux out: (mass, mom n, mom t1, mom t2, energy, B t1, B t2). */
void orc_phys_flux(const double w[7], double bn, double gamma, double f[7],
                   double u[7]);
int orc_hlld(const double wl[7], const double wr[7], double bn, double gamma,
             double f[7]);
void orc_hll(const double wl[7], const double wr[7], double bn, double gamma,
             double f[7]);
/* mass flux of the face as handed to the CT upwinding (zero when it is zero
 * up to rounding, see mhd_oracle.c) */
double orc_ct_mass_flux(const double wl[7], const double wr[7], double bn,
                        double gamma);
/* Corner EMF of the contact-upwinded constrained-transport average.
 * fa1/fa0: edge-component EMF on the two a-faces (b index ib, ib-1);
 * fb1/fb0: on the two b-faces (a index ia, ia-1); ec[2][2] cell values
 * indexed [b offset][a offset] with offset 0 = lower cell; ma1/ma0 mass flux
 * on the a-faces (ib, ib-1), mb1/mb0 on the b-faces (ia, ia-1). */
double orc_ct_corner(double fa1, double fa0, double fb1, double fb0,
                     const double ec[4], double ma1, double ma0, double mb1,
                     double mb0);
/* Upwind-CT corner EMF along c = (a, b) x (Londrillo & Del Zanna 2004,
 * HLL form) from the four corner states: va[k], vb[k] the velocity
 * components along a and b of state k = 2*sb + sa (sa, sb = 0: the lower
 * side along a, b; 1: the upper side); ba[sb] the a-face field carried to
 * the corner from the lower (0) and upper (1) side along b; bb[sa] the
 * b-face field from the lower and upper side along a; alpha = {a+_a, a-_a,
 * a+_b, a-_b} the right- and left-going speed bounds (>= 0, each pair with a
 * positive sum). */
double orc_uct_hll(const double va[4], const double vb[4], const double ba[2],
                   const double bb[2], const double alpha[4]);

#ifdef __cplusplus
}
#endif
#endif
