/*
 * mhd.h -- C ABI of the MI355X ideal-MHD finite-volume library.
 *
 * The library advances the ideal-MHD conservation laws with the main cycle
 * that arXiv 2606.12753 §2.2.3 describes: per direction, reconstruction of
 * primitive variables, a Riemann solve at every interface and a
 * flux-conservative update; constrained transport (CT) for the magnetic
 * field; Runge-Kutta stepping.  Concretely: PLM reconstruction (minmod, MC
 * or van Leer slopes of primitive or characteristic variables), HLLD fluxes
 * with HLL fallback (or HLL alone), the flux-divergence update, CT corner
 * EMFs (contact-upwinded, E0 or arithmetic average, or upwind CT) with the
 * face-field
 * update, the CFL time step from a max-reduction of the fast magnetosonic
 * rate and the SSP Runge-Kutta stage combines (two or three stages), on 3D
 * structured boxes (2D and 1D as boxes with inactive axes of one cell).
 *
 * All entry points return MHD_OK (0) or a negative status and never throw,
 * abort or exit across the ABI.  A context is used by one host thread at a
 * time.  Every compute step runs in the library's HIP kernels on the current
 * HIP device of mhd_create; there is no CPU fallback.
 *
 * Array layout at this boundary (host or device memory, caller-owned):
 * C order [z][y][x], x fastest, FP64.
 *   cons[5]  = rho, m_x, m_y, m_z, E (total energy incl. |B|^2/2 of the
 *              face-averaged field); nz*ny*nx doubles each.
 *   bface[3] = face-centred B_x, B_y, B_z including both bounding faces:
 *              B_x nz*ny*(nx+1), B_y nz*(ny+1)*nx, B_z (nz+1)*ny*nx.  On a
 *              periodic axis the last face must equal the first.
 * Caller arrays are never retained past the call that receives them.
 */
#ifndef MHD_H
#define MHD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define MHD_OK 0
#define MHD_E_INVAL (-1)   /* bad argument; nothing was changed */
#define MHD_E_NOMEM (-2)   /* device allocation failed or workspace too small */
#define MHD_E_DEVICE (-3)  /* HIP runtime error or no usable device */
#define MHD_E_NONPHYS (-4) /* a cell had rho <= 0 or a non-finite state */
#define MHD_E_STATE (-5)   /* call out of order (e.g. step before set_state) */

/* boundary conditions, per axis (both sides of an axis must agree) */
#define MHD_BC_PERIODIC 0
#define MHD_BC_OUTFLOW 1 /* zero-gradient: ghosts copy the boundary cell */

/* arithmetic of the reconstruction / Riemann / EMF work */
#define MHD_FP64 0  /* everything FP64 */
#define MHD_MIXED 1 /* FP32 reconstruction, fluxes, EMFs, residual; FP64
                       state, pressure recovery, RK accumulation, dt */

/* Riemann solver of every face (the paper's 3D runs use HLLD, its 2D
 * Riemann runs HLL) */
#define MHD_RS_HLLD 0 /* HLLD (Miyoshi & Kusano 2005); HLL where its star
                         states are not physical */
#define MHD_RS_HLL 1  /* HLL (Harten, Lax & van Leer 1983) with the same
                         outer wave speeds */

/* variables the PLM slopes are limited in (with the limiter of
 * mhd_config.limiter) */
#define MHD_REC_PRIM 0 /* primitive variables */
#define MHD_REC_CHAR 1 /* characteristic fields of each cell's own state
                          (eigenvectors of the primitive-variable system,
                          Roe & Balsara 1996 normalisation); a cell whose
                          slope would give a non-positive face density or
                          pressure takes the primitive slope.  The paper
                          allows reconstruction in either variable set
                          (its section 2.2.3). */

/* slope limiter of the PLM reconstruction (in either variable set) */
#define MHD_LIM_MINMOD 0  /* minmod */
#define MHD_LIM_MC 1      /* monotonised central (van Leer 1977) */
#define MHD_LIM_VANLEER 2 /* van Leer's harmonic mean (van Leer 1974) */

/* corner EMF of the constrained transport */
#define MHD_EMF_CONTACT 0 /* contact-upwinded average (Gardiner & Stone
                             2005): face-to-corner derivatives taken on the
                             upwind side of the face's mass flux */
#define MHD_EMF_E0 1      /* their E0 average: each derivative the mean of
                             its two sides */
#define MHD_EMF_ARITH 2   /* mean of the four face EMFs (Balsara & Spicer
                             1999) */
#define MHD_EMF_UCT_HLL 3 /* upwind CT (Londrillo & Del Zanna 2004, HLL
                             form): the two-dimensional HLL flux of the four
                             corner states (cell velocities and face fields
                             carried to the corner with limited slopes),
                             with speed bounds from the outer wave speeds of
                             the adjacent faces; the face EMFs are not used.
                             Needs two more face arrays per axis. */

/* where caller arrays live */
#define MHD_HOST 0
#define MHD_DEVICE 1

/* config flags */
#define MHD_F_GRAPH 1u      /* replay each step from a captured HIP graph */
#define MHD_F_PERSISTENT 2u /* persistent-grid launches over the tile table */
#define MHD_F_TIMING 4u     /* time every kernel launch with HIP events on the
                               context stream (serialises steps; no graph) */
#define MHD_F_AUTOTUNE 8u   /* before the first step, time the launch variants
                               on the context's own boxes and keep the fastest
                               (the state is saved and restored around the
                               trials; needs workspace for one state copy) */

/* kernel kinds reported by mhd_kernel_times */
#define MHD_K_LAMBDA 0   /* CFL rate max-reduction, per tile */
#define MHD_K_DT 1       /* per-box time step from the tile maxima */
#define MHD_K_SWEEP_X 2  /* x faces: PLM + Riemann solver */
#define MHD_K_SWEEP_Y 3  /* y faces + x/y flux divergence (fused march:
                            the x faces too) */
#define MHD_K_SWEEP_Z 4  /* z faces + divergence + RK stage combine */
#define MHD_K_CT_EDGE 5  /* constrained-transport corner EMFs */
#define MHD_K_CT_FACE 6  /* face-field update + RK stage combine */
#define MHD_NKERNELS 7

typedef struct {
  int32_t n[3];            /* cells per axis, 1..2^20; n == 1 makes the axis
                              inactive; at least one axis active; at most
                              2^29 cells and 2^29 face positions
                              (product of the face counts) per box */
  double lo[3], hi[3];     /* domain corners; dx = (hi - lo) / n */
  int32_t bc_lo[3], bc_hi[3];
  double gamma;            /* ratio of specific heats (> 1) */
  double cfl;              /* CFL number (> 0) */
} mhd_box;

typedef struct {
  int32_t nboxes;          /* >= 1 independent boxes, advanced together */
  const mhd_box *boxes;    /* nboxes descriptors (copied by mhd_create) */
  int32_t precision;       /* MHD_FP64 or MHD_MIXED */
  double p_floor;          /* pressure floor of the primitive recovery; <= 0:
                              1e-10.  Total energy is never modified. */
  void *stream;            /* hipStream_t to run on; NULL: the library
                              creates its own */
  void *workspace;         /* caller-owned device memory for all device
                              buffers (e.g. a torch tensor), kept alive until
                              mhd_destroy; NULL: the library allocates */
  uint64_t workspace_bytes;
  uint32_t flags;          /* MHD_F_* */
  int32_t rk_stages;       /* time integrator: 2 (SSP-RK2; also when 0) or 3
                              (SSP-RK3, Shu & Osher 1988: the paper's default
                              third-order scheme; one more state copy in the
                              workspace) */
  int32_t riemann;         /* MHD_RS_HLLD (0) or MHD_RS_HLL */
  int32_t recon;           /* MHD_REC_PRIM (0) or MHD_REC_CHAR */
  int32_t ct_emf;          /* MHD_EMF_CONTACT (0), MHD_EMF_E0, MHD_EMF_ARITH
                              or MHD_EMF_UCT_HLL */
  int32_t limiter;         /* MHD_LIM_MINMOD (0), MHD_LIM_MC or MHD_LIM_VANLEER */
} mhd_config;

typedef struct mhd_ctx mhd_ctx;

/* Device bytes the configuration needs (for a caller-provided workspace).
 * Validates cfg like mhd_create; touches no device. */
int mhd_workspace_bytes(const mhd_config *cfg, uint64_t *bytes);

/* Validates cfg (before any device call), then creates a context on the
 * current HIP device.  *out is set only on MHD_OK.
 * Defines: the set of independent structured boxes on which the main cycle of
 * the paper's section 2.2.3 runs, with the scheme options that section leaves
 * open (integrator stages, Riemann solver, reconstruction variables, corner
 * EMF, limiter).  Ownership: cfg and cfg->boxes are copied; a caller
 * workspace (cfg->workspace) must stay allocated until mhd_destroy.
 * Errors: MHD_E_INVAL (bad field, nothing allocated), MHD_E_NOMEM (device
 * allocation failed or workspace too small), MHD_E_DEVICE (HIP error). */
int mhd_create(const mhd_config *cfg, mhd_ctx **out);

/* Copies the state of one box in (boundary layout; where = MHD_HOST or
 * MHD_DEVICE) and sets its time.  Returns after the copy has completed.
 * Defines: the conserved state of the conservation laws the code evolves
 * (paper section 2.2 and its 2.2.3): mass, momentum and total energy per
 * cell, and the face-centred magnetic field that constrained transport
 * evolves (one normal component per face, so the discrete divergence of a
 * cell is the sum of its face differences).  Arguments: box in
 * [0, nboxes); cons[5] and bface[3] as described at the top of this file,
 * read only, not retained; t the box time.  Resets the box's event counters
 * and its non-physical flag.  Errors: MHD_E_INVAL if box is out of range, a
 * pointer is NULL, where is unknown or a periodic axis has last face !=
 * first face (nothing changed); MHD_E_DEVICE on a copy failure. */
int mhd_set_state(mhd_ctx *ctx, int32_t box, const double *const cons[5],
                  const double *const bface[3], double t, int32_t where);

/* Enqueues nsteps full Runge-Kutta steps (rk_stages stages each) of every box
 * on the context stream.
 * Defines: the main cycle of the paper's section 2.2.3.  Each stage
 * reconstructs, per direction, the primitive variables (or their
 * characteristic fields, MHD_REC_CHAR) with limited linear slopes,
 * solves a Riemann problem at every interface (HLLD, or HLL for the
 * paper's 2D Riemann runs) and applies the flux-conservative update, then
 * constrained transport updates the face field; the Runge-Kutta stage
 * combine closes the stage (third order by default in the paper; two
 * stages here unless rk_stages = 3).
 * Each box steps with its own CFL time step computed on the device from its
 * state at the start of the step, clamped to t_stop - t when t_stop > 0
 * (steps at t >= t_stop are no-ops).  Returns without waiting; device errors
 * surface at the next mhd_dt / mhd_get_state.  Errors: MHD_E_INVAL if
 * nsteps < 0; MHD_E_STATE if a box has no state yet or its last set_state
 * was rejected; MHD_E_DEVICE on a launch failure. */
int mhd_step(mhd_ctx *ctx, int32_t nsteps, double t_stop);

/* Waits for the stream, then returns the CFL time step the next step of the
 * box would take (no t_stop clamp) and the box time.
 * Defines: the time step from the largest signal speed over the box, the
 * maximum that the Riemann sweep of the paper's section 3.1.1 listing
 * writes into its cmax array: dt = cfl / max over cells and active axes d of
 * (|v_d| + c_f,d) / dx_d, c_f,d the fast magnetosonic speed along d.
 * Arguments: dt_next and t are host pointers, written on MHD_OK and
 * MHD_E_NONPHYS.  Errors: MHD_E_INVAL (box out of range, NULL pointer),
 * MHD_E_STATE (no state), MHD_E_NONPHYS if a non-physical cell was met
 * since the last set_state (values still returned), MHD_E_DEVICE. */
int mhd_dt(mhd_ctx *ctx, int32_t box, double *dt_next, double *t);

/* Waits for the stream, then copies the state of one box out (boundary
 * layout; where = MHD_HOST or MHD_DEVICE).
 * Defines: the conserved state of the paper's section 2.2 (as for
 * mhd_set_state) after the steps enqueued so far; on periodic axes the last
 * face is written equal to the first.  Arguments: cons[5], bface[3] are
 * caller arrays of the boundary layout, written; t (host pointer, may be
 * NULL) receives the box time.  Errors: MHD_E_INVAL, MHD_E_STATE,
 * MHD_E_NONPHYS as for mhd_dt (the state is still copied), MHD_E_DEVICE. */
int mhd_get_state(mhd_ctx *ctx, int32_t box, double *const cons[5],
                  double *const bface[3], double *t, int32_t where);

/* Waits for the stream, then returns the box's event counters since its last
 * set_state: [0] pressure-floor hits (cells x stages), [1] HLL fallbacks
 * (faces x stages), [2] non-physical cells (cells x stages). */
int mhd_counters(mhd_ctx *ctx, int32_t box, int64_t counters[3]);

/* With MHD_F_TIMING: total device milliseconds and launch counts of each
 * kernel kind (MHD_K_*) since creation or the last reset (reset != 0 clears
 * after reading).  Waits for the stream.  MHD_E_STATE without the flag. */
int mhd_kernel_times(mhd_ctx *ctx, double ms[MHD_NKERNELS],
                     int64_t launches[MHD_NKERNELS], int32_t reset);

/* The launch variant in use, five entries:
 * [0] the x direction.  1, 3 or 4: the x sweep, with at least that many
 *     waves per SIMD in its register budget (1 = unconstrained).  0 or 2:
 *     no x sweep; the y march also solves the x faces of its rows (fused
 *     march), with its sliding window in registers and workgroups of 512
 *     lanes (0) or, in the mixed path only, in LDS with 256 lanes (2).  The
 *     fused march is offered for primitive minmod slopes without the upwind
 *     CT when every box has more than one cell along x and y.
 * [1] the march variant, of the y and z marches (with the fused march, of
 *     the z march alone).  1: unconstrained registers with the update
 *     inputs prefetched ahead of the Riemann solve; 2: unconstrained
 *     without prefetch; 3 / 4: at least 3 / 4 waves per SIMD without
 *     prefetch; 5 / 6 / 7: the sliding window kept in LDS, with prefetch /
 *     without / at least 3 waves per SIMD; 8 / 9 / 10: variants 2 / 6 / 7
 *     whose z march keeps the swept state of its last three cells in LDS
 *     for the RK combine instead of reading it again.
 * [2] y march segment length (cells).
 * [3] persistent grid (0/1).
 * [4] z march segment length (cells).
 * The variants differ only in scheduling: FP64 results are identical.  With
 * MHD_REC_CHAR or a limiter other than minmod the sweeps run one variant
 * ([0] and [1] are then ignored). */
int mhd_tuning(mhd_ctx *ctx, int32_t variant[5]);

/* Frees the context and every buffer the library allocated (a caller
 * workspace is left alone).  NULL is a no-op. */
void mhd_destroy(mhd_ctx *ctx);

/* Allocation-free CFL time step of one box whose state the caller holds in
 * device memory: a variant of mhd_dt for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  It needs no context and calls no hipMalloc,
 * hipFree or other allocating routine: its per-tile partial maxima go to a
 * static device array of the library (8 MiB, one copy per GPU, held until
 * the process ends).
 * Arguments: box as for mhd_create (validated the same way); cons[5] and
 * bface[3] are DEVICE pointers to the state in the boundary layout of this
 * file (read only, not retained); p_floor the pressure floor of the
 * primitive recovery (<= 0: 1e-10); dt_out a DEVICE pointer that receives
 * one double, dt = cfl / max over cells and active axes d of
 * (|v_d| + c_f,d) / dx_d, the value mhd_dt returns for the same state (0 if
 * a cell is non-physical: rho <= 0 or a non-finite state); stream a
 * hipStream_t (NULL: the null stream).  The two kernels are enqueued on the
 * stream and the call returns without waiting.
 * Limit: at most 2^28 cells (2^20 tiles of 256 cells); larger boxes are
 * rejected with MHD_E_INVAL before any device work.  All calls on one GPU
 * share its scratch array, which keeps the last call's partials: calls that
 * overlap in time on one GPU (different streams or host threads) race.
 * Errors: MHD_E_INVAL (bad box, NULL pointer, non-finite p_floor, box too
 * large), MHD_E_DEVICE (no device, symbol lookup or launch failure); the
 * message is read with mhd_last_error(NULL). */
int mhd_dt_noalloc(const mhd_box *box, const double *const cons[5],
                   const double *const bface[3], double p_floor, double *dt_out,
                   void *stream);

/* Message of the last failed call on ctx ("" if none); for ctx == NULL, the
 * last failure of mhd_create / mhd_workspace_bytes / mhd_dt_noalloc in this
 * thread. */
const char *mhd_last_error(const mhd_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
