// mhd_lib.hip -- host runtime and C ABI of the MI355X ideal-MHD library.
//
// One context owns the device buffers of an ensemble of boxes (one box is an
// ensemble of one), a tile table per kernel kind and the launch sequence of
// one SSP-RK2 step (arXiv 2606.12753 §2.2.3: reconstruct, Riemann solve,
// conservative update per direction, constrained transport, Runge-Kutta):
//
//   stage 1 and stage 2:
//     k_sweep_x                x faces (LDS row segments); in stage 1 also
//                              the CFL rate max-reduction of the state,
//     (stage 1) k_dt           -> dt, t per box
//     k_sweep_march<y>         y faces (column march), x+y residual
//     k_sweep_march<z>         z faces, residual, RK stage combine
//     k_ct_edge                contact-upwinded corner EMFs
//     k_ct_face                face-field update + RK stage combine
//
// The sequence can be captured once into a HIP graph and replayed per step;
// dt and t never leave the device between steps.
#include "../../include/mhd.h"
#include "mhd_kernels.hpp"
#include "mhd_step.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using mhd::Box;
using mhd::kTPB;

// defined in mhd_fp32.hip (FP32 kernels of the mixed path)
int mhd_enqueue_fp32(const mhd::StepCtx& sc);
int mhd_enqueue_opt64(const mhd::StepCtx& sc);
int mhd_enqueue_opt32(const mhd::StepCtx& sc);

namespace {

thread_local std::string g_create_error;

constexpr size_t kAlign = 256;

inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Gap after every array of a box (bytes, a multiple of kAlign): arrays of
// 2^k bytes would otherwise start a power of two apart, and the arrays a
// kernel reads at the same index would meet the same HBM channels.
// 128 KiB + 256 B measured about 1.3% faster than no gap on blast 256^3 in
// both precisions (a gap that is itself a power of two gains nothing).
// MHD_SKEW overrides it for measurement.
constexpr size_t kArraySkew = 131072 + 256;
inline size_t array_skew() {
  static const size_t v = [] {
    if (const char* e = std::getenv("MHD_SKEW")) {
      const long x = std::atol(e);
      if (x >= 0 && x <= (1L << 20)) return align_up((size_t)x);
    }
    return kArraySkew;
  }();
  return v;
}
inline size_t slot(size_t v) { return align_up(v) + array_skew(); }

struct Geom {
  int n[3], nf[3], per[3], act[3];
  size_t N, F[3], E[3];
};

Geom geom_of(const mhd_box& b) {
  Geom g;
  for (int d = 0; d < 3; d++) {
    g.n[d] = b.n[d];
    g.per[d] = b.bc_lo[d] == MHD_BC_PERIODIC;
    g.nf[d] = g.per[d] ? b.n[d] : b.n[d] + 1;
    g.act[d] = b.n[d] > 1;
  }
  g.N = (size_t)g.n[0] * g.n[1] * g.n[2];
  for (int d = 0; d < 3; d++) {
    size_t f = 1, e = 1;
    for (int a = 0; a < 3; a++) {
      f *= (size_t)(a == d ? g.nf[a] : g.n[a]);
      e *= (size_t)(a == d ? g.n[a] : g.nf[a]);
    }
    g.F[d] = f;
    g.E[d] = e;
  }
  return g;
}

int validate_box(const mhd_box& b, std::string& err) {
  for (int d = 0; d < 3; d++) {
    if (b.n[d] < 1 || b.n[d] > (1 << 20)) {
      err = "box: n[" + std::to_string(d) + "] out of range";
      return MHD_E_INVAL;
    }
    if (!(b.hi[d] > b.lo[d]) || !std::isfinite(b.hi[d] - b.lo[d])) {
      err = "box: hi must exceed lo on every axis";
      return MHD_E_INVAL;
    }
    if (b.bc_lo[d] != b.bc_hi[d] ||
        (b.bc_lo[d] != MHD_BC_PERIODIC && b.bc_lo[d] != MHD_BC_OUTFLOW)) {
      err = "box: boundary conditions must be periodic or outflow and alike on both sides";
      return MHD_E_INVAL;
    }
  }
  if (!(b.gamma > 1.0) || !std::isfinite(b.gamma)) {
    err = "box: gamma must be > 1";
    return MHD_E_INVAL;
  }
  if (!(b.cfl > 0.0) || !std::isfinite(b.cfl)) {
    err = "box: cfl must be > 0";
    return MHD_E_INVAL;
  }
  if (b.n[0] == 1 && b.n[1] == 1 && b.n[2] == 1) {
    // no axis carries a wave: the CFL rate is zero and dt undefined
    err = "box: at least one axis needs more than one cell";
    return MHD_E_INVAL;
  }
  const Geom g = geom_of(b);
  // the kernels address every cell, face, edge and corner array with a
  // 32-bit byte offset: at most 2^29 elements of 8 bytes per array
  const size_t P = (size_t)g.nf[0] * g.nf[1] * g.nf[2];
  if (g.N > ((size_t)1 << 29) || P > ((size_t)1 << 29)) {
    err = "box: more than 2^29 cells or face positions";
    return MHD_E_INVAL;
  }
  return MHD_OK;
}

int validate_config(const mhd_config* cfg, std::string& err) {
  if (!cfg) {
    err = "config is NULL";
    return MHD_E_INVAL;
  }
  if (cfg->nboxes < 1 || cfg->nboxes > (1 << 20) || !cfg->boxes) {
    err = "config: need nboxes >= 1 and a boxes array";
    return MHD_E_INVAL;
  }
  if (cfg->precision != MHD_FP64 && cfg->precision != MHD_MIXED) {
    err = "config: precision must be MHD_FP64 or MHD_MIXED";
    return MHD_E_INVAL;
  }
  if (cfg->flags & ~(uint32_t)(MHD_F_GRAPH | MHD_F_PERSISTENT | MHD_F_TIMING | MHD_F_AUTOTUNE)) {
    err = "config: unknown flag bits";
    return MHD_E_INVAL;
  }
  if (!std::isfinite(cfg->p_floor)) {
    err = "config: p_floor must be finite";
    return MHD_E_INVAL;
  }
  if (cfg->rk_stages != 0 && cfg->rk_stages != 2 && cfg->rk_stages != 3) {
    err = "config: rk_stages must be 2 or 3 (0: 2)";
    return MHD_E_INVAL;
  }
  if (cfg->riemann != MHD_RS_HLLD && cfg->riemann != MHD_RS_HLL) {
    err = "config: riemann must be MHD_RS_HLLD or MHD_RS_HLL";
    return MHD_E_INVAL;
  }
  if (cfg->recon != MHD_REC_PRIM && cfg->recon != MHD_REC_CHAR) {
    err = "config: recon must be MHD_REC_PRIM or MHD_REC_CHAR";
    return MHD_E_INVAL;
  }
  if (cfg->limiter != MHD_LIM_MINMOD && cfg->limiter != MHD_LIM_MC &&
      cfg->limiter != MHD_LIM_VANLEER) {
    err = "config: limiter must be MHD_LIM_MINMOD, MHD_LIM_MC or MHD_LIM_VANLEER";
    return MHD_E_INVAL;
  }
  if (cfg->ct_emf != MHD_EMF_CONTACT && cfg->ct_emf != MHD_EMF_E0 &&
      cfg->ct_emf != MHD_EMF_ARITH && cfg->ct_emf != MHD_EMF_UCT_HLL) {
    err = "config: ct_emf must be MHD_EMF_CONTACT, MHD_EMF_E0, MHD_EMF_ARITH or MHD_EMF_UCT_HLL";
    return MHD_E_INVAL;
  }
  for (int b = 0; b < cfg->nboxes; b++) {
    int rc = validate_box(cfg->boxes[b], err);
    if (rc) {
      err = "box " + std::to_string(b) + ": " + err;
      return rc;
    }
  }
  return MHD_OK;
}

// planes per lane of the corner-EMF kernel (turbulence 512^3, per launch
// FP64 / mixed: 1 plane 3.88 / 1.68 ms, 2 3.59 / 1.59, 4 3.48 / 1.61,
// 8 3.56 / 1.60, 16 3.56 / 1.63)
constexpr int kDefaultCzk = 4;

// tiling of one box (the y/z march segment lengths are tunable)
struct Tiling {
  int xft, ctx, czk, ysl, yseg, zsl, zseg;
  int ntile[6];
};

// ycols: columns per y-march tile (kTPB, or kYXW for the y march with the
// x faces in registers, x variant 0)
Tiling tiling_of(const Geom& g, int ysl, int zsl, bool fp64, int ycols = kTPB) {
  Tiling t;
  // x sweep: kTPB consecutive faces of the rows per tile when the pieces of
  // rows they touch fit the LDS, else whole rows
  const int nf = g.nf[0];
  const int pieces = (kTPB - 1) / nf + 2;
  if (kTPB + 3 * pieces <= mhd::kLdsCells) {
    t.xft = kTPB;
  } else {
    const int R = std::max(1, std::min(kTPB / nf, mhd::kLdsCells / (nf + 3)));
    t.xft = R * nf;
  }
  t.ysl = g.act[1] ? std::max(1, std::min(ysl, g.n[1])) : 1;
  t.yseg = (g.n[1] + t.ysl - 1) / t.ysl;
  t.zsl = g.act[2] ? std::max(1, std::min(zsl, g.n[2])) : 1;
  t.zseg = (g.n[2] + t.zsl - 1) / t.zsl;
  const long long nrows = (long long)g.n[1] * g.n[2];
  t.ntile[mhd::kXS] = (int)((nrows * nf + t.xft - 1) / t.xft);
  t.ntile[mhd::kYS] = (int)(((long long)g.n[0] * g.n[2] + ycols - 1) / ycols * t.yseg);
  t.ntile[mhd::kZS] = (int)(((long long)g.n[0] * g.n[1] + kTPB - 1) / kTPB * t.zseg);
  // corner-EMF kernel: tiles of ctx x (kTPB / ctx) positions per xy plane,
  // rows of 32 in FP64 and of 128 in the mixed path (measured best on rows
  // of 256, 352 and 768 positions), narrower or wider ones if those leave
  // more than an eighth of the lanes idle, flat order if all do.  The face
  // update runs in flat order (measured fastest).
  t.ctx = 0;
  {
    static const int pref64[] = {32, 64, 16, 128};
    static const int prefmx[] = {128, 64, 256, 32};
    const int* pref = fp64 ? pref64 : prefmx;
    for (int c = 0; c < 4; c++) {
      const int w = pref[c], h = kTPB / w;
      const double used = (double)g.nf[0] * g.nf[1];
      const double all = (double)((g.nf[0] + w - 1) / w * w) * ((g.nf[1] + h - 1) / h * h);
      if (8.0 * (all - used) <= all) {
        t.ctx = w;
        break;
      }
    }
    // measurement override: MHD_CTX = 0 (flat), 16, 32, 64, 128 or 256
    if (const char* v = std::getenv("MHD_CTX")) {
      const int w = std::atoi(v);
      if (w == 0 || w == 16 || w == 32 || w == 64 || w == 128 || w == 256) t.ctx = w;
    }
  }
  // planes each lane of the corner-EMF kernel walks (its plane-below values
  // then come from registers; see k_ct_edge); one in flat order
  t.czk = kDefaultCzk;
  if (const char* v = std::getenv("MHD_CZK")) t.czk = std::max(1, std::atoi(v));
  if (t.ctx == 0) t.czk = 1;
  const long long P = (long long)g.nf[0] * g.nf[1] * g.nf[2];
  if (t.ctx == 0) {
    t.ntile[mhd::kCTE] = (int)((P + kTPB - 1) / kTPB);
  } else {
    const long long cy = kTPB / t.ctx;
    const long long nbx = (g.nf[0] + t.ctx - 1) / t.ctx, nby = (g.nf[1] + cy - 1) / cy;
    t.ntile[mhd::kCTE] = (int)(nbx * nby * ((g.nf[2] + t.czk - 1) / t.czk));
  }
  t.ntile[mhd::kCTF] = (int)((P + kTPB - 1) / kTPB);

  t.ntile[mhd::kLAM] = (int)((g.N + kTPB - 1) / kTPB);
  return t;
}

constexpr int kDefaultSeg = 32;

// byte layout of the workspace
struct Plan {
  size_t total;
  size_t boxes_off, base_off, flag_off, backup_off, backup_bytes;
  std::vector<size_t> box_off;  // start of each box's region
  std::vector<size_t> box_bytes;
};

// bytes of one box's restorable state: U, face B, scalars, counters
size_t backup_bytes_of(const Geom& g) {
  return align_up(mhd::kNQ * g.N * 8) + align_up((g.F[0] + g.F[1] + g.F[2]) * 8) + 4 * 8 + 3 * 8;
}

// state copies: the start of the step and one stage state (SSP-RK2), or two
// stage states (SSP-RK3)
int state_copies(const mhd_config* cfg) { return cfg->rk_stages == 3 ? 3 : 2; }

// per-tile CFL partials of a box: one per tile of the kernel that reduces
// the rate (the x sweep, the y march with the x faces, the mhd_dt query),
// sized for the y march's shortest segment (one cell) so that no segment
// length a launch variant or the autotuner sets can overrun it
size_t lam_slots(const Geom& g, const Tiling& t) {
  const size_t ymax = ((size_t)g.n[0] * g.n[2] + kTPB - 1) / kTPB * (size_t)g.n[1];
  return std::max({(size_t)t.ntile[mhd::kLAM], (size_t)t.ntile[mhd::kXS], ymax});
}

size_t box_bytes(const Geom& g, const Tiling& t, size_t rs, int copies, bool uct) {
  size_t s = 0;
  s += copies * mhd::kNQ * slot(g.N * 8);
  for (int d = 0; d < 3; d++) s += copies * slot(g.F[d] * 8);
  s += 3 * slot(g.N * rs);                      // Ec
  s += mhd::kNQ * slot(g.F[0] * rs);            // FX
  for (int d = 0; d < 3; d++) s += 3 * slot(g.F[d] * rs);  // EF x2 + MF
  s += mhd::kNQ * slot(g.N * rs);               // R
  for (int c = 0; c < 3; c++) s += slot(g.E[c] * rs);  // ED
  if (uct) {
    for (int d = 0; d < 3; d++) s += 2 * slot(g.F[d] * rs);  // SP
    s += 3 * slot(g.N * rs);                                 // V
  }
  s += slot(lam_slots(g, t) * 8);               // lam
  s += slot(4 * 8);                             // scal
  s += slot(3 * 8);                             // cnt
  return s;
}

Plan make_plan(const mhd_config* cfg, int ysl, int zsl) {
  Plan p;
  const size_t rs = cfg->precision == MHD_FP64 ? 8 : 4;
  size_t off = 0;
  p.boxes_off = off;
  off += align_up(sizeof(Box) * (size_t)cfg->nboxes);
  p.base_off = off;
  off += align_up(sizeof(int) * 6 * ((size_t)cfg->nboxes + 1));
  p.flag_off = off;
  off += align_up(sizeof(int));
  for (int b = 0; b < cfg->nboxes; b++) {
    Geom g = geom_of(cfg->boxes[b]);
    Tiling t = tiling_of(g, ysl, zsl, cfg->precision == MHD_FP64);
    size_t bb = box_bytes(g, t, rs, state_copies(cfg), cfg->ct_emf == MHD_EMF_UCT_HLL);
    p.box_off.push_back(off);
    p.box_bytes.push_back(bb);
    off += bb;
  }
  p.backup_off = off;
  p.backup_bytes = 0;
  if (cfg->flags & MHD_F_AUTOTUNE) {
    for (int b = 0; b < cfg->nboxes; b++) p.backup_bytes += backup_bytes_of(geom_of(cfg->boxes[b]));
    off += align_up(p.backup_bytes);
  }
  p.total = off;
  return p;
}

}  // namespace

struct mhd_ctx {
  std::vector<mhd_box> boxes;
  int precision = MHD_FP64;
  int rk = 2;  // Runge-Kutta stages
  int rs = 0;  // Riemann solver (MHD_RS_*)
  int fz = 0;  // every box: one cell along z, more along y (no z march)
  int sl = 0;  // slope kind: recon + 2 * limiter (MHD_REC_*, MHD_LIM_*)
  int uct = 0;  // corner EMFs by the upwind CT (MHD_EMF_UCT_HLL)
  int emf = 0;  // corner average (config ct_emf)
  int fusable = 0;  // the y march may compute the x faces (x variant 0):
                    // primitive minmod slopes, no upwind CT, no fused 2D y
                    // march, x and y active in every box
  double pfloor = 1e-10;
  uint32_t flags = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  bool own_ws = false;
  std::vector<Box> hbox;
  std::vector<Geom> geom;
  std::vector<int> base;  // 6 * (nboxes + 1)
  int total[6] = {0, 0, 0, 0, 0, 0};
  int grid[6] = {0, 0, 0, 0, 0, 0};
  // launch variant: register budget of the x sweep and of the marches (min
  // waves per SIMD), march segment length, persistent grid
  int var_x = 1, var_m = 1, var_seg = 64, var_segz = 64, var_pers = 0;
  int var_xcd = 0;  // XCD-grouped tile order per kernel kind (bit mask)
  int cu_count = 0;
  bool tuned = false;
  char* backup = nullptr;  // state copy for the autotuner's trial steps
  size_t backup_bytes = 0;
  Box* dbox = nullptr;
  int* dbase = nullptr;
  int* dflag = nullptr;
  std::vector<char> state_set;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  // MHD_F_TIMING: one event pair per launch of a step, reused every step
  std::vector<hipEvent_t> ev;
  std::vector<int> ev_kind;
  double kms[MHD_NKERNELS] = {0, 0, 0, 0, 0, 0, 0};
  int64_t kcount[MHD_NKERNELS] = {0, 0, 0, 0, 0, 0, 0};
  std::string err;
};

namespace {

int fail(mhd_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPCHK(ctx, call)                                                      \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess)                                                      \
      return fail((ctx), MHD_E_DEVICE,                                         \
                  std::string(#call) + ": " + hipGetErrorString(e_));          \
  } while (0)

// one step's launches (csrc/mhd_step.hpp); the FP32 kernels of the mixed
// path are instantiated in mhd_fp32.hip, built with FMA contraction
int enqueue_step_t(mhd_ctx* c) {
  mhd::StepCtx sc;
  sc.L.boxes = c->dbox;
  sc.L.base = c->dbase;
  sc.L.nboxes = (int)c->boxes.size();
  sc.L.lam = 0;
  sc.L.stage = 0;
  sc.L.ntiles = 0;
  sc.total = c->total;
  sc.grid = c->grid;
  sc.var_x = c->var_x;
  sc.var_m = c->var_m;
  sc.rk = c->rk;
  sc.rs = c->rs;
  sc.fz = c->fz;
  sc.sl = c->sl;
  sc.xcd = c->var_xcd;
  sc.uct = c->uct;
  sc.emf = c->emf;
  sc.stream = c->stream;
  const bool timing = (c->flags & MHD_F_TIMING) != 0;
  sc.ev = timing ? c->ev.data() : nullptr;
  sc.ev_kind = timing ? c->ev_kind.data() : nullptr;
  const bool fp64 = c->precision == MHD_FP64;
  const int slots = sc.sl == 0 ? (fp64 ? mhd::enqueue_step_sl<double, 0>(sc) : mhd_enqueue_fp32(sc))
                               : (fp64 ? mhd_enqueue_opt64(sc) : mhd_enqueue_opt32(sc));
  HIPCHK(c, hipGetLastError());
  if (timing) {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int k = 0; k < slots; k++) {
      float ms = 0.f;
      HIPCHK(c, hipEventElapsedTime(&ms, c->ev[2 * k], c->ev[2 * k + 1]));
      c->kms[c->ev_kind[k]] += ms;
      c->kcount[c->ev_kind[k]] += 1;
    }
  }
  return MHD_OK;
}

constexpr int kLaunchesPerStep = mhd::kLaunchesPerStep;

int enqueue_step(mhd_ctx* c) { return enqueue_step_t(c); }

__global__ void k_set_scalar(const Box* boxes, int nboxes, int slot, double v) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nboxes) boxes[b].scal[slot] = v;
}

__global__ void k_reset_box(const Box* boxes, int box, double t) {
  const Box& b = boxes[box];
  if (threadIdx.x == 0) {
    b.scal[0] = 0.0;
    b.scal[1] = t;
    b.scal[2] = 0.0;
    b.scal[3] = 0.0;
    b.cnt[0] = 0;
    b.cnt[1] = 0;
    b.cnt[2] = 0;
  }
}

void set_persistent(mhd_ctx* c, int on) {
  c->var_pers = on;
  // eight resident workgroups per compute unit
  for (int k = 0; k < 6; k++) c->grid[k] = on ? c->cu_count * 8 : 0;
}

// re-tile the y/z marches with segment length seg (device tables updated
// on the context stream)
// segment lengths of the y and z marches
// columns per y-march tile for the context's x variant
int ycols_of(const mhd_ctx* c) { return c->var_x == 0 ? mhd::kYXW : kTPB; }

int apply_tiling(mhd_ctx* c, int segy, int segz) {
  const int nb = (int)c->boxes.size();
  c->var_seg = segy;
  c->var_segz = segz;
  for (int k = 0; k < 6; k++) c->total[k] = 0;
  for (int bi = 0; bi < nb; bi++) {
    Tiling t = tiling_of(c->geom[bi], segy, segz, c->precision == MHD_FP64, ycols_of(c));
    Box& b = c->hbox[bi];
    b.ysl = t.ysl;
    b.yseg = t.yseg;
    b.zsl = t.zsl;
    b.zseg = t.zseg;
    for (int k = 0; k < 6; k++) {
      b.ntile[k] = t.ntile[k];
      c->base[k * (nb + 1) + bi] = c->total[k];
      c->total[k] += t.ntile[k];
    }
  }
  for (int k = 0; k < 6; k++) c->base[k * (nb + 1) + nb] = c->total[k];
  HIPCHK(c, hipMemcpyAsync(c->dbox, c->hbox.data(), sizeof(Box) * nb, hipMemcpyHostToDevice,
                           c->stream));
  HIPCHK(c, hipMemcpyAsync(c->dbase, c->base.data(), sizeof(int) * c->base.size(),
                           hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return MHD_OK;
}

// copy every box's state (U, B, t, counters) to (save) or from the backup
int backup_state(mhd_ctx* c, bool save) {
  char* p = c->backup;
  for (size_t bi = 0; bi < c->boxes.size(); bi++) {
    const Geom& g = c->geom[bi];
    const Box& b = c->hbox[bi];
    auto cp = [&](void* dev, size_t bytes) -> int {
      if (save)
        HIPCHK(c, hipMemcpyAsync(p, dev, bytes, hipMemcpyDeviceToDevice, c->stream));
      else
        HIPCHK(c, hipMemcpyAsync(dev, p, bytes, hipMemcpyDeviceToDevice, c->stream));
      p += bytes;
      return MHD_OK;
    };
    char* start = p;
    for (int q = 0; q < mhd::kNQ; q++)
      if (cp(b.U[0][q], g.N * 8)) return MHD_E_DEVICE;
    p = start + align_up(mhd::kNQ * g.N * 8);
    start = p;
    for (int d = 0; d < 3; d++)
      if (cp(b.B[0][d], g.F[d] * 8)) return MHD_E_DEVICE;
    p = start + align_up((g.F[0] + g.F[1] + g.F[2]) * 8);
    if (cp(b.scal, 4 * 8)) return MHD_E_DEVICE;
    if (cp(b.cnt, 3 * 8)) return MHD_E_DEVICE;
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return MHD_OK;
}

int enqueue_step(mhd_ctx* c);

// time `steps` steps of the current variant (state restored afterwards)
int trial(mhd_ctx* c, int steps, float* ms) {
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  int rc = enqueue_step(c);  // warm-up
  if (!rc) {
    (void)hipEventRecord(e0, c->stream);
    for (int s = 0; s < steps && !rc; s++) rc = enqueue_step(c);
    (void)hipEventRecord(e1, c->stream);
  }
  hipError_t e = hipEventSynchronize(e1);
  if (!rc && e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  if (e != hipSuccess) return fail(c, MHD_E_DEVICE, std::string("autotune: ") + hipGetErrorString(e));
  return backup_state(c, false);
}

// MHD_TUNE_LOG set: the autotuner prints each trial's time to stderr
static bool tune_log() { return std::getenv("MHD_TUNE_LOG") != nullptr; }

// Coordinate search over the launch variants on the context's own boxes and
// state: register budget of the x sweep and of the marches, march segment
// length, persistent grid.  The arithmetic of every variant is the same, so
// the FP64 results do not depend on the choice.  A candidate replaces the
// current variant only when it is more than 1% faster, so that timing noise
// between near-equal variants does not change the choice from run to run.
int autotune(mhd_ctx* c) {
  if (!c->backup) return fail(c, MHD_E_STATE, "autotune needs a context created with MHD_F_AUTOTUNE");
  int rc = backup_state(c, true);
  if (rc) return rc;
  const int steps = 3;
  float best = 0.f;
  rc = trial(c, steps, &best);
  if (rc) return rc;
  auto try_var = [&](int* field, int value, auto apply) -> int {
    const int old = *field;
    int r = apply(value);
    if (r) return r;
    float ms = 0.f;
    r = trial(c, steps, &ms);
    if (r) return r;
    if (tune_log())
      std::fprintf(stderr, "[mhd autotune] x %d m %d seg %d/%d pers %d: %.3f ms (best %.3f)\n",
                   c->var_x, c->var_m, c->var_seg, c->var_segz, c->var_pers, ms, best);
    if (ms < 0.99f * best) {
      best = ms;
    } else {
      r = apply(old);
      if (r) return r;
    }
    return MHD_OK;
  };
  auto set_x = [&](int v) {
    // the y march's tiles are wider with the x faces in registers
    const bool retile = (v == 0) != (c->var_x == 0);
    c->var_x = v;
    return retile ? apply_tiling(c, c->var_seg, c->var_segz) : MHD_OK;
  };
  auto set_m = [&](int v) { c->var_m = v; return MHD_OK; };
  auto set_seg = [&](int v) { return apply_tiling(c, v, c->var_segz); };
  auto set_segz = [&](int v) { return apply_tiling(c, c->var_seg, v); };
  auto set_pers = [&](int v) { set_persistent(c, v); return MHD_OK; };
  // the x and march variants apply to the default slope kind only (the
  // others run one variant)
  if (c->sl == 0) {
    for (int v : {2, 3, 5, 6, 7, 8, 9, 10})
      if ((rc = try_var(&c->var_m, v, set_m))) return rc;
    for (int v : {3, 4})
      if ((rc = try_var(&c->var_x, v, set_x))) return rc;
    if (c->fusable) {
      // the x faces in the y march, its window in registers and (mixed
      // path) in LDS; the z march keeps the variant chosen above
      for (int v : {0, 2})
        if ((v == 0 || c->precision != MHD_FP64) && (rc = try_var(&c->var_x, v, set_x))) return rc;
      // with the y march fused, the march variant chooses the z march alone:
      // its choice above was made beside the unfused y march, so try again
      if (c->var_x == 0 || c->var_x == 2)
        for (int v : {1, 2, 3, 5, 6, 7, 8, 9, 10})
          if (v != c->var_m && (rc = try_var(&c->var_m, v, set_m))) return rc;
    }
  }
  for (int v : {16, 32, 64, 128})
    if (v != c->var_seg && (rc = try_var(&c->var_seg, v, set_seg))) return rc;
  for (int v : {16, 32, 64, 128})
    if (v != c->var_segz && (rc = try_var(&c->var_segz, v, set_segz))) return rc;
  if ((rc = try_var(&c->var_pers, 1 - c->var_pers, set_pers))) return rc;
  c->tuned = true;
  return MHD_OK;
}

int build_ctx(mhd_ctx* c, const mhd_config* cfg) {
  const int nb = cfg->nboxes;
  const Plan plan = make_plan(cfg, kDefaultSeg, kDefaultSeg);
  if (cfg->workspace) {
    if (cfg->workspace_bytes < plan.total)
      return fail(c, MHD_E_NOMEM, "workspace smaller than mhd_workspace_bytes()");
    if ((uintptr_t)cfg->workspace % kAlign)
      return fail(c, MHD_E_INVAL, "workspace must be 256-byte aligned");
    c->ws = static_cast<char*>(cfg->workspace);
    c->ws_bytes = cfg->workspace_bytes;
    c->own_ws = false;
  } else {
    void* p = nullptr;
    if (hipMalloc(&p, plan.total) != hipSuccess)
      return fail(c, MHD_E_NOMEM, "hipMalloc of " + std::to_string(plan.total) + " bytes failed");
    c->ws = static_cast<char*>(p);
    c->ws_bytes = plan.total;
    c->own_ws = true;
  }
  const size_t rs = cfg->precision == MHD_FP64 ? 8 : 4;
  c->dbox = reinterpret_cast<Box*>(c->ws + plan.boxes_off);
  c->dbase = reinterpret_cast<int*>(c->ws + plan.base_off);
  c->dflag = reinterpret_cast<int*>(c->ws + plan.flag_off);
  c->hbox.resize(nb);
  c->geom.resize(nb);
  c->base.assign(6 * (nb + 1), 0);
  for (int k = 0; k < 6; k++) c->total[k] = 0;
  for (int bi = 0; bi < nb; bi++) {
    const mhd_box& mb = cfg->boxes[bi];
    Geom g = geom_of(mb);
    Tiling t = tiling_of(g, c->var_seg, c->var_segz, c->precision == MHD_FP64, ycols_of(c));
    c->geom[bi] = g;
    Box& b = c->hbox[bi];
    std::memset(&b, 0, sizeof(Box));
    for (int d = 0; d < 3; d++) {
      b.n[d] = g.n[d];
      b.nf[d] = g.nf[d];
      b.per[d] = g.per[d];
      b.act[d] = g.act[d];
      b.dx[d] = (mb.hi[d] - mb.lo[d]) / (double)mb.n[d];
      b.idx[d] = 1.0 / b.dx[d];
    }
    b.gamma = mb.gamma;
    b.igm1 = 1.0 / (mb.gamma - 1.0);
    b.cfl = mb.cfl;
    b.pfloor = cfg->p_floor > 0.0 ? cfg->p_floor : 1e-10;
    char* p = c->ws + plan.box_off[bi];
    auto take = [&](size_t bytes) {
      char* q = p;
      p += slot(bytes);
      return q;
    };
    const int copies = state_copies(cfg);
    for (int s = 0; s < 3; s++)
      for (int q = 0; q < mhd::kNQ; q++)
        b.U[s][q] = s < copies ? reinterpret_cast<double*>(take(g.N * 8)) : nullptr;
    for (int s = 0; s < 3; s++)
      for (int d = 0; d < 3; d++)
        b.B[s][d] = s < copies ? reinterpret_cast<double*>(take(g.F[d] * 8)) : nullptr;
    for (int d = 0; d < 3; d++) b.Ec[d] = take(g.N * rs);
    for (int q = 0; q < mhd::kNQ; q++) b.FX[q] = take(g.F[0] * rs);
    for (int d = 0; d < 3; d++) {
      b.EF[d][0] = take(g.F[d] * rs);
      b.EF[d][1] = take(g.F[d] * rs);
      b.MF[d] = take(g.F[d] * rs);
    }
    for (int q = 0; q < mhd::kNQ; q++) b.R[q] = take(g.N * rs);
    for (int cc = 0; cc < 3; cc++) b.ED[cc] = take(g.E[cc] * rs);
    if (cfg->ct_emf == MHD_EMF_UCT_HLL)
      for (int d = 0; d < 3; d++) {
        b.SP[d][0] = take(g.F[d] * rs);
        b.SP[d][1] = take(g.F[d] * rs);
        b.V[d] = take(g.N * rs);
      }
    b.lam = reinterpret_cast<double*>(take(lam_slots(g, t) * 8));
    b.scal = reinterpret_cast<double*>(take(4 * 8));
    b.cnt = reinterpret_cast<unsigned long long*>(take(3 * 8));
    b.xft = t.xft;
    b.ctx = t.ctx;
    b.czk = t.czk;
    b.emf = cfg->ct_emf;
    b.lim = cfg->limiter;
    b.ysl = t.ysl;
    b.yseg = t.yseg;
    b.zsl = t.zsl;
    b.zseg = t.zseg;
    for (int k = 0; k < 6; k++) {
      b.ntile[k] = t.ntile[k];
      c->base[k * (nb + 1) + bi] = c->total[k];
      c->total[k] += t.ntile[k];
    }
    if ((size_t)(p - c->ws) > plan.box_off[bi] + plan.box_bytes[bi])
      return fail(c, MHD_E_NOMEM, "internal: workspace plan overflow");
  }
  for (int k = 0; k < 6; k++) {
    c->base[k * (nb + 1) + nb] = c->total[k];
    if (c->total[k] < 0) return fail(c, MHD_E_INVAL, "tile count overflow");
  }
  if (c->flags & MHD_F_TIMING) {
    c->ev.assign(2 * kLaunchesPerStep, nullptr);
    c->ev_kind.assign(kLaunchesPerStep, 0);
    for (auto& e : c->ev) HIPCHK(c, hipEventCreate(&e));
  }
  {
    hipDeviceProp_t prop;
    HIPCHK(c, hipGetDeviceProperties(&prop, c->device));
    c->cu_count = prop.multiProcessorCount;
  }
  if (c->flags & MHD_F_PERSISTENT) c->var_pers = 1;
  set_persistent(c, c->var_pers);
  c->backup = plan.backup_bytes ? c->ws + plan.backup_off : nullptr;
  c->backup_bytes = plan.backup_bytes;
  HIPCHK(c, hipMemcpyAsync(c->dbox, c->hbox.data(), sizeof(Box) * nb, hipMemcpyHostToDevice,
                           c->stream));
  HIPCHK(c, hipMemcpyAsync(c->dbase, c->base.data(), sizeof(int) * c->base.size(),
                           hipMemcpyHostToDevice, c->stream));
  for (int bi = 0; bi < nb; bi++)
    hipLaunchKernelGGL(k_reset_box, dim3(1), dim3(64), 0, c->stream, c->dbox, bi, 0.0);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->state_set.assign(nb, 0);
  return MHD_OK;
}

int check_box_index(mhd_ctx* c, int32_t box) {
  if (!c) return MHD_E_INVAL;
  if (box < 0 || box >= (int32_t)c->boxes.size())
    return fail(c, MHD_E_INVAL, "box index out of range");
  return MHD_OK;
}

// copy between the boundary layout (n+1 faces) and the internal layout (n
// faces on periodic axes)
int copy_faces(mhd_ctx* c, const Geom& g, int d, double* dst, const double* src, bool to_internal,
               hipMemcpyKind kind) {
  const size_t nx = g.n[0], ny = g.n[1], nz = g.n[2];
  if (!g.per[d]) {
    HIPCHK(c, hipMemcpyAsync(dst, src, g.F[d] * 8, kind, c->stream));
    return MHD_OK;
  }
  size_t width, rows, ext_pitch, int_pitch;
  if (d == 0) {
    width = nx * 8;
    rows = ny * nz;
    ext_pitch = (nx + 1) * 8;
    int_pitch = nx * 8;
  } else if (d == 1) {
    width = ny * nx * 8;
    rows = nz;
    ext_pitch = (ny + 1) * nx * 8;
    int_pitch = ny * nx * 8;
  } else {
    HIPCHK(c, hipMemcpyAsync(dst, src, nz * ny * nx * 8, kind, c->stream));
    if (!to_internal) {
      // last plane = first plane
      HIPCHK(c, hipMemcpyAsync(dst + nz * ny * nx, src, ny * nx * 8, kind, c->stream));
    }
    return MHD_OK;
  }
  if (kind != hipMemcpyDeviceToDevice) {
    // host side: rows are packed or unpacked on the host around one plain
    // copy, so that no pitched copy touches pageable host memory (a pitched
    // copy may be staged through whole pitch spans and write the face-n
    // column of the rows it skips)
    const size_t wd = width / 8, ip = int_pitch / 8, ep = ext_pitch / 8, fw = d == 0 ? 1 : nx;
    std::vector<double> tmp(rows * ip);
    if (to_internal) {
      for (size_t r = 0; r < rows; r++) std::memcpy(&tmp[r * ip], src + r * ep, width);
      HIPCHK(c, hipMemcpyAsync(dst, tmp.data(), rows * int_pitch, kind, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
    } else {
      HIPCHK(c, hipMemcpyAsync(tmp.data(), src, rows * int_pitch, kind, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      for (size_t r = 0; r < rows; r++) {
        std::memcpy(dst + r * ep, &tmp[r * ip], width);
        std::memcpy(dst + r * ep + wd, &tmp[r * ip], fw * 8);  // face n = face 0
      }
    }
    return MHD_OK;
  }
  if (to_internal) {
    HIPCHK(c, hipMemcpy2DAsync(dst, int_pitch, src, ext_pitch, width, rows, kind, c->stream));
  } else {
    HIPCHK(c, hipMemcpy2DAsync(dst, ext_pitch, src, int_pitch, width, rows, kind, c->stream));
    // duplicate face 0 into face n
    const size_t first_w = d == 0 ? 8 : nx * 8;
    HIPCHK(c, hipMemcpy2DAsync(reinterpret_cast<char*>(dst) + width, ext_pitch, src, int_pitch,
                               first_w, rows, kind, c->stream));
  }
  return MHD_OK;
}

bool host_periodic_ok(const Geom& g, int d, const double* a) {
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const int ex = nx + (d == 0), ey = ny + (d == 1);
  const int e0 = d == 0 ? 1 : nx, e1 = d == 1 ? 1 : ny, e2 = d == 2 ? 1 : nz;
  for (int k = 0; k < e2; k++)
    for (int j = 0; j < e1; j++)
      for (int i = 0; i < e0; i++) {
        int i2 = i, j2 = j, k2 = k;
        if (d == 0) i2 = nx; else if (d == 1) j2 = ny; else k2 = nz;
        if (a[((size_t)k * ey + j) * ex + i] != a[((size_t)k2 * ey + j2) * ex + i2]) return false;
      }
  return true;
}

int read_flags(mhd_ctx* c, int32_t box, unsigned long long cnt[3]) {
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(cnt, c->hbox[box].cnt, 3 * sizeof(unsigned long long),
                      hipMemcpyDeviceToHost));
  return MHD_OK;
}

}  // namespace

extern "C" {

int mhd_workspace_bytes(const mhd_config* cfg, uint64_t* bytes) {
  std::string err;
  int rc = validate_config(cfg, err);
  if (rc) {
    g_create_error = err;
    return rc;
  }
  if (!bytes) {
    g_create_error = "bytes is NULL";
    return MHD_E_INVAL;
  }
  *bytes = make_plan(cfg, kDefaultSeg, kDefaultSeg).total;
  return MHD_OK;
}

int mhd_create(const mhd_config* cfg, mhd_ctx** out) {
  std::string err;
  if (!out) {
    g_create_error = "out is NULL";
    return MHD_E_INVAL;
  }
  int rc = validate_config(cfg, err);
  if (rc) {
    g_create_error = err;
    return rc;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    g_create_error = "no HIP device";
    return MHD_E_DEVICE;
  }
  mhd_ctx* c = new (std::nothrow) mhd_ctx();
  if (!c) {
    g_create_error = "out of host memory";
    return MHD_E_NOMEM;
  }
  c->boxes.assign(cfg->boxes, cfg->boxes + cfg->nboxes);
  c->precision = cfg->precision;
  c->pfloor = cfg->p_floor > 0.0 ? cfg->p_floor : 1e-10;
  c->flags = cfg->flags;
  c->rk = cfg->rk_stages == 3 ? 3 : 2;
  c->rs = cfg->riemann;
  c->sl = cfg->recon + 2 * cfg->limiter;
  c->uct = cfg->ct_emf == MHD_EMF_UCT_HLL;
  c->emf = cfg->ct_emf;
  c->fz = 1;
  for (int b = 0; b < cfg->nboxes; b++)
    if (cfg->boxes[b].n[2] != 1 || cfg->boxes[b].n[1] == 1) c->fz = 0;
  c->fusable = c->sl == 0 && !c->uct && !c->fz;
  for (int b = 0; b < cfg->nboxes; b++)
    if (cfg->boxes[b].n[0] == 1 || cfg->boxes[b].n[1] == 1) c->fusable = 0;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    g_create_error = "hipGetDevice failed";
    return MHD_E_DEVICE;
  }
  if (cfg->stream) {
    c->stream = static_cast<hipStream_t>(cfg->stream);
    c->own_stream = false;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      g_create_error = "hipStreamCreate failed";
      return MHD_E_DEVICE;
    }
    c->own_stream = true;
  }
  // default march segments (measured on 256^3): 64 cells along y; along z
  // 64 in FP64, 128 in the mixed path
  c->var_segz = cfg->precision == MHD_FP64 ? 64 : 128;
  if (const char* v = std::getenv("MHD_VARIANT")) {
    // "x,m,seg,persistent[,segz]": fixed launch variant (tests, experiments);
    // seg is the y march segment, and the z march's too unless segz is given
    int x = 1, m = 1, sg = 32, pe = 0, sz = -1;
    const int got = std::sscanf(v, "%d,%d,%d,%d,%d", &x, &m, &sg, &pe, &sz);
    if (got == 4) sz = sg;
    const bool fx = c->fusable && (x == 0 || (x == 2 && cfg->precision != MHD_FP64));
    if ((got == 4 || got == 5) && (x == 1 || x == 3 || x == 4 || fx) &&
        (m >= 1 && m <= 10) &&
        sg >= 1 && sg <= 4096 && sz >= 1 && sz <= 4096 && (pe == 0 || pe == 1)) {
      c->var_x = x;
      c->var_m = m;
      c->var_seg = sg;
      c->var_segz = sz;
      c->var_pers = pe;
    }
  }
  if (const char* v = std::getenv("MHD_XCD")) c->var_xcd = std::atoi(v) & 31;
  rc = build_ctx(c, cfg);
  if (rc) {
    g_create_error = c->err;
    mhd_destroy(c);
    return rc;
  }
  *out = c;
  return MHD_OK;
}

int mhd_set_state(mhd_ctx* c, int32_t box, const double* const cons[5],
                  const double* const bface[3], double t, int32_t where) {
  int rc = check_box_index(c, box);
  if (rc) return rc;
  if (!cons || !bface) return fail(c, MHD_E_INVAL, "cons/bface is NULL");
  for (int q = 0; q < 5; q++)
    if (!cons[q]) return fail(c, MHD_E_INVAL, "cons array is NULL");
  for (int d = 0; d < 3; d++)
    if (!bface[d]) return fail(c, MHD_E_INVAL, "bface array is NULL");
  if (where != MHD_HOST && where != MHD_DEVICE) return fail(c, MHD_E_INVAL, "bad where");
  if (!std::isfinite(t)) return fail(c, MHD_E_INVAL, "t must be finite");
  const Geom& g = c->geom[box];
  const hipMemcpyKind kind = where == MHD_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  if (where == MHD_HOST) {
    for (int d = 0; d < 3; d++)
      if (g.per[d] && !host_periodic_ok(g, d, bface[d]))
        return fail(c, MHD_E_INVAL, "periodic axis " + std::to_string(d) +
                                        ": last face differs from the first");
  } else {
    int zero = 0;
    HIPCHK(c, hipMemcpyAsync(c->dflag, &zero, sizeof(int), hipMemcpyHostToDevice, c->stream));
    for (int d = 0; d < 3; d++) {
      if (!g.per[d]) continue;
      hipLaunchKernelGGL(mhd::k_check_periodic, dim3(256), dim3(kTPB), 0, c->stream, bface[d], d,
                         g.n[0], g.n[1], g.n[2], c->dflag);
    }
    HIPCHK(c, hipGetLastError());
    int bad = 0;
    HIPCHK(c, hipMemcpyAsync(&bad, c->dflag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (bad) return fail(c, MHD_E_INVAL, "periodic axis: last face differs from the first");
  }
  const Box& b = c->hbox[box];
  for (int q = 0; q < 5; q++)
    HIPCHK(c, hipMemcpyAsync(b.U[0][q], cons[q], g.N * 8, kind, c->stream));
  for (int d = 0; d < 3; d++) {
    rc = copy_faces(c, g, d, b.B[0][d], bface[d], true, kind);
    if (rc) return rc;
  }
  hipLaunchKernelGGL(k_reset_box, dim3(1), dim3(64), 0, c->stream, c->dbox, box, t);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->state_set[box] = 1;
  return MHD_OK;
}

int mhd_step(mhd_ctx* c, int32_t nsteps, double t_stop) {
  if (!c) return MHD_E_INVAL;
  if (nsteps < 0) return fail(c, MHD_E_INVAL, "nsteps < 0");
  if (!std::isfinite(t_stop)) return fail(c, MHD_E_INVAL, "t_stop must be finite");
  for (size_t b = 0; b < c->boxes.size(); b++)
    if (!c->state_set[b]) return fail(c, MHD_E_STATE, "mhd_step before mhd_set_state of every box");
  if (nsteps == 0) return MHD_OK;
  const int nb = (int)c->boxes.size();
  if ((c->flags & MHD_F_AUTOTUNE) && !c->tuned) {
    int rc = autotune(c);
    if (rc) return rc;
  }
  hipLaunchKernelGGL(k_set_scalar, dim3((nb + 255) / 256), dim3(256), 0, c->stream, c->dbox, nb, 2,
                     t_stop > 0.0 ? t_stop : 0.0);
  HIPCHK(c, hipGetLastError());
  if ((c->flags & MHD_F_GRAPH) && !(c->flags & MHD_F_TIMING)) {
    if (!c->gexec) {
      HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
      int rc = enqueue_step(c);
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(c->stream, &g);
      if (rc || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        if (rc) return rc;
      }
      if (e != hipSuccess) return fail(c, MHD_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
      c->graph = g;
      HIPCHK(c, hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
    }
    for (int s = 0; s < nsteps; s++) HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
  } else {
    for (int s = 0; s < nsteps; s++) {
      int rc = enqueue_step(c);
      if (rc) return rc;
    }
  }
  return MHD_OK;
}

int mhd_dt(mhd_ctx* c, int32_t box, double* dt_next, double* t) {
  int rc = check_box_index(c, box);
  if (rc) return rc;
  if (!c->state_set[box]) return fail(c, MHD_E_STATE, "mhd_dt before mhd_set_state");
  mhd::Launch L;
  L.boxes = c->dbox;
  L.base = c->dbase;
  L.nboxes = (int)c->boxes.size();
  L.stage = 0;
  L.lam = 0;
  L.xcd = 0;
  L.ntiles = c->total[mhd::kLAM];
  hipLaunchKernelGGL(mhd::k_lambda, dim3(std::max(1, L.ntiles)), dim3(kTPB), 0, c->stream, L);
  hipLaunchKernelGGL(mhd::k_dt, dim3(L.nboxes), dim3(kTPB), 0, c->stream, c->dbox, 1,
                     (int)mhd::kLAM);
  HIPCHK(c, hipGetLastError());
  double scal[4];
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(scal, c->hbox[box].scal, sizeof(scal), hipMemcpyDeviceToHost));
  if (dt_next) *dt_next = scal[3];
  if (t) *t = scal[1];
  unsigned long long cnt[3];
  rc = read_flags(c, box, cnt);
  if (rc) return rc;
  if (cnt[2]) return fail(c, MHD_E_NONPHYS, "non-physical cells were met");
  return MHD_OK;
}

int mhd_get_state(mhd_ctx* c, int32_t box, double* const cons[5], double* const bface[3],
                  double* t, int32_t where) {
  int rc = check_box_index(c, box);
  if (rc) return rc;
  if (!c->state_set[box]) return fail(c, MHD_E_STATE, "mhd_get_state before mhd_set_state");
  if (where != MHD_HOST && where != MHD_DEVICE) return fail(c, MHD_E_INVAL, "bad where");
  if (!cons || !bface) return fail(c, MHD_E_INVAL, "cons/bface is NULL");
  for (int q = 0; q < 5; q++)
    if (!cons[q]) return fail(c, MHD_E_INVAL, "cons array is NULL");
  for (int d = 0; d < 3; d++)
    if (!bface[d]) return fail(c, MHD_E_INVAL, "bface array is NULL");
  const Geom& g = c->geom[box];
  const Box& b = c->hbox[box];
  const hipMemcpyKind kind = where == MHD_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
  for (int q = 0; q < 5; q++)
    HIPCHK(c, hipMemcpyAsync(cons[q], b.U[0][q], g.N * 8, kind, c->stream));
  for (int d = 0; d < 3; d++) {
    rc = copy_faces(c, g, d, bface[d], b.B[0][d], false, kind);
    if (rc) return rc;
  }
  double scal[4];
  HIPCHK(c, hipMemcpyAsync(scal, b.scal, sizeof(scal), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (t) *t = scal[1];
  unsigned long long cnt[3];
  rc = read_flags(c, box, cnt);
  if (rc) return rc;
  if (cnt[2]) return fail(c, MHD_E_NONPHYS, "non-physical cells were met");
  return MHD_OK;
}

int mhd_counters(mhd_ctx* c, int32_t box, int64_t counters[3]) {
  int rc = check_box_index(c, box);
  if (rc) return rc;
  if (!counters) return fail(c, MHD_E_INVAL, "counters is NULL");
  unsigned long long cnt[3];
  rc = read_flags(c, box, cnt);
  if (rc) return rc;
  for (int k = 0; k < 3; k++) counters[k] = (int64_t)cnt[k];
  return MHD_OK;
}

int mhd_kernel_times(mhd_ctx* c, double ms[MHD_NKERNELS], int64_t launches[MHD_NKERNELS],
                     int32_t reset) {
  if (!c) return MHD_E_INVAL;
  if (!(c->flags & MHD_F_TIMING)) return fail(c, MHD_E_STATE, "context created without MHD_F_TIMING");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int k = 0; k < MHD_NKERNELS; k++) {
    if (ms) ms[k] = c->kms[k];
    if (launches) launches[k] = c->kcount[k];
    if (reset) {
      c->kms[k] = 0.0;
      c->kcount[k] = 0;
    }
  }
  return MHD_OK;
}

int mhd_tuning(mhd_ctx* c, int32_t variant[5]) {
  if (!c) return MHD_E_INVAL;
  if (!variant) return fail(c, MHD_E_INVAL, "variant is NULL");
  variant[0] = c->var_x;
  variant[1] = c->var_m;
  variant[2] = c->var_seg;
  variant[3] = c->var_pers;
  variant[4] = c->var_segz;
  return MHD_OK;
}

void mhd_destroy(mhd_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (auto& e : c->ev)
    if (e) (void)hipEventDestroy(e);
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  if (c->own_ws && c->ws) (void)hipFree(c->ws);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

const char* mhd_last_error(const mhd_ctx* c) {
  if (!c) return g_create_error.c_str();
  return c->err.c_str();
}

}  // extern "C"

// ---------------------------------------------------------------- no-alloc dt
//
// Device memory of the allocation-free time-step query: one partial maximum
// per tile of kTPB cells.  Each GPU the library runs on holds its own copy
// until the process ends.  Host code never uses the array's name as a device
// address: the address is looked up per device (hipGetSymbolAddress) on the
// entry point's first call on that device and cached below.
namespace {

constexpr int kScratchTiles = 1 << 20;  // 8 MiB: boxes of up to 2^28 cells
static __device__ __align__(256) double scratch[kScratchTiles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

int scratch_on_current_device(double** out, std::string& err) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    err = std::string("hipGetDevice: ") + hipGetErrorString(e);
    return MHD_E_DEVICE;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    err = "device index beyond the library's per-device table";
    return MHD_E_DEVICE;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return MHD_E_DEVICE;
    }
    g_scratch_ptr[dev] = (double*)p;
  }
  *out = g_scratch_ptr[dev];
  return MHD_OK;
}

}  // namespace

extern "C" int mhd_dt_noalloc(const mhd_box* box, const double* const cons[5],
                              const double* const bface[3], double p_floor, double* dt_out,
                              void* stream) {
  std::string err;
  if (!box) {
    g_create_error = "mhd_dt_noalloc: box is NULL";
    return MHD_E_INVAL;
  }
  int rc = validate_box(*box, err);
  if (rc) {
    g_create_error = "mhd_dt_noalloc: " + err;
    return rc;
  }
  const size_t N = (size_t)box->n[0] * box->n[1] * box->n[2];
  const size_t ntiles = (N + kTPB - 1) / kTPB;
  if (ntiles > (size_t)kScratchTiles) {
    g_create_error = "mhd_dt_noalloc: box of " + std::to_string(N) +
                     " cells exceeds the scratch capacity of " +
                     std::to_string((size_t)kScratchTiles * kTPB) + " cells";
    return MHD_E_INVAL;
  }
  if (!cons || !bface || !dt_out) {
    g_create_error = "mhd_dt_noalloc: cons, bface or dt_out is NULL";
    return MHD_E_INVAL;
  }
  for (int q = 0; q < 5; q++)
    if (!cons[q]) {
      g_create_error = "mhd_dt_noalloc: cons array is NULL";
      return MHD_E_INVAL;
    }
  for (int d = 0; d < 3; d++)
    if (!bface[d]) {
      g_create_error = "mhd_dt_noalloc: bface array is NULL";
      return MHD_E_INVAL;
    }
  if (!std::isfinite(p_floor)) {
    g_create_error = "mhd_dt_noalloc: p_floor must be finite";
    return MHD_E_INVAL;
  }
  double* part = nullptr;
  rc = scratch_on_current_device(&part, err);
  if (rc) {
    g_create_error = "mhd_dt_noalloc: " + err;
    return rc;
  }
  mhd::FlatBox f;
  for (int q = 0; q < 5; q++) f.U[q] = cons[q];
  for (int d = 0; d < 3; d++) {
    f.B[d] = bface[d];
    f.n[d] = box->n[d];
    f.act[d] = box->n[d] > 1;
    // the same cell size and reciprocal as a context's box descriptor
    const double dx = (box->hi[d] - box->lo[d]) / (double)box->n[d];
    f.idx[d] = 1.0 / dx;
  }
  f.gamma = box->gamma;
  f.pfloor = p_floor > 0.0 ? p_floor : 1e-10;
  f.cfl = box->cfl;
  f.ntiles = (int)ntiles;
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(mhd::k_lambda_flat, dim3((unsigned)ntiles), dim3(kTPB), 0, st, f, part);
  hipLaunchKernelGGL(mhd::k_dt_flat, dim3(1), dim3(kTPB), 0, st, (const double*)part, (int)ntiles,
                     box->cfl, dt_out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    g_create_error = std::string("mhd_dt_noalloc: launch: ") + hipGetErrorString(e);
    return MHD_E_DEVICE;
  }
  return MHD_OK;
}
