"""ctypes wrapper of the CPU oracle (TEST INFRASTRUCTURE ONLY).

The oracle itself is ``mhd_oracle.c``: a plain serial FP64 implementation of
the ideal-MHD finite-volume update of arXiv 2606.12753 §2.2.3 (reconstruct,
Riemann solve, conservative update per direction; constrained transport;
Runge-Kutta stepping).  This module only marshals numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_LIB = None

_dp = C.POINTER(C.c_double)

# Riemann solvers of the scheme (values of ORC_HLLD / ORC_HLL)
SOLVERS = {"hlld": 0, "hll": 1}
# reconstructions (values of ORC_REC_PRIM / ORC_REC_CHAR)
RECONS = {"prim": 0, "char": 1}
# corner EMFs (values of ORC_EMF_CONTACT / ORC_EMF_E0 / ORC_EMF_ARITH / ORC_EMF_UCT_HLL)
EMFS = {"contact": 0, "e0": 1, "arith": 2, "uct_hll": 3}
# slope limiters (values of ORC_LIM_MINMOD / ORC_LIM_MC / ORC_LIM_VANLEER)
LIMITERS = {"minmod": 0, "mc": 1, "vanleer": 2}


def _lib():
    global _LIB
    if _LIB is None:
        path = os.environ.get("MHD_ORACLE_LIB")
        if not path:
            path = os.path.join(_build.HERE, "liboracle.so")
            if not os.path.exists(path) or (
                os.path.getmtime(path) < os.path.getmtime(_build.SRC)
            ):
                _build.build()
        lib = C.CDLL(path)
        lib.orc_box_new.restype = C.c_void_p
        lib.orc_box_new.argtypes = [C.POINTER(C.c_int), _dp, _dp, C.POINTER(C.c_int),
                                    C.c_double, C.c_double, C.c_double]
        lib.orc_box_free.argtypes = [C.c_void_p]
        lib.orc_set_state.argtypes = [C.c_void_p, C.POINTER(_dp), C.POINTER(_dp), C.c_double]
        lib.orc_set_state.restype = C.c_int
        lib.orc_get_state.argtypes = [C.c_void_p, C.POINTER(_dp), C.POINTER(_dp), _dp]
        lib.orc_step.argtypes = [C.c_void_p, C.c_int, C.c_double]
        lib.orc_step_fixed_dt.argtypes = [C.c_void_p, C.c_double]
        lib.orc_set_rk.argtypes = [C.c_void_p, C.c_int]
        lib.orc_set_rk.restype = C.c_int
        lib.orc_set_solver.argtypes = [C.c_void_p, C.c_int]
        lib.orc_set_solver.restype = C.c_int
        lib.orc_set_recon.argtypes = [C.c_void_p, C.c_int]
        lib.orc_set_recon.restype = C.c_int
        lib.orc_set_emf.argtypes = [C.c_void_p, C.c_int]
        lib.orc_set_emf.restype = C.c_int
        lib.orc_ct_corner_kind.argtypes = [C.c_int] + [C.c_double] * 4 + [_dp] + [C.c_double] * 4
        lib.orc_ct_corner_kind.restype = C.c_double
        lib.orc_uct_hll.argtypes = [_dp] * 5
        lib.orc_uct_hll.restype = C.c_double
        lib.orc_prim_eigen.argtypes = [_dp, C.c_double, C.c_double, _dp, _dp, _dp]
        lib.orc_slope.argtypes = [_dp, _dp, _dp, C.c_double, C.c_double, C.c_int, C.c_int, _dp]
        lib.orc_set_limiter.argtypes = [C.c_void_p, C.c_int]
        lib.orc_set_limiter.restype = C.c_int
        lib.orc_limit.argtypes = [C.c_int, C.c_double, C.c_double]
        lib.orc_limit.restype = C.c_double
        lib.orc_threads.argtypes = [C.c_int]
        lib.orc_threads.restype = C.c_int
        lib.orc_dt.argtypes = [C.c_void_p]
        lib.orc_dt.restype = C.c_double
        lib.orc_rhs.argtypes = [C.c_void_p, C.POINTER(_dp), C.POINTER(_dp)]
        lib.orc_counters.argtypes = [C.c_void_p, C.POINTER(C.c_longlong)]
        lib.orc_divb_max.argtypes = [C.c_void_p]
        lib.orc_divb_max.restype = C.c_double
        lib.orc_cons_to_prim.argtypes = [_dp, _dp, C.c_double, C.c_double, _dp]
        lib.orc_cons_to_prim.restype = C.c_int
        lib.orc_fast_speed.argtypes = [C.c_double] * 6
        lib.orc_fast_speed.restype = C.c_double
        lib.orc_minmod.argtypes = [C.c_double, C.c_double]
        lib.orc_minmod.restype = C.c_double
        lib.orc_plm_face.argtypes = [C.c_double] * 4 + [_dp, _dp]
        lib.orc_phys_flux.argtypes = [_dp, C.c_double, C.c_double, _dp, _dp]
        lib.orc_hlld.argtypes = [_dp, _dp, C.c_double, C.c_double, _dp]
        lib.orc_hlld.restype = C.c_int
        lib.orc_hll.argtypes = [_dp, _dp, C.c_double, C.c_double, _dp]
        lib.orc_ct_mass_flux.argtypes = [_dp, _dp, C.c_double, C.c_double]
        lib.orc_ct_mass_flux.restype = C.c_double
        lib.orc_ct_corner.argtypes = [C.c_double] * 4 + [_dp] + [C.c_double] * 4
        lib.orc_ct_corner.restype = C.c_double
        _LIB = lib
    return _LIB


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _vec(x, n):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    assert a.shape == (n,)
    return a


class OracleBox:
    """One box of the oracle.  ``spec`` needs n, lo, hi, bc, gamma, cfl."""

    def __init__(self, spec, pfloor: float = 1e-10, rk: int = 2, solver: str = "hlld",
                 recon: str = "prim", emf: str = "contact", limiter: str = "minmod"):
        lib = _lib()
        self.spec = spec
        self.n = tuple(int(v) for v in spec.n)
        n = (C.c_int * 3)(*self.n)
        lo = (C.c_double * 3)(*spec.lo)
        hi = (C.c_double * 3)(*spec.hi)
        bc = (C.c_int * 3)(*spec.bc)
        self._h = lib.orc_box_new(n, lo, hi, bc, spec.gamma, spec.cfl, pfloor)
        if not self._h:
            raise ValueError("oracle: bad box description or out of memory")
        if lib.orc_set_rk(self._h, int(rk)) != 0:
            self.close()
            raise ValueError("oracle: rk must be 2 or 3")
        if solver not in SOLVERS or lib.orc_set_solver(self._h, SOLVERS[solver]) != 0:
            self.close()
            raise ValueError("oracle: solver must be 'hlld' or 'hll'")
        if recon not in RECONS or lib.orc_set_recon(self._h, RECONS[recon]) != 0:
            self.close()
            raise ValueError("oracle: recon must be 'prim' or 'char'")
        if emf not in EMFS or lib.orc_set_emf(self._h, EMFS[emf]) != 0:
            self.close()
            raise ValueError("oracle: emf must be 'contact', 'e0' or 'arith'")
        if limiter not in LIMITERS or lib.orc_set_limiter(self._h, LIMITERS[limiter]) != 0:
            self.close()
            raise ValueError("oracle: limiter must be 'minmod', 'mc' or 'vanleer'")

    def close(self):
        if self._h:
            _lib().orc_box_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def shapes(self):
        nx, ny, nz = self.n
        cell = (nz, ny, nx)
        faces = [(nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx)]
        return cell, faces

    def set_state(self, cons, bface, t=0.0):
        cell, faces = self.shapes()
        cons = [np.ascontiguousarray(c, dtype=np.float64) for c in cons]
        bface = [np.ascontiguousarray(b, dtype=np.float64) for b in bface]
        for c in cons:
            assert c.shape == cell
        for b, s in zip(bface, faces):
            assert b.shape == s
        cp = (_dp * 5)(*[_ptr(c) for c in cons])
        bp = (_dp * 3)(*[_ptr(b) for b in bface])
        rc = _lib().orc_set_state(self._h, cp, bp, float(t))
        if rc != 0:
            raise ValueError("oracle: periodic face mismatch")

    def get_state(self):
        cell, faces = self.shapes()
        cons = [np.empty(cell) for _ in range(5)]
        bface = [np.empty(s) for s in faces]
        t = C.c_double(0.0)
        cp = (_dp * 5)(*[_ptr(c) for c in cons])
        bp = (_dp * 3)(*[_ptr(b) for b in bface])
        _lib().orc_get_state(self._h, cp, bp, C.byref(t))
        return cons, bface, t.value

    def step(self, nsteps: int, t_stop: float = 0.0):
        _lib().orc_step(self._h, int(nsteps), float(t_stop))

    def step_fixed_dt(self, dt: float):
        _lib().orc_step_fixed_dt(self._h, float(dt))

    def dt(self) -> float:
        return _lib().orc_dt(self._h)

    def rhs(self):
        cell, faces = self.shapes()
        R = [np.empty(cell) for _ in range(5)]
        rB = [np.empty(s) for s in faces]
        rp = (_dp * 5)(*[_ptr(c) for c in R])
        bp = (_dp * 3)(*[_ptr(b) for b in rB])
        _lib().orc_rhs(self._h, rp, bp)
        return R, rB

    def counters(self):
        c = (C.c_longlong * 3)()
        _lib().orc_counters(self._h, c)
        return {"floor": c[0], "hll": c[1], "bad": c[2]}

    def divb_max(self) -> float:
        return _lib().orc_divb_max(self._h)


# ---- point functions ------------------------------------------------------

def cons_to_prim(u, bc, gamma, pfloor=1e-10):
    u = _vec(u, 5)
    bc = _vec(bc, 3)
    w = np.empty(8)
    fl = _lib().orc_cons_to_prim(_ptr(u), _ptr(bc), gamma, pfloor, _ptr(w))
    return w, fl


def fast_speed(rho, p, bn, bt1, bt2, gamma):
    return _lib().orc_fast_speed(rho, p, bn, bt1, bt2, gamma)


def minmod(a, b):
    return _lib().orc_minmod(a, b)


def plm_face(qm2, qm1, q0, qp1):
    ql = C.c_double()
    qr = C.c_double()
    _lib().orc_plm_face(qm2, qm1, q0, qp1, C.byref(ql), C.byref(qr))
    return ql.value, qr.value


def prim_eigen(w, bn, gamma):
    """Wave speeds (u-c_f, u-c_a, u-c_s, u, u+c_s, u+c_a, u+c_f), right
    eigenvectors R (columns) and left eigenvectors L (rows) of the
    primitive-variable system along one axis."""
    w = _vec(w, 7)
    lam = np.empty(7)
    R = np.empty((7, 7))
    L = np.empty((7, 7))
    _lib().orc_prim_eigen(_ptr(w), bn, gamma, _ptr(lam), _ptr(R), _ptr(L))
    return lam, R, L


def slope(qm, q0, qp, bn, gamma, recon="prim", limiter="minmod"):
    qm, q0, qp = _vec(qm, 7), _vec(q0, 7), _vec(qp, 7)
    d = np.empty(7)
    _lib().orc_slope(_ptr(qm), _ptr(q0), _ptr(qp), bn, gamma, RECONS[recon], LIMITERS[limiter],
                     _ptr(d))
    return d


def limit(a, b, limiter="minmod"):
    return _lib().orc_limit(LIMITERS[limiter], a, b)


def threads(n: int = 0) -> int:
    """Sets the oracle's thread count (n > 0); returns the count in use."""
    return _lib().orc_threads(int(n))


_TAG = b"MHDSTAT1"


def write_state(path, spec, cons, bface, t=0.0):
    """One box in the command-line oracle's state file (boundary layout)."""
    with open(path, "wb") as fh:
        fh.write(_TAG)
        fh.write(np.asarray(spec.n, dtype="<i4").tobytes())
        fh.write(np.asarray(spec.lo, dtype="<f8").tobytes())
        fh.write(np.asarray(spec.hi, dtype="<f8").tobytes())
        fh.write(np.asarray(spec.bc, dtype="<i4").tobytes())
        fh.write(np.asarray([spec.gamma, spec.cfl, t], dtype="<f8").tobytes())
        for a in list(cons) + list(bface):
            fh.write(np.ascontiguousarray(a, dtype="<f8").tobytes())


def read_state(path):
    """(n, lo, hi, bc, gamma, cfl, t, cons, bface) of a state file."""
    with open(path, "rb") as fh:
        raw = fh.read()
    if raw[:8] != _TAG:
        raise ValueError("not a state file")
    o = 8
    n = tuple(int(v) for v in np.frombuffer(raw, "<i4", 3, o)); o += 12
    lo = tuple(np.frombuffer(raw, "<f8", 3, o)); o += 24
    hi = tuple(np.frombuffer(raw, "<f8", 3, o)); o += 24
    bc = tuple(int(v) for v in np.frombuffer(raw, "<i4", 3, o)); o += 12
    gamma, cfl, t = np.frombuffer(raw, "<f8", 3, o); o += 24
    nx, ny, nz = n
    cons = []
    for _ in range(5):
        cons.append(np.frombuffer(raw, "<f8", nx * ny * nz, o).reshape(nz, ny, nx).copy())
        o += 8 * nx * ny * nz
    bface = []
    for shp in ((nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx)):
        cnt = shp[0] * shp[1] * shp[2]
        bface.append(np.frombuffer(raw, "<f8", cnt, o).reshape(shp).copy())
        o += 8 * cnt
    return n, lo, hi, bc, float(gamma), float(cfl), float(t), cons, bface


def phys_flux(w, bn, gamma):
    w = _vec(w, 7)
    f = np.empty(7)
    u = np.empty(7)
    _lib().orc_phys_flux(_ptr(w), bn, gamma, _ptr(f), _ptr(u))
    return f, u


def hlld(wl, wr, bn, gamma):
    wl = _vec(wl, 7)
    wr = _vec(wr, 7)
    f = np.empty(7)
    used_hll = _lib().orc_hlld(_ptr(wl), _ptr(wr), bn, gamma, _ptr(f))
    return f, bool(used_hll)


def hll(wl, wr, bn, gamma):
    wl = _vec(wl, 7)
    wr = _vec(wr, 7)
    f = np.empty(7)
    _lib().orc_hll(_ptr(wl), _ptr(wr), bn, gamma, _ptr(f))
    return f


def ct_mass_flux(wl, wr, bn, gamma):
    wl = _vec(wl, 7)
    wr = _vec(wr, 7)
    return _lib().orc_ct_mass_flux(_ptr(wl), _ptr(wr), bn, gamma)


def ct_corner(fa1, fa0, fb1, fb0, ec, ma1, ma0, mb1, mb0, kind="contact"):
    if kind not in ("contact", "e0", "arith"):
        raise ValueError("ct_corner averages face EMFs: contact, e0 or arith")
    ec = _vec(ec, 4)
    return _lib().orc_ct_corner_kind(EMFS[kind], fa1, fa0, fb1, fb0, _ptr(ec), ma1, ma0, mb1,
                                     mb0)


def uct_hll(va, vb, ba, bb, alpha):
    """Upwind-CT (HLL) corner EMF from the four corner states; see orc_uct_hll."""
    va, vb, ba, bb, alpha = _vec(va, 4), _vec(vb, 4), _vec(ba, 2), _vec(bb, 2), _vec(alpha, 4)
    return _lib().orc_uct_hll(_ptr(va), _ptr(vb), _ptr(ba), _ptr(bb), _ptr(alpha))


__all__ = [
    "OracleBox", "cons_to_prim", "fast_speed", "minmod", "plm_face", "phys_flux", "hlld",
    "hll", "ct_mass_flux", "ct_corner", "uct_hll", "prim_eigen", "slope", "limit", "threads", "write_state", "read_state", "SOLVERS", "RECONS",
    "EMFS", "LIMITERS",
]
