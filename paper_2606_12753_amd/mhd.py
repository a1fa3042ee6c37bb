"""Python binding of the C ABI in include/mhd.h (argument marshalling only).

Every step of the update runs in the HIP kernels of ``libmhd355.so``; this
module only converts arguments.  The library must have been built
(``paper_2606_12753_amd.build.build()``); there is no fallback.

Host arrays are numpy float64 arrays in the boundary layout of mhd.h (C order
[z][y][x]); device arrays are torch CUDA float64 tensors, passed by pointer.
PyTorch is used only for device memory and streams.
"""
from __future__ import annotations

import ctypes as C
import os
import warnings
from typing import Sequence

import numpy as np

from . import build as _build

MHD_OK = 0
MHD_E_INVAL = -1
MHD_E_NOMEM = -2
MHD_E_DEVICE = -3
MHD_E_NONPHYS = -4
MHD_E_STATE = -5

MHD_BC_PERIODIC = 0
MHD_BC_OUTFLOW = 1
MHD_FP64 = 0
MHD_MIXED = 1
MHD_HOST = 0
MHD_DEVICE = 1
MHD_F_GRAPH = 1
MHD_F_PERSISTENT = 2
MHD_F_TIMING = 4
MHD_F_AUTOTUNE = 8
MHD_RS_HLLD = 0
MHD_RS_HLL = 1
SOLVERS = {"hlld": MHD_RS_HLLD, "hll": MHD_RS_HLL}
MHD_REC_PRIM = 0
MHD_REC_CHAR = 1
RECONS = {"prim": MHD_REC_PRIM, "char": MHD_REC_CHAR}
MHD_EMF_CONTACT = 0
MHD_EMF_E0 = 1
MHD_EMF_ARITH = 2
MHD_EMF_UCT_HLL = 3
EMFS = {"contact": MHD_EMF_CONTACT, "e0": MHD_EMF_E0, "arith": MHD_EMF_ARITH,
        "uct_hll": MHD_EMF_UCT_HLL}
MHD_LIM_MINMOD = 0
MHD_LIM_MC = 1
MHD_LIM_VANLEER = 2
LIMITERS = {"minmod": MHD_LIM_MINMOD, "mc": MHD_LIM_MC, "vanleer": MHD_LIM_VANLEER}
KERNELS = ["lambda", "dt", "sweep_x", "sweep_y", "sweep_z", "ct_edge", "ct_face"]

EXPORTED = [
    "mhd_workspace_bytes", "mhd_create", "mhd_set_state", "mhd_step", "mhd_dt",
    "mhd_get_state", "mhd_counters", "mhd_kernel_times", "mhd_tuning",
    "mhd_destroy", "mhd_last_error", "mhd_dt_noalloc",
]


class MhdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mhd error {code}: {msg}")
        self.code = code


class mhd_box(C.Structure):
    _fields_ = [
        ("n", C.c_int32 * 3),
        ("lo", C.c_double * 3),
        ("hi", C.c_double * 3),
        ("bc_lo", C.c_int32 * 3),
        ("bc_hi", C.c_int32 * 3),
        ("gamma", C.c_double),
        ("cfl", C.c_double),
    ]


class mhd_config(C.Structure):
    _fields_ = [
        ("nboxes", C.c_int32),
        ("boxes", C.POINTER(mhd_box)),
        ("precision", C.c_int32),
        ("p_floor", C.c_double),
        ("stream", C.c_void_p),
        ("workspace", C.c_void_p),
        ("workspace_bytes", C.c_uint64),
        ("flags", C.c_uint32),
        ("rk_stages", C.c_int32),
        ("riemann", C.c_int32),
        ("recon", C.c_int32),
        ("ct_emf", C.c_int32),
        ("limiter", C.c_int32),
    ]


_LIB = None
_dp = C.POINTER(C.c_double)


def lib_path() -> str:
    return _build.LIB


def load():
    """Load libmhd355.so (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(_build.LIB):
        raise RuntimeError(
            f"{_build.LIB} is missing: build the HIP library first "
            "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = C.CDLL(_build.LIB)
    lib.mhd_workspace_bytes.argtypes = [C.POINTER(mhd_config), C.POINTER(C.c_uint64)]
    lib.mhd_create.argtypes = [C.POINTER(mhd_config), C.POINTER(C.c_void_p)]
    lib.mhd_set_state.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p),
                                  C.POINTER(C.c_void_p), C.c_double, C.c_int32]
    lib.mhd_step.argtypes = [C.c_void_p, C.c_int32, C.c_double]
    lib.mhd_dt.argtypes = [C.c_void_p, C.c_int32, _dp, _dp]
    lib.mhd_get_state.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p),
                                  C.POINTER(C.c_void_p), _dp, C.c_int32]
    lib.mhd_counters.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_int64)]
    lib.mhd_kernel_times.argtypes = [C.c_void_p, _dp, C.POINTER(C.c_int64), C.c_int32]
    lib.mhd_tuning.argtypes = [C.c_void_p, C.POINTER(C.c_int32)]
    lib.mhd_destroy.argtypes = [C.c_void_p]
    lib.mhd_destroy.restype = None
    lib.mhd_dt_noalloc.argtypes = [C.POINTER(mhd_box), C.POINTER(C.c_void_p),
                                   C.POINTER(C.c_void_p), C.c_double, C.c_void_p, C.c_void_p]
    lib.mhd_last_error.argtypes = [C.c_void_p]
    lib.mhd_last_error.restype = C.c_char_p
    for name in EXPORTED:
        if name not in ("mhd_destroy", "mhd_last_error"):
            getattr(lib, name).restype = C.c_int
    _LIB = lib
    return lib


def _box_struct(spec) -> mhd_box:
    b = mhd_box()
    for d in range(3):
        b.n[d] = int(spec.n[d])
        b.lo[d] = float(spec.lo[d])
        b.hi[d] = float(spec.hi[d])
        b.bc_lo[d] = int(spec.bc[d])
        b.bc_hi[d] = int(spec.bc[d])
    b.gamma = float(spec.gamma)
    b.cfl = float(spec.cfl)
    return b


def make_config(boxes: Sequence, precision: int = MHD_FP64, p_floor: float = 0.0,
                stream=None, workspace=None, workspace_bytes: int = 0, flags: int = 0,
                rk: int = 2, solver: str = "hlld", recon: str = "prim", emf: str = "contact",
                limiter: str = "minmod"):
    arr = (mhd_box * len(boxes))(*[_box_struct(s) for s in boxes])
    cfg = mhd_config()
    cfg.nboxes = len(boxes)
    cfg.boxes = C.cast(arr, C.POINTER(mhd_box))
    cfg.precision = int(precision)
    cfg.p_floor = float(p_floor)
    cfg.stream = stream
    cfg.workspace = workspace
    cfg.workspace_bytes = int(workspace_bytes)
    cfg.flags = int(flags)
    cfg.rk_stages = int(rk)
    cfg.riemann = SOLVERS[solver] if isinstance(solver, str) else int(solver)
    cfg.recon = RECONS[recon] if isinstance(recon, str) else int(recon)
    cfg.ct_emf = EMFS[emf] if isinstance(emf, str) else int(emf)
    cfg.limiter = LIMITERS[limiter] if isinstance(limiter, str) else int(limiter)
    return cfg, arr  # keep arr alive with cfg


def mhd_workspace_bytes(boxes, precision=MHD_FP64, flags=0, rk=2, solver="hlld",
                        recon="prim", emf="contact", limiter="minmod") -> int:
    lib = load()
    cfg, _keep = make_config(boxes, precision, flags=flags, rk=rk, solver=solver, recon=recon,
                             emf=emf, limiter=limiter)
    out = C.c_uint64()
    rc = lib.mhd_workspace_bytes(C.byref(cfg), C.byref(out))
    if rc != MHD_OK:
        raise MhdError(rc, lib.mhd_last_error(None).decode())
    return out.value


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


class Sim:
    """One library context: an ensemble of boxes advanced together."""

    def __init__(self, boxes: Sequence, precision: int = MHD_FP64, p_floor: float = 0.0,
                 stream=None, workspace=None, flags: int = 0, rk: int = 2,
                 solver: str = "hlld", recon: str = "prim", emf: str = "contact",
                 limiter: str = "minmod"):
        self._lib = load()
        self.boxes = list(boxes)
        self._h = None
        ws_ptr, ws_bytes = None, 0
        if workspace is not None:
            ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel() * workspace.element_size()
        self._workspace = workspace
        cfg, self._keep = make_config(self.boxes, precision, p_floor, stream, ws_ptr, ws_bytes,
                                      flags, rk, solver, recon, emf, limiter)
        h = C.c_void_p()
        rc = self._lib.mhd_create(C.byref(cfg), C.byref(h))
        if rc != MHD_OK:
            raise MhdError(rc, self._lib.mhd_last_error(None).decode())
        self._h = h
        self.nonphysical = False

    def _check(self, rc: int, allow_nonphys: bool = False):
        if rc == MHD_OK:
            return
        msg = self._lib.mhd_last_error(self._h).decode()
        if rc == MHD_E_NONPHYS and allow_nonphys:
            self.nonphysical = True
            warnings.warn(msg)
            return
        raise MhdError(rc, msg)

    def close(self):
        if self._h:
            self._lib.mhd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _shapes(self, box: int):
        nx, ny, nz = (int(v) for v in self.boxes[box].n)
        return (nz, ny, nx), [(nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx)]

    def _ptrs(self, arrays, shapes, writable: bool):
        ptrs = []
        dev = None
        for a, s in zip(arrays, shapes):
            if _is_torch(a):
                import torch
                if a.dtype != torch.float64 or tuple(a.shape) != tuple(s) or not a.is_contiguous():
                    raise ValueError(f"need a contiguous float64 tensor of shape {s}")
                d = MHD_DEVICE if a.is_cuda else MHD_HOST
                ptrs.append(a.data_ptr())
            else:
                if not isinstance(a, np.ndarray) or a.dtype != np.float64 or a.shape != tuple(s) \
                        or not a.flags.c_contiguous or (writable and not a.flags.writeable):
                    raise ValueError(f"need a C-contiguous float64 array of shape {s}")
                d = MHD_HOST
                ptrs.append(a.ctypes.data)
            if dev is None:
                dev = d
            elif dev != d:
                raise ValueError("all arrays of one call must live in the same memory")
        return ptrs, dev

    def set_state(self, box: int, cons, bface, t: float = 0.0):
        cell, faces = self._shapes(box)
        cons = [a if _is_torch(a) else np.ascontiguousarray(a, dtype=np.float64) for a in cons]
        bface = [a if _is_torch(a) else np.ascontiguousarray(a, dtype=np.float64) for a in bface]
        cp, w1 = self._ptrs(cons, [cell] * 5, False)
        bp, w2 = self._ptrs(bface, faces, False)
        if w1 != w2:
            raise ValueError("cons and bface must live in the same memory")
        ca = (C.c_void_p * 5)(*cp)
        ba = (C.c_void_p * 3)(*bp)
        self._check(self._lib.mhd_set_state(self._h, int(box), ca, ba, float(t), w1))

    def step(self, nsteps: int, t_stop: float = 0.0):
        self._check(self._lib.mhd_step(self._h, int(nsteps), float(t_stop)))

    def dt(self, box: int = 0):
        dt = C.c_double()
        t = C.c_double()
        self._check(self._lib.mhd_dt(self._h, int(box), C.byref(dt), C.byref(t)), True)
        return dt.value, t.value

    def get_state(self, box: int = 0, out=None):
        """Returns (cons, bface, t).  ``out`` = (cons, bface) preallocated
        arrays (numpy or torch CUDA tensors); default: new numpy arrays."""
        cell, faces = self._shapes(box)
        if out is None:
            cons = [np.empty(cell) for _ in range(5)]
            bface = [np.empty(s) for s in faces]
        else:
            cons, bface = out
        cp, w1 = self._ptrs(cons, [cell] * 5, True)
        bp, w2 = self._ptrs(bface, faces, True)
        if w1 != w2:
            raise ValueError("cons and bface must live in the same memory")
        ca = (C.c_void_p * 5)(*cp)
        ba = (C.c_void_p * 3)(*bp)
        t = C.c_double()
        self._check(self._lib.mhd_get_state(self._h, int(box), ca, ba, C.byref(t), w1), True)
        return cons, bface, t.value

    def kernel_times(self, reset: bool = False):
        """{kernel: (total ms, launches)} (context created with MHD_F_TIMING)."""
        ms = (C.c_double * len(KERNELS))()
        n = (C.c_int64 * len(KERNELS))()
        self._check(self._lib.mhd_kernel_times(self._h, ms, n, int(bool(reset))))
        return {k: (ms[i], int(n[i])) for i, k in enumerate(KERNELS)}

    def tuning(self):
        """Launch variant in use: (x direction: the x sweep's minimum waves
        per SIMD, or 0 / 2 for the fused x + y march; march variant; y march
        segment length; persistent grid; z march segment length), as
        mhd_tuning describes."""
        v = (C.c_int32 * 5)()
        self._check(self._lib.mhd_tuning(self._h, v))
        return tuple(int(x) for x in v)

    def counters(self, box: int = 0):
        c = (C.c_int64 * 3)()
        self._check(self._lib.mhd_counters(self._h, int(box), c))
        return {"floor": int(c[0]), "hll": int(c[1]), "bad": int(c[2])}


def dt_noalloc(spec, cons, bface, dt_out, p_floor: float = 0.0, stream=None):
    """Allocation-free CFL time step (mhd_dt_noalloc) of one box whose state
    is held in torch CUDA float64 tensors in the boundary layout; the step is
    written into ``dt_out`` (a CUDA float64 tensor of at least one element)
    on ``stream`` (a torch stream or None for the null stream), without
    waiting."""
    lib = load()
    nx, ny, nz = (int(v) for v in spec.n)
    shapes = [(nz, ny, nx)] * 5 + [(nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx)]
    arrays = list(cons) + list(bface) + [dt_out]
    import torch
    for a, s in zip(arrays, shapes + [None]):
        if not (_is_torch(a) and a.is_cuda and a.dtype == torch.float64 and a.is_contiguous()):
            raise ValueError("dt_noalloc needs contiguous CUDA float64 tensors")
        if s is not None and tuple(a.shape) != s:
            raise ValueError(f"need shape {s}, got {tuple(a.shape)}")
    if dt_out.numel() < 1:
        raise ValueError("dt_out needs one element")
    box = _box_struct(spec)
    ca = (C.c_void_p * 5)(*[a.data_ptr() for a in cons])
    ba = (C.c_void_p * 3)(*[a.data_ptr() for a in bface])
    st = None if stream is None else C.c_void_p(stream.cuda_stream)
    rc = lib.mhd_dt_noalloc(C.byref(box), ca, ba, float(p_floor), C.c_void_p(dt_out.data_ptr()), st)
    if rc != MHD_OK:
        raise MhdError(rc, lib.mhd_last_error(None).decode())
