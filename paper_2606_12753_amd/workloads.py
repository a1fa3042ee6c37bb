"""Seeded synthetic inputs (initial states) of the ideal-MHD workloads.

This module holds only input recipes: it builds FP64 host arrays in the
boundary layout of the library (C order [z][y][x]; cell arrays nz*ny*nx; face
arrays with both bounding faces: Bx nz*ny*(nx+1), By nz*(ny+1)*nx,
Bz (nz+1)*ny*nx) and converts the primitive description of each initial
condition to conserved variables once, so that every consumer gets the same
bits.  It holds none of the scheme's arithmetic.

Random numbers come from ``numpy.random.default_rng(seed)`` (PCG64) drawn in
C order (z, y, x).  The paper (arXiv 2606.12753 §2.2.3) names its test
problems (3D Orszag-Tang, 2D Riemann) but prints no initial data, so the
recipes below are the standard textbook set-ups; each docstring states the
choices its recipe makes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

PERIODIC = 0
OUTFLOW = 1

GAMMA = 5.0 / 3.0


@dataclass
class BoxSpec:
    n: Tuple[int, int, int]
    lo: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    hi: Tuple[float, float, float] = (1.0, 1.0, 1.0)
    bc: Tuple[int, int, int] = (PERIODIC, PERIODIC, PERIODIC)
    gamma: float = GAMMA
    cfl: float = 0.3

    @property
    def cells(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])

    @property
    def dx(self):
        return tuple((self.hi[d] - self.lo[d]) / self.n[d] for d in range(3))


@dataclass
class State:
    cons: List[np.ndarray]   # rho, mx, my, mz, E  (nz, ny, nx)
    bface: List[np.ndarray]  # Bx, By, Bz (boundary face layout)
    t: float = 0.0

    def copy(self) -> "State":
        return State([c.copy() for c in self.cons], [b.copy() for b in self.bface], self.t)


@dataclass
class Workload:
    name: str
    boxes: List[BoxSpec]
    states: List[State]
    steps: int
    meta: dict = field(default_factory=dict)

    @property
    def cells(self) -> int:
        return sum(b.cells for b in self.boxes)


# ---------------------------------------------------------------------------
# coordinates

def centres(spec: BoxSpec, d: int) -> np.ndarray:
    return spec.lo[d] + (np.arange(spec.n[d]) + 0.5) * spec.dx[d]


def faces(spec: BoxSpec, d: int) -> np.ndarray:
    return spec.lo[d] + np.arange(spec.n[d] + 1) * spec.dx[d]


def _grid(spec: BoxSpec, stagger: int = -1):
    """Broadcastable (z, y, x) coordinates of cell centres, or of the faces
    normal to axis ``stagger``."""
    xs = [faces(spec, d) if d == stagger else centres(spec, d) for d in range(3)]
    return xs[2][:, None, None], xs[1][None, :, None], xs[0][None, None, :]


def face_shapes(spec: BoxSpec):
    nx, ny, nz = spec.n
    return [(nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx)]


def conserved(spec: BoxSpec, rho, vx, vy, vz, p, bface) -> State:
    """Total energy with the magnetic energy of the face-averaged field."""
    nx, ny, nz = spec.n
    shp = (nz, ny, nx)
    rho = np.broadcast_to(np.asarray(rho, dtype=np.float64), shp).copy()
    vx = np.broadcast_to(np.asarray(vx, dtype=np.float64), shp)
    vy = np.broadcast_to(np.asarray(vy, dtype=np.float64), shp)
    vz = np.broadcast_to(np.asarray(vz, dtype=np.float64), shp)
    p = np.broadcast_to(np.asarray(p, dtype=np.float64), shp)
    bx = 0.5 * (bface[0][:, :, :-1] + bface[0][:, :, 1:])
    by = 0.5 * (bface[1][:, :-1, :] + bface[1][:, 1:, :])
    bz = 0.5 * (bface[2][:-1, :, :] + bface[2][1:, :, :])
    en = (p / (spec.gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy + vz * vz)
          + 0.5 * (bx * bx + by * by + bz * bz))
    cons = [rho, rho * vx, rho * vy, rho * vz, en]
    cons = [np.ascontiguousarray(c, dtype=np.float64) for c in cons]
    bface = [np.ascontiguousarray(b, dtype=np.float64) for b in bface]
    return State(cons, bface, 0.0)


def periodic_faces(spec: BoxSpec, bface):
    """On periodic axes the last face is the first one: copy it exactly (a
    field sampled from a periodic function can differ in the last bit)."""
    for d in range(3):
        if spec.bc[d] == PERIODIC:
            last = [slice(None)] * 3
            first = [slice(None)] * 3
            last[2 - d] = slice(-1, None)
            first[2 - d] = slice(0, 1)
            bface[d][tuple(last)] = bface[d][tuple(first)]
    return bface


def _face_field(spec: BoxSpec, d: int, fn) -> np.ndarray:
    z, y, x = _grid(spec, stagger=d)
    val = fn(x, y, z)
    return np.array(np.broadcast_to(val, face_shapes(spec)[d]), dtype=np.float64, copy=True)


# ---------------------------------------------------------------------------
# workloads

def orszag_tang_2d(n: int = 128, steps: int = 50) -> Workload:
    """2D Orszag-Tang vortex on [0,1]^2, periodic, CFL 0.4.  Face fields are
    point samples at face centres (discretely divergence-free)."""
    spec = BoxSpec((n, n, 1), cfl=0.4)
    z, y, x = _grid(spec)
    s4 = math.sqrt(4.0 * math.pi)
    bface = [
        _face_field(spec, 0, lambda x, y, z: -np.sin(2 * np.pi * y) / s4 + 0 * x),
        _face_field(spec, 1, lambda x, y, z: np.sin(4 * np.pi * x) / s4 + 0 * y),
        _face_field(spec, 2, lambda x, y, z: 0.0 * x * y),
    ]
    bface = periodic_faces(spec, bface)
    st = conserved(spec, 25.0 / (36.0 * math.pi), -np.sin(2 * np.pi * y) + 0 * x,
                   np.sin(2 * np.pi * x) + 0 * y, 0.0, 5.0 / (12.0 * math.pi), bface)
    return Workload("orszag_tang_2d", [spec], [st], steps)


def blast_3d(n: int = 256, seed: int = 2606, steps: int = 100) -> Workload:
    """3D magnetised blast in the periodic unit cube: ambient rho=1 with
    seeded multiplicative noise 1e-6*U[-1,1), p=0.1, over-pressure 1000 in
    r<0.1 (cell centres), B = 10(1,1,1)/sqrt(3), CFL 0.3."""
    spec = BoxSpec((n, n, n), cfl=0.3)
    rng = np.random.default_rng(seed)
    xi = rng.uniform(-1.0, 1.0, size=(n, n, n))
    z, y, x = _grid(spec)
    r2 = (x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2
    p = np.where(r2 < 0.01, 1000.0, 0.1)
    rho = 1.0 * (1.0 + 1e-6 * xi)
    b0 = 10.0 / math.sqrt(3.0)
    bface = [np.full(s, b0) for s in face_shapes(spec)]
    st = conserved(spec, rho, 0.0, 0.0, 0.0, p, bface)
    return Workload("blast_3d", [spec], [st], steps, {"seed": seed})


def turbulence_3d(n: int = 512, seed: int = 2607, steps: int = 200,
                  k_peak: float = 4.0, v_rms: float = 0.5) -> Workload:
    """Decaying turbulence: rho=1, p=0.6, B=(1,0,0); solenoidal velocity with
    a Gaussian spectrum exp(-(|k|-k_peak)^2/2) (k in units of 2*pi),
    normalised to rms |v| = v_rms."""
    spec = BoxSpec((n, n, n), cfl=0.3)
    rng = np.random.default_rng(seed)
    kz = np.fft.fftfreq(n, d=1.0 / n)[:, None, None]
    ky = np.fft.fftfreq(n, d=1.0 / n)[None, :, None]
    kx = np.fft.rfftfreq(n, d=1.0 / n)[None, None, :]
    kk = np.sqrt(kx * kx + ky * ky + kz * kz)
    filt = np.exp(-0.5 * (kk - k_peak) ** 2)
    vh = []
    for _ in range(3):
        w = rng.standard_normal((n, n, n))
        vh.append(np.fft.rfftn(w) * filt)
        del w
    k2 = kx * kx + ky * ky + kz * kz
    k2[0, 0, 0] = 1.0
    div = (kx * vh[0] + ky * vh[1] + kz * vh[2]) / k2
    vh[0] = vh[0] - kx * div
    vh[1] = vh[1] - ky * div
    vh[2] = vh[2] - kz * div
    del div
    for c in vh:
        c[0, 0, 0] = 0.0
    v = [np.fft.irfftn(c, s=(n, n, n), axes=(0, 1, 2)) for c in vh]
    del vh
    rms = math.sqrt(float(np.mean(v[0] ** 2 + v[1] ** 2 + v[2] ** 2)))
    v = [c * (v_rms / rms) for c in v]
    bface = [np.full(face_shapes(spec)[0], 1.0), np.zeros(face_shapes(spec)[1]),
             np.zeros(face_shapes(spec)[2])]
    st = conserved(spec, 1.0, v[0], v[1], v[2], 0.6, bface)
    return Workload("turbulence_3d", [spec], [st], steps, {"seed": seed})


def ensemble(nboxes: int = 96, seed: int = 2608, steps: int = 100,
             sizes=(32, 48, 64, 96, 128)) -> Workload:
    """Ensemble of periodic unit boxes of uneven sizes, each an Orszag-Tang
    field extended in z with a random phase phi and a uniform guide field
    B_z = A (A in [0.1, 2])."""
    rng = np.random.default_rng(seed)
    ns = rng.choice(np.asarray(sizes), size=nboxes)
    phis = rng.uniform(0.0, 1.0, size=nboxes)
    amps = rng.uniform(0.1, 2.0, size=nboxes)
    boxes, states = [], []
    for n, phi, amp in zip(ns, phis, amps):
        spec, st = _orszag_tang_z(int(n), float(phi), float(amp))
        boxes.append(spec)
        states.append(st)
    return Workload("ensemble", boxes, states, steps,
                    {"seed": seed, "sizes": [int(v) for v in ns]})


def _orszag_tang_z(n: int, phi: float, amp: float, cfl: float = 0.3):
    """Orszag-Tang vortex on the periodic unit cube, extended along z by
    shifting the phase with z: rho = 25/(36 pi), p = 5/(12 pi),
    v = (-sin 2pi(y+phi+z), sin 2pi(x+phi+z), 0),
    B = (-sin 2pi(y+phi+z)/sqrt(4 pi), sin 4pi(x+phi+z)/sqrt(4 pi), amp),
    sampled at face centres (B_x does not vary along x nor B_y along y, so the
    discrete divergence is zero)."""
    s4 = math.sqrt(4.0 * math.pi)
    spec = BoxSpec((n, n, n), cfl=cfl)
    z, y, x = _grid(spec)
    bface = [
        _face_field(spec, 0, lambda x, y, z: -np.sin(2 * np.pi * (y + phi + z)) / s4 + 0 * x),
        _face_field(spec, 1, lambda x, y, z: np.sin(4 * np.pi * (x + phi + z)) / s4 + 0 * y),
        np.full(face_shapes(spec)[2], float(amp)),
    ]
    bface = periodic_faces(spec, bface)
    st = conserved(spec, 25.0 / (36.0 * math.pi), -np.sin(2 * np.pi * (y + phi + z)) + 0 * x,
                   np.sin(2 * np.pi * (x + phi + z)) + 0 * y, 0.0,
                   5.0 / (12.0 * math.pi), bface)
    return spec, st


def orszag_tang_3d(n: int = 352, steps: int = 10) -> Workload:
    """The paper's profiled workload, the 3D Orszag-Tang vortex on 352^3 cells
    for 10 steps with third-order Runge-Kutta.  Its initial data are not
    published: this is the 2D vortex extended along z (phase shifted with z,
    no guide field), CFL 0.3."""
    spec, st = _orszag_tang_z(n, 0.0, 0.0)
    return Workload("orszag_tang_3d", [spec], [st], steps, {"rk": 3})


def riemann_2d(n: int = 3200, steps: int = 10) -> Workload:
    """The paper's thin 2D case: a four-quadrant Riemann problem on n x n x 1
    cells of the unit square (3200^2 in the paper, solved with HLL at every
    face).  Its initial data are not published; these quadrant states are
    this code's own: rho = 1, p = 1 in the upper-right and lower-left
    quadrants, rho = 0.5, p = 0.35 in the other two; v = (0.75 left of
    x = 1/2, 0.75 below y = 1/2) componentwise, v_z = 0; uniform
    B = (0.5, 0.5, 0.25); gamma = 5/3, outflow walls, CFL 0.4, SSP-RK3.  The
    data are symmetric under the reflection x <-> y."""
    spec = BoxSpec((n, n, 1), bc=(OUTFLOW, OUTFLOW, PERIODIC), cfl=0.4)
    z, y, x = _grid(spec)
    right, top = x > 0.5, y > 0.5
    diag = right == top
    rho = np.where(diag, 1.0, 0.5) + 0 * z
    p = np.where(diag, 1.0, 0.35) + 0 * z
    vx = np.where(right, 0.0, 0.75) + 0 * y + 0 * z
    vy = np.where(top, 0.0, 0.75) + 0 * x + 0 * z
    bface = [np.full(s, v) for s, v in zip(face_shapes(spec), (0.5, 0.5, 0.25))]
    st = conserved(spec, rho, vx, vy, 0.0, p, bface)
    return Workload("riemann_2d", [spec], [st], steps, {"rk": 3, "solver": "hll"})


def kelvin_helmholtz(nx: int = 768, ny: int = 384, nz: int = 384, seed: int = 2609,
                     steps: int = 100) -> Workload:
    """Shear layer on [-1,1]x[-0.5,0.5]^2, periodic in x and z, outflow in y:
    rho = 2 for |y|<0.25 else 1, v_x = -0.5 tanh((|y|-0.25)/0.01),
    v_y = 1e-2 * U[-1,1) white noise, p = 2.5, B = (0.1, 0, 0)."""
    spec = BoxSpec((nx, ny, nz), lo=(-1.0, -0.5, -0.5), hi=(1.0, 0.5, 0.5),
                   bc=(PERIODIC, OUTFLOW, PERIODIC), cfl=0.3)
    rng = np.random.default_rng(seed)
    xi = rng.uniform(-1.0, 1.0, size=(nz, ny, nx))
    z, y, x = _grid(spec)
    ay = np.abs(y)
    rho = np.where(ay < 0.25, 2.0, 1.0) + 0 * x + 0 * z
    vx = -0.5 * np.tanh((ay - 0.25) / 0.01) + 0 * x + 0 * z
    vy = 1e-2 * xi
    bface = [np.full(face_shapes(spec)[0], 0.1), np.zeros(face_shapes(spec)[1]),
             np.zeros(face_shapes(spec)[2])]
    st = conserved(spec, rho, vx, vy, 0.0, 2.5, bface)
    return Workload("kelvin_helmholtz", [spec], [st], steps, {"seed": seed})


# ---------------------------------------------------------------------------
# test states

def uniform(n=(8, 8, 8), rho=1.3, v=(0.3, -0.2, 0.1), p=0.7, b=(0.5, -0.4, 0.25),
            bc=(PERIODIC, PERIODIC, PERIODIC), cfl=0.3) -> Workload:
    spec = BoxSpec(tuple(n), bc=tuple(bc), cfl=cfl)
    bface = [np.full(s, float(b[d])) for d, s in enumerate(face_shapes(spec))]
    st = conserved(spec, rho, v[0], v[1], v[2], p, bface)
    return Workload("uniform", [spec], [st], 1)


def cp_alfven(n: int, axis: int = 0, amp: float = 0.1, rho: float = 1.0, p: float = 0.1,
              b_par: float = 1.0, cfl: float = 0.4) -> Workload:
    """Circularly polarised Alfven wave along one axis (the others inactive),
    wavelength 1, travelling in +axis at v_A = b_par/sqrt(rho).  An exact
    nonlinear solution: after t = 1/v_A it equals the initial state."""
    nn = [1, 1, 1]
    nn[axis] = n
    spec = BoxSpec(tuple(nn), cfl=cfl)
    t1, t2 = (axis + 1) % 3, (axis + 2) % 3
    s = centres(spec, axis)
    bt1 = amp * np.sin(2 * np.pi * s)
    bt2 = amp * np.cos(2 * np.pi * s)
    va = b_par / math.sqrt(rho)

    def shape_along(vals, stagger_axis):
        shp = face_shapes(spec)[stagger_axis] if stagger_axis is not None else (nn[2], nn[1], nn[0])
        out = np.empty(shp)
        idx = [None, None, None]
        # broadcast the 1D profile along its axis (array axis 2 - axis)
        v = np.asarray(vals)
        view = [1, 1, 1]
        view[2 - axis] = v.size
        out[...] = v.reshape(view)
        return out

    bface = [None, None, None]
    bface[axis] = np.full(face_shapes(spec)[axis], b_par)
    bface[t1] = shape_along(bt1, t1)
    bface[t2] = shape_along(bt2, t2)
    bface = periodic_faces(spec, bface)
    v = [np.zeros((nn[2], nn[1], nn[0])) for _ in range(3)]
    v[t1] = shape_along(-bt1 / math.sqrt(rho), None)
    v[t2] = shape_along(-bt2 / math.sqrt(rho), None)
    st = conserved(spec, rho, v[0], v[1], v[2], p, bface)
    return Workload("cp_alfven", [spec], [st], 0, {"t_end": 1.0 / va, "axis": axis})


def cp_alfven_oblique(n: int, amp: float = 0.1, rho: float = 1.0, p: float = 0.1,
                      b_par: float = 1.0, cfl: float = 0.4) -> Workload:
    """Circularly polarised Alfven wave on a 2n x n periodic grid over
    [0,2]x[0,1], wave vector 2*pi*(1/2, 1) (oblique to both axes).  The
    in-plane perpendicular field comes from a vector potential sampled at
    cell corners, so the face field is discretely divergence-free."""
    spec = BoxSpec((2 * n, n, 1), lo=(0.0, 0.0, 0.0), hi=(2.0, 1.0, 1.0), cfl=cfl)
    kvec = np.array([0.5, 1.0])
    lam = 1.0 / np.linalg.norm(kvec)
    ca, sa = kvec / np.linalg.norm(kvec)
    dx, dy, _ = spec.dx

    def x1(x, y):
        return x * ca + y * sa

    # A_z(x, y) = amp*lam/(2 pi) cos(2 pi x1/lam)  ->  B2 = -dA/dx1 = amp sin(.)
    def az(x, y):
        return amp * lam / (2 * np.pi) * np.cos(2 * np.pi * x1(x, y) / lam)

    xf = faces(spec, 0)
    yf = faces(spec, 1)
    xc = centres(spec, 0)
    yc = centres(spec, 1)
    # Bx at (x_f, y_c) = dAz/dy ; By at (x_c, y_f) = -dAz/dx  (plus the guide field)
    bx = (az(xf[None, :], yf[1:, None]) - az(xf[None, :], yf[:-1, None])) / dy + b_par * ca
    by = -(az(xf[None, 1:], yf[:, None]) - az(xf[None, :-1], yf[:, None])) / dx + b_par * sa
    X, Y = xc[None, :], yc[:, None]
    ph = 2 * np.pi * x1(X, Y) / lam
    b2 = amp * np.sin(ph)
    b3 = amp * np.cos(ph)
    e2 = np.array([-sa, ca])
    vx = -b2 * e2[0] / math.sqrt(rho)
    vy = -b2 * e2[1] / math.sqrt(rho)
    vz = -b3 / math.sqrt(rho)
    bface = periodic_faces(spec, [bx[None, :, :].copy(), by[None, :, :].copy(),
                                  np.broadcast_to(b3[None, :, :], (2, n, 2 * n)).copy()])
    st = conserved(spec, rho, vx[None], vy[None], vz[None], p, bface)
    va = b_par / math.sqrt(rho)
    return Workload("cp_alfven_oblique", [spec], [st], 0, {"t_end": lam / va})


def random_smooth(n=(12, 10, 8), seed: int = 7, bc=(PERIODIC, PERIODIC, PERIODIC),
                  amp: float = 0.2, cfl: float = 0.3) -> Workload:
    """Random smooth-ish state (a few random Fourier modes) with a
    divergence-free face field from a random vector potential: exercises every
    branch of the scheme on small grids."""
    spec = BoxSpec(tuple(n), bc=tuple(bc), cfl=cfl,
                   hi=(1.0, 1.0 * n[1] / n[0], 1.0 * n[2] / n[0]))
    rng = np.random.default_rng(seed)
    z, y, x = _grid(spec)
    L = [spec.hi[d] - spec.lo[d] for d in range(3)]

    def field_(scale, offset, ncomp=4):
        out = offset + 0 * x * y * z
        for _ in range(ncomp):
            k = rng.integers(0, 3, size=3)
            ph = rng.uniform(0, 2 * np.pi)
            a = rng.uniform(-1, 1) * scale
            out = out + a * np.sin(2 * np.pi * (k[0] * x / L[0] + k[1] * y / L[1] + k[2] * z / L[2]) + ph)
        return out

    rho = field_(amp, 1.0)
    p = field_(amp, 1.0)
    vx, vy, vz = field_(0.5, 0.1), field_(0.5, -0.1), field_(0.5, 0.05)
    # vector potential at edges -> face field (discretely divergence-free)
    xf, yf, zf = faces(spec, 0), faces(spec, 1), faces(spec, 2)
    xc, yc, zc = centres(spec, 0), centres(spec, 1), centres(spec, 2)
    modes = [(rng.integers(0, 3, size=3), rng.uniform(0, 2 * np.pi), rng.uniform(-0.1, 0.1))
             for _ in range(9)]

    def pot(comp, X, Y, Z):
        out = 0.0 * X * Y * Z
        for m, (k, ph, a) in enumerate(modes):
            if m % 3 != comp:
                continue
            out = out + a * np.cos(2 * np.pi * (k[0] * X / L[0] + k[1] * Y / L[1] + k[2] * Z / L[2]) + ph)
        return out

    dx, dy, dz = spec.dx
    # A_x at (xc, yf, zf), A_y at (xf, yc, zf), A_z at (xf, yf, zc)
    Ax = pot(0, xc[None, None, :], yf[None, :, None], zf[:, None, None])
    Ay = pot(1, xf[None, None, :], yc[None, :, None], zf[:, None, None])
    Az = pot(2, xf[None, None, :], yf[None, :, None], zc[:, None, None])
    bx = (Az[:, 1:, :] - Az[:, :-1, :]) / dy - (Ay[1:, :, :] - Ay[:-1, :, :]) / dz
    by = (Ax[1:, :, :] - Ax[:-1, :, :]) / dz - (Az[:, :, 1:] - Az[:, :, :-1]) / dx
    bz = (Ay[:, :, 1:] - Ay[:, :, :-1]) / dx - (Ax[:, 1:, :] - Ax[:, :-1, :]) / dy
    b0 = rng.uniform(-0.5, 0.5, size=3)
    bface = periodic_faces(spec, [bx + b0[0], by + b0[1], bz + b0[2]])
    st = conserved(spec, rho, vx, vy, vz, p, [np.ascontiguousarray(b) for b in bface])
    return Workload("random_smooth", [spec], [st], 1, {"seed": seed})


def by_name(name: str, **kw) -> Workload:
    table = {
        "orszag_tang_2d": orszag_tang_2d,
        "blast_3d": blast_3d,
        "turbulence_3d": turbulence_3d,
        "ensemble": ensemble,
        "orszag_tang_3d": orszag_tang_3d,
        "riemann_2d": riemann_2d,
        "kelvin_helmholtz": kelvin_helmholtz,
    }
    return table[name](**kw)
