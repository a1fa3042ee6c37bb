"""Pins of the oracle's point functions against facts fixed independently of
its own formulas: textbook special cases, eigen-structure of the flux
Jacobian, exactness properties of HLLD proven by Miyoshi & Kusano (2005),
symmetries of the equations, and the plane-parallel reduction of the
contact-upwinded CT average (Gardiner & Stone 2005)."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2606_12753_amd import workloads as W

G = 5.0 / 3.0


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(1e-300, float(np.max(np.abs(b)))))


def rand_state(rng, umag=1.0):
    return np.array([
        rng.uniform(0.2, 3.0),          # rho
        rng.uniform(-umag, umag),       # vn
        rng.uniform(-umag, umag),       # vt1
        rng.uniform(-umag, umag),       # vt2
        rng.uniform(0.05, 3.0),         # p
        rng.uniform(-2, 2),             # bt1
        rng.uniform(-2, 2),             # bt2
    ])


# ---------------------------------------------------------------- minmod/PLM

def test_minmod_cases():
    assert O.minmod(1.0, 2.0) == 1.0
    assert O.minmod(2.0, 1.0) == 1.0
    assert O.minmod(-1.0, -3.0) == -1.0
    assert O.minmod(-3.0, -1.0) == -1.0
    assert O.minmod(1.0, -1.0) == 0.0
    assert O.minmod(0.0, 5.0) == 0.0
    assert O.minmod(-2.0, 0.0) == 0.0


def test_plm_exact_on_linear_data():
    # a linear profile is reproduced exactly at the interface
    for a, s in [(0.3, 0.7), (-1.25, 2.5), (4.0, -0.5)]:
        q = [a + s * i for i in range(4)]          # cells c-2..c+1
        ql, qr = O.plm_face(*q)
        exact = a + s * 1.5                        # interface between c-1 and c
        assert ql == pytest.approx(exact, rel=1e-15, abs=1e-15)
        assert qr == pytest.approx(exact, rel=1e-15, abs=1e-15)


def test_plm_flat_at_extrema_and_bounded():
    # local maximum at c-1: its slope is zero, so q_L = q(c-1)
    ql, qr = O.plm_face(0.0, 2.0, 1.0, 0.5)
    assert ql == 2.0
    # TVD: interface values stay within the neighbouring cell values
    rng = np.random.default_rng(3)
    for _ in range(2000):
        q = rng.normal(size=4)
        ql, qr = O.plm_face(*q)
        assert min(q[0], q[1], q[2]) - 1e-15 <= ql <= max(q[0], q[1], q[2]) + 1e-15
        assert min(q[1], q[2], q[3]) - 1e-15 <= qr <= max(q[1], q[2], q[3]) + 1e-15


def test_plm_brute_force_tiny():
    # brute force over a small integer lattice against the limiter definition
    # (the smaller-magnitude one-sided difference when both agree in sign)
    vals = [-2.0, -1.0, 0.0, 1.0, 3.0]
    for a in vals:
        for b in vals:
            for c in vals:
                for d in vals:
                    ql, qr = O.plm_face(a, b, c, d)
                    s1 = [x for x in (b - a, c - b)]
                    s2 = [x for x in (c - b, d - c)]
                    def lim(u, v):
                        if u * v <= 0:
                            return 0.0
                        return u if abs(u) < abs(v) else v
                    assert ql == b + 0.5 * lim(*s1)
                    assert qr == c - 0.5 * lim(*s2)


# ---------------------------------------------------------------- cons/prim

def test_cons_prim_roundtrip():
    rng = np.random.default_rng(5)
    spec = W.BoxSpec((4, 3, 2))
    for _ in range(200):
        rho, p = rng.uniform(0.1, 5), rng.uniform(0.01, 5)
        v = rng.uniform(-3, 3, size=3)
        b = rng.uniform(-2, 2, size=3)
        bface = [np.full(s, b[d]) for d, s in enumerate(W.face_shapes(spec))]
        st = W.conserved(spec, rho, v[0], v[1], v[2], p, bface)
        u = [c[0, 0, 0] for c in st.cons]
        w, fl = O.cons_to_prim(u, b, G)
        assert fl == 0
        assert rel(w, [rho, *v, p, *b]) < 1e-12


def test_pressure_floor_and_bad_flags():
    w, fl = O.cons_to_prim([1.0, 0.0, 0.0, 0.0, 0.1], [1.0, 0.0, 0.0], G, 1e-10)
    assert fl & 1 and w[4] == 1e-10            # E below magnetic energy: floored
    w, fl = O.cons_to_prim([-1.0, 0.0, 0.0, 0.0, 1.0], [0.0, 0.0, 0.0], G)
    assert fl & 2                               # negative density flagged
    w, fl = O.cons_to_prim([np.nan, 0.0, 0.0, 0.0, 1.0], [0.0, 0.0, 0.0], G)
    assert fl & 2


# ---------------------------------------------------------------- wave speeds

def test_fast_speed_special_cases():
    rho, p = 1.7, 0.9
    a = math.sqrt(G * p / rho)
    # no field: sound speed
    assert O.fast_speed(rho, p, 0.0, 0.0, 0.0, G) == pytest.approx(a, rel=1e-15)
    # field along the normal: max(sound, Alfven)
    for bn in (0.3, 2.5):
        ca = abs(bn) / math.sqrt(rho)
        assert O.fast_speed(rho, p, bn, 0.0, 0.0, G) == pytest.approx(max(a, ca), rel=1e-14)
    # field perpendicular: sqrt(a^2 + b^2/rho)
    b1, b2 = 0.8, -0.6
    assert O.fast_speed(rho, p, 0.0, b1, b2, G) == pytest.approx(
        math.sqrt(a * a + (b1 * b1 + b2 * b2) / rho), rel=1e-14)


def test_flux_jacobian_eigenvalues():
    """The eigenvalues of dF/dU (7-wave system, face frame) are u, u +- c_a,
    u +- c_s, u +- c_f: pins the physical flux and the fast speed at once."""
    rng = np.random.default_rng(11)
    for _ in range(20):
        w = rand_state(rng)
        bn = rng.uniform(-1.5, 1.5)
        h = 1e-6
        # U(w) and F(w); J = dF/dw (dU/dw)^-1 by central differences
        dF = np.zeros((7, 7))
        dU = np.zeros((7, 7))
        for k in range(7):
            e = np.zeros(7)
            e[k] = h * max(1.0, abs(w[k]))
            fp, up = O.phys_flux(w + e, bn, G)
            fm, um = O.phys_flux(w - e, bn, G)
            dF[:, k] = (fp - fm) / (2 * e[k])
            dU[:, k] = (up - um) / (2 * e[k])
        J = dF @ np.linalg.inv(dU)
        ev = np.sort(np.linalg.eigvals(J).real)
        rho, u, p = w[0], w[1], w[4]
        bt2 = w[5] ** 2 + w[6] ** 2
        a2 = G * p / rho
        ca = abs(bn) / math.sqrt(rho)
        b2 = (bn * bn + bt2) / rho
        cf = O.fast_speed(rho, p, bn, w[5], w[6], G)
        cs2 = 0.5 * (a2 + b2 - math.sqrt(max(0.0, (a2 + b2) ** 2 - 4 * a2 * bn * bn / rho)))
        cs = math.sqrt(max(cs2, 0.0))
        exact = np.sort([u - cf, u - ca, u - cs, u, u + cs, u + ca, u + cf])
        assert np.allclose(ev, exact, atol=1e-5 * (abs(u) + cf)), (ev, exact)


def test_static_flux():
    w = np.array([1.3, 0.0, 0.0, 0.0, 0.7, 0.4, -0.9])
    bn = 0.6
    f, _ = O.phys_flux(w, bn, G)
    pt = 0.7 + 0.5 * (0.36 + 0.16 + 0.81)
    assert rel(f, [0.0, pt - 0.36, -0.6 * 0.4, -0.6 * -0.9, 0.0, 0.0, 0.0]) < 1e-15


# ---------------------------------------------------------------- HLLD

def test_hlld_consistency_random():
    rng = np.random.default_rng(21)
    for _ in range(500):
        w = rand_state(rng, umag=3.0)
        bn = rng.uniform(-2, 2)
        f, used = O.hlld(w, w, bn, G)
        fe, _ = O.phys_flux(w, bn, G)
        assert not used
        scale = np.max(np.abs(fe)) + 1.0
        assert np.max(np.abs(f - fe)) <= 5e-15 * scale * 10


def test_hlld_supersonic_upwind():
    rng = np.random.default_rng(22)
    for _ in range(50):
        wl = rand_state(rng)
        wr = rand_state(rng)
        wl[1] += 20.0
        wr[1] += 20.0
        f, _ = O.hlld(wl, wr, 0.3, G)
        fl, _ = O.phys_flux(wl, 0.3, G)
        assert np.array_equal(f, fl)
        wl[1] -= 40.0
        wr[1] -= 40.0
        f, _ = O.hlld(wl, wr, 0.3, G)
        fr, _ = O.phys_flux(wr, 0.3, G)
        assert np.array_equal(f, fr)


def test_hlld_isolated_stationary_contact():
    """A contact (density jump only, at rest) is resolved exactly: zero mass
    and energy flux, the momentum flux is the total pressure minus Bn^2."""
    for bn in (0.0, 0.75, -1.2):
        for bt in ((0.0, 0.0), (0.5, -0.3)):
            wl = np.array([1.0, 0.0, 0.0, 0.0, 0.8, bt[0], bt[1]])
            wr = np.array([0.125, 0.0, 0.0, 0.0, 0.8, bt[0], bt[1]])
            f, used = O.hlld(wl, wr, bn, G)
            assert not used
            pt = 0.8 + 0.5 * (bn * bn + bt[0] ** 2 + bt[1] ** 2)
            exact = [0.0, pt - bn * bn, -bn * bt[0], -bn * bt[1], 0.0, 0.0, 0.0]
            assert np.max(np.abs(f - exact)) < 1e-14


@pytest.mark.parametrize("family", [-1, +1])
@pytest.mark.parametrize("frame", [0.0, 0.37, -0.8])
def test_hlld_isolated_rotational_discontinuity(family, frame):
    """Two states joined by a rotational (Alfven) discontinuity alone: the
    HLLD flux equals the exact Godunov flux (Miyoshi & Kusano 2005)."""
    rho, p, bn = 1.4, 0.6, 0.9
    ca = bn / math.sqrt(rho)
    th = 1.1
    btl = np.array([0.7, -0.2])
    btr = np.array([math.cos(th) * btl[0] - math.sin(th) * btl[1],
                    math.sin(th) * btl[0] + math.cos(th) * btl[1]])
    # discontinuity speed relative to the fluid: family*ca; lab speed S
    # jump condition: [v_t] = -family * [B_t] / sqrt(rho) * sign(bn)
    vtl = np.array([0.1, 0.25])
    vtr = vtl - family * (btr - btl) / math.sqrt(rho)
    u = -family * ca + frame   # S = u + family*ca = frame
    wl = np.array([rho, u, vtl[0], vtl[1], p, btl[0], btl[1]])
    wr = np.array([rho, u, vtr[0], vtr[1], p, btr[0], btr[1]])
    f, used = O.hlld(wl, wr, bn, G)
    assert not used
    S = frame
    fl, ul = O.phys_flux(wl, bn, G)
    fr, ur = O.phys_flux(wr, bn, G)
    # Rankine-Hugoniot across the discontinuity holds for the constructed states
    assert np.max(np.abs((fr - fl) - S * (ur - ul))) < 1e-13
    exact = fl if S > 0 else (fr if S < 0 else fl)
    assert np.max(np.abs(f - exact)) < 1e-13, (f, exact)


def test_hlld_mirror_symmetry():
    rng = np.random.default_rng(31)
    sgn = np.array([-1, 1, -1, -1, -1, -1, -1], dtype=float)
    m = np.array([1, -1, 1, 1, 1, 1, 1], dtype=float)
    for _ in range(300):
        wl, wr = rand_state(rng, 2.0), rand_state(rng, 2.0)
        bn = rng.uniform(-2, 2)
        f, _ = O.hlld(wl, wr, bn, G)
        g, _ = O.hlld(wr * m, wl * m, -bn, G)
        assert np.max(np.abs(g - sgn * f)) <= 1e-13 * (1 + np.max(np.abs(f)))


def test_hlld_transverse_rotation():
    """Rotating the transverse plane by 90 degrees rotates the flux."""
    rng = np.random.default_rng(32)
    for _ in range(200):
        wl, wr = rand_state(rng, 2.0), rand_state(rng, 2.0)
        bn = rng.uniform(-2, 2)

        def rot(w):
            return np.array([w[0], w[1], -w[3], w[2], w[4], -w[6], w[5]])

        f, _ = O.hlld(wl, wr, bn, G)
        g, _ = O.hlld(rot(wl), rot(wr), bn, G)
        assert np.max(np.abs(g - rot(f))) <= 1e-13 * (1 + np.max(np.abs(f)))


def test_hlld_bn_to_zero_continuity():
    rng = np.random.default_rng(33)
    for _ in range(100):
        wl, wr = rand_state(rng), rand_state(rng)
        f0, _ = O.hlld(wl, wr, 0.0, G)
        f1, _ = O.hlld(wl, wr, 1e-7, G)
        assert np.max(np.abs(f1 - f0)) < 1e-5 * (1 + np.max(np.abs(f0)))


def test_hll_fallback_on_strong_rarefaction():
    # two streams flying apart: the HLLD star pressure is not positive
    wl = np.array([1.0, -30.0, 0.0, 0.0, 1e-4, 0.1, 0.0])
    wr = np.array([1.0, 30.0, 0.0, 0.0, 1e-4, 0.1, 0.0])
    f, used = O.hlld(wl, wr, 0.05, G)
    assert used
    assert np.all(np.isfinite(f))
    g = O.hll(wl, wr, 0.05, G)
    assert np.array_equal(f, g)
    # symmetric: zero mass flux through the centre
    assert abs(f[0]) < 1e-12


def _cf_textbook(w, bn):
    """Fast magnetosonic speed along n: the larger root of
    c^4 - (a^2 + b^2) c^2 + a^2 b_n^2 = 0 (a^2 = gamma p / rho, b = B/sqrt(rho))."""
    a2 = G * w[4] / w[0]
    b2 = (bn * bn + w[5] ** 2 + w[6] ** 2) / w[0]
    bn2 = bn * bn / w[0]
    return math.sqrt(0.5 * (a2 + b2 + math.sqrt((a2 + b2) ** 2 - 4.0 * a2 * bn2)))


def _textbook_flux_state(w, bn):
    """Physical flux and conserved vector of a face-frame state, from the
    ideal-MHD conservation laws (7 components: rho, m_n, m_t1, m_t2, E,
    B_t1, B_t2)."""
    rho, u, v1, v2, p, b1, b2 = w
    bsq = bn * bn + b1 * b1 + b2 * b2
    pt = p + 0.5 * bsq
    en = p / (G - 1.0) + 0.5 * rho * (u * u + v1 * v1 + v2 * v2) + 0.5 * bsq
    vb = u * bn + v1 * b1 + v2 * b2
    U = np.array([rho, rho * u, rho * v1, rho * v2, en, b1, b2])
    F = np.array([rho * u, rho * u * u + pt - bn * bn, rho * u * v1 - bn * b1,
                  rho * u * v2 - bn * b2, (en + pt) * u - bn * vb, u * b1 - v1 * bn,
                  u * b2 - v2 * bn])
    return F, U


def _star_thermal_pressures(wl, wr, bn):
    """Outer speeds, contact speed, star total pressure and the two
    single-star thermal pressures of Miyoshi & Kusano (2005), from their
    jump conditions: mass and momentum balance across S_L and S_R with one
    normal velocity S_M and one total pressure in the star region (this
    only decides which branch the state exercises)."""
    c = max(_cf_textbook(wl, bn), _cf_textbook(wr, bn))
    sl, sr = min(wl[1], wr[1]) - c, max(wl[1], wr[1]) + c
    pt = [w[4] + 0.5 * (bn * bn + w[5] ** 2 + w[6] ** 2) for w in (wl, wr)]
    ml, mr = wl[0] * (sl - wl[1]), wr[0] * (sr - wr[1])  # mass fluxes through S_L, S_R
    sm = (mr * wr[1] - ml * wl[1] - pt[1] + pt[0]) / (mr - ml)
    pts = pt[0] + ml * (sm - wl[1])  # momentum jump across S_L
    ps = []
    for w, s, m, ptw in ((wl, sl, ml, pt[0]), (wr, sr, mr, pt[1])):
        rs = m / (s - sm)
        den = m * (s - sm) - bn * bn
        bt = [b * (m * (s - w[1]) - bn * bn) / den for b in (w[5], w[6])]
        vt = [v - bn * b * (sm - w[1]) / den for v, b in ((w[2], w[5]), (w[3], w[6]))]
        en = _textbook_flux_state(w, bn)[1][4]
        vb = w[1] * bn + w[2] * w[5] + w[3] * w[6]
        vbs = sm * bn + vt[0] * bt[0] + vt[1] * bt[1]
        ens = ((s - w[1]) * en - ptw * w[1] + pts * sm + bn * (vb - vbs)) / (s - sm)
        ps.append((G - 1.0) * (ens - 0.5 * rs * (sm * sm + vt[0] ** 2 + vt[1] ** 2)
                               - 0.5 * (bn * bn + bt[0] ** 2 + bt[1] ** 2)))
    return sl, sr, sm, pts, ps


@pytest.mark.parametrize("mirror", [False, True])
def test_hll_fallback_on_negative_star_thermal_pressure(mirror):
    """A cold stationary jump of density and tangential field (B_n = 1,
    p = 0.001): the contact speed lies strictly between the outer speeds
    and the star total pressure is positive, but the single-star state on
    the weak-field side would need a negative thermal pressure (the
    compressed field alone exceeds the star total pressure).  The HLLD star
    states are then not physical and the solver must return the HLL flux,
    written out here from its closed form (Harten, Lax & van Leer 1983) with
    the same outer speeds, and flag the fallback."""
    wl = np.array([0.5, 0.0, 0.0, 0.0, 0.001, -1.5, 0.0])
    wr = np.array([0.2, 0.0, 0.0, 0.0, 0.001, -0.5, 0.0])
    bn = 1.0
    if mirror:  # the same jump seen from the other side: x -> -x
        flip = np.array([1.0, -1.0, 1.0, 1.0, 1.0, 1.0, 1.0])
        wl, wr = wr * flip, wl * flip
        bn = -bn
    sl, sr, sm, pts, ps = _star_thermal_pressures(wl, wr, bn)
    assert sl < sm < sr and pts > 0.0
    assert min(ps) < -0.4 * pts and max(ps) > 0.0
    f, used = O.hlld(wl, wr, bn, G)
    assert used
    fl, ul = _textbook_flux_state(wl, bn)
    fr, ur = _textbook_flux_state(wr, bn)
    hll = (sr * fl - sl * fr + sl * sr * (ur - ul)) / (sr - sl)
    assert np.max(np.abs(f - hll)) <= 1e-14 * np.max(np.abs(hll)), (f, hll)
    # the scheme counts the fallback: one x sweep over a two-state tube
    # (piecewise constant, so the face at the jump sees exactly wl | wr)
    spec = W.BoxSpec((8, 1, 1), bc=(W.OUTFLOW, W.PERIODIC, W.PERIODIC), gamma=G)
    rho = np.where(np.arange(8) < 4, wl[0], wr[0]).reshape(1, 1, 8)
    by = np.where(np.arange(8) < 4, wl[5], wr[5]).reshape(1, 1, 8)
    bface = [np.full((1, 1, 9), bn), np.broadcast_to(by, (1, 2, 8)).copy(),
             np.broadcast_to(np.zeros((1, 1, 8)), (2, 1, 8)).copy()]
    st = W.conserved(spec, rho, 0.0, 0.0, 0.0, 0.001 + 0 * rho, bface)
    ob = O.OracleBox(spec)
    ob.set_state(st.cons, st.bface)
    ob.rhs()
    assert ob.counters()["hll"] == 1


@pytest.mark.parametrize("degenerate_side", ["left", "right"])
def test_hlld_degenerate_star_denominator_stationary_contact(degenerate_side):
    """An isolated stationary contact (density jump at rest, equal pressure
    and field) whose low-density side has an Alfven speed above its sound
    speed and a tangential field of 1e-7 B_n: its fast speed, the outer
    speed of that side, then equals its Alfven speed to O(B_t^2), so the
    single-star denominator rho (S - u)(S - S_M) - B_n^2 vanishes to
    rounding (the degenerate case of Miyoshi & Kusano 2005), while B_t is
    not zero.  The solver must still resolve the contact exactly (a property
    of HLLD proven in that paper): zero mass, energy and tangential-field
    flux, normal momentum flux p_T - B_n^2, tangential momentum flux
    -B_n B_t.  The limit of the star-state formulas as S_M -> u fixes the
    tangential star velocity and field to the side's own values; any other
    value enters the flux through the star or double-star states."""
    bn, p, bt = 1.0, 0.1, 1e-7
    lo, hi = 0.5, 1.0  # densities: Alfven speed 1.41 > sound speed 0.58 at 0.5
    rl, rr = (lo, hi) if degenerate_side == "left" else (hi, lo)
    wl = np.array([rl, 0.0, 0.0, 0.0, p, bt, -bt])
    wr = np.array([rr, 0.0, 0.0, 0.0, p, bt, -bt])
    c = max(_cf_textbook(wl, bn), _cf_textbook(wr, bn))
    w = wl if degenerate_side == "left" else wr
    s = -c if degenerate_side == "left" else c
    pt = p + 0.5 * (bn * bn + 2 * bt * bt)
    assert abs(w[0] * s * s - bn * bn) <= 1e-12 * pt  # degenerate denominator (S_M = u = 0)
    f, used = O.hlld(wl, wr, bn, G)
    assert not used
    exact = np.array([0.0, pt - bn * bn, -bn * bt, bn * bt, 0.0, 0.0, 0.0])
    assert np.max(np.abs(f - exact)) <= 1e-15 * c * pt, (f, exact)


def test_hll_consistency():
    rng = np.random.default_rng(34)
    for _ in range(100):
        w = rand_state(rng)
        bn = rng.uniform(-2, 2)
        f = O.hll(w, w, bn, G)
        fe, _ = O.phys_flux(w, bn, G)
        assert np.max(np.abs(f - fe)) <= 1e-13 * (1 + np.max(np.abs(fe)))


# ---------------------------------------------------------------- CT corner

def test_ct_plane_parallel_reduction():
    """Grid-aligned plane-parallel flow: the corner EMF equals the face EMF
    of the direction of variation, whatever the transverse mass flux."""
    rng = np.random.default_rng(41)
    for _ in range(200):
        F = rng.normal()
        ec_lo, ec_hi = rng.normal(size=2)       # cells ia-1, ia
        m = rng.normal(size=2)
        mt = rng.choice([-1.0, 0.0, 1.0])
        # variation along a: a-faces carry F, b-faces carry the cell values
        ec = np.array([ec_lo, ec_hi, ec_lo, ec_hi])
        e = O.ct_corner(F, F, ec_hi, ec_lo, ec, m[0], m[0], mt, mt)
        assert e == pytest.approx(F, abs=1e-14 * (1 + abs(F) + abs(ec_lo) + abs(ec_hi)))
        # variation along b: b-faces carry G, a-faces the cell values (ib, ib-1)
        ec = np.array([ec_lo, ec_lo, ec_hi, ec_hi])
        e = O.ct_corner(ec_hi, ec_lo, F, F, ec, mt, mt, m[1], m[1])
        assert e == pytest.approx(F, abs=1e-14 * (1 + abs(F) + abs(ec_lo) + abs(ec_hi)))


def test_ct_corner_kinds():
    """E0 (Gardiner & Stone): the contact formula with every derivative
    averaged, so independent of the mass fluxes and equal to the contact
    average where they vanish; it still reduces to the face EMF for a
    grid-aligned plane-parallel flow.  The arithmetic mean (Balsara &
    Spicer) ignores the cell EMFs and does not reduce: for variation along
    a it gives F/2 + (E_c(ia-1) + E_c(ia))/4."""
    rng = np.random.default_rng(43)
    for _ in range(200):
        f = rng.normal(size=4)
        ec = rng.normal(size=4)
        m = rng.normal(size=4)
        e0 = O.ct_corner(*f, ec, *m, kind="e0")
        assert e0 == O.ct_corner(*f, ec, 0.0, 0.0, 0.0, 0.0, kind="contact")
        assert e0 == O.ct_corner(*f, ec, *rng.normal(size=4), kind="e0")
        ar = O.ct_corner(*f, ec, *m, kind="arith")
        assert ar == pytest.approx(0.25 * sum(f), abs=1e-15 * (1 + np.sum(np.abs(f))))
        assert ar == O.ct_corner(*f, rng.normal(size=4), *rng.normal(size=4), kind="arith")
        F = rng.normal()
        ec_lo, ec_hi = rng.normal(size=2)
        ec2 = np.array([ec_lo, ec_hi, ec_lo, ec_hi])
        tol = 1e-14 * (1 + abs(F) + abs(ec_lo) + abs(ec_hi))
        assert O.ct_corner(F, F, ec_hi, ec_lo, ec2, *m, kind="e0") == pytest.approx(F, abs=tol)
        ar = O.ct_corner(F, F, ec_hi, ec_lo, ec2, *m, kind="arith")
        assert ar == pytest.approx(0.5 * F + 0.25 * (ec_lo + ec_hi), abs=tol)


def test_ct_upwind_selection():
    """With all transverse derivatives on one side zero and the other side
    non-zero, the sign of the mass flux picks which side contributes."""
    ec = np.array([0.0, 0.0, 0.0, 1.0])      # only cell (ia, ib) non-zero
    faces = (0.0, 0.0, 0.0, 0.0)
    # flux > 0 through both faces: upwind = lower cells, which are all zero
    assert O.ct_corner(*faces, ec, 1.0, 1.0, 1.0, 1.0) == 0.0
    # flux < 0 through both: upper cells, (ia, ib) enters d_b+ and d_a+
    e = O.ct_corner(*faces, ec, -1.0, -1.0, -1.0, -1.0)
    assert e == pytest.approx(-0.5)
    # zero flux: averages -> half weight
    e = O.ct_corner(*faces, ec, 0.0, 0.0, 0.0, 0.0)
    assert e == pytest.approx(-0.25)


# ---------------------------------------------------------------- characteristic reconstruction

def prim_jacobian(w, bn, gamma):
    """Coefficient matrix A of the primitive-variable ideal-MHD equations
    along x, dW/dt + A dW/dx = 0, W = (rho, u, v, w, p, B_y, B_z), B_x = bn,
    written out from continuity, momentum, pressure and induction."""
    rho, u, v, ww, p, by, bz = w
    A = np.zeros((7, 7))
    A[0, 0], A[0, 1] = u, rho
    A[1, 1], A[1, 4], A[1, 5], A[1, 6] = u, 1 / rho, by / rho, bz / rho
    A[2, 2], A[2, 5] = u, -bn / rho
    A[3, 3], A[3, 6] = u, -bn / rho
    A[4, 1], A[4, 4] = gamma * p, u
    A[5, 1], A[5, 2], A[5, 5] = by, -bn, u
    A[6, 1], A[6, 3], A[6, 6] = bz, -bn, u
    return A


def eigen_states():
    rng = np.random.default_rng(17)
    out = [(rand_state(rng)[[0, 1, 2, 3, 4, 5, 6]], rng.uniform(-2, 2)) for _ in range(300)]
    rho, p = 1.2, 0.7
    a = math.sqrt(G * p / rho)
    out += [
        (np.array([rho, 0.1, 0.2, -0.3, p, 0.0, 0.0]), 0.9),        # B along the normal
        (np.array([rho, 0.1, 0.2, -0.3, p, 0.5, -0.4]), 0.0),       # B_n = 0
        (np.array([rho, 0.1, 0.2, -0.3, p, 0.0, 0.0]), 0.0),        # no field
        (np.array([rho, 0.1, 0.2, -0.3, p, 0.0, 0.0]), a * math.sqrt(rho)),   # c_A = a, B_t = 0
        (np.array([rho, 0.1, 0.2, -0.3, p, 1e-9, 2e-9]), 0.8),      # B_t nearly 0
        (np.array([rho, 0.1, 0.2, -0.3, p, 0.3, 0.4]), -1.1),       # B_n < 0
    ]
    return out


def test_prim_eigenvectors_solve_the_jacobian():
    """A R_k = lambda_k R_k for every wave, L R = I, and the wave speeds equal
    the eigenvalues of A (numpy) and the fast speed of the flux code."""
    for w, bn in eigen_states():
        lam, R, L = O.prim_eigen(w, bn, G)
        A = prim_jacobian(w, bn, G)
        scale = np.max(np.abs(A)) * max(1.0, np.max(np.abs(R)))
        assert np.max(np.abs(A @ R - R * lam)) <= 1e-12 * scale, (w, bn)
        assert np.max(np.abs(L @ R - np.eye(7))) <= 1e-12, (w, bn)
        ev = np.sort(np.linalg.eigvals(A).real)
        assert np.allclose(np.sort(lam), ev, rtol=0, atol=1e-7 * (1 + np.max(np.abs(ev)))), (w, bn)
        cf = O.fast_speed(w[0], w[4], bn, w[5], w[6], G)
        assert lam[6] - w[1] == pytest.approx(cf, rel=1e-13)
        assert np.all(np.diff(lam) >= -1e-12 * (1 + abs(w[1])))


def test_char_slope_exact_on_linear_data():
    rng = np.random.default_rng(3)
    for _ in range(100):
        q0 = rand_state(rng)
        dq = 0.01 * rng.uniform(-1, 1, 7)
        bn = rng.uniform(-1, 1)
        for rec in ("prim", "char"):
            d = O.slope(q0 - dq, q0, q0 + dq, bn, G, rec)
            assert np.allclose(d, dq, rtol=0, atol=1e-13), rec


def test_char_slope_limits_each_wave_separately():
    """Differences made of right eigenvectors: each characteristic field is
    limited on its own (minmod of its two amplitudes), so a field whose
    amplitude changes sign drops out while the others keep the smaller
    amplitude; the primitive slope mixes them instead."""
    rng = np.random.default_rng(5)
    for _ in range(100):
        q0 = rand_state(rng)
        bn = rng.uniform(-1, 1)
        lam, R, L = O.prim_eigen(q0, bn, G)
        k, j = rng.choice(7, size=2, replace=False)
        am, ap = rng.uniform(0.1, 1.0, 2) * 1e-3
        gm, gp = rng.uniform(0.1, 1.0, 2) * 1e-3
        dm = am * R[:, k] + gm * R[:, j]
        dp = -ap * R[:, k] + gp * R[:, j]
        d = O.slope(q0 - dm, q0, q0 + dp, bn, G, "char")
        want = min(gm, gp) * R[:, j]
        assert np.allclose(d, want, rtol=0, atol=1e-12 * (1 + np.max(np.abs(R)))), (k, j)


def test_char_slope_mirror_antisymmetric():
    """Reversing the stencil negates the slope exactly (both reconstructions)."""
    rng = np.random.default_rng(9)
    for _ in range(200):
        qm, q0, qp = rand_state(rng), rand_state(rng), rand_state(rng)
        bn = rng.uniform(-1, 1)
        for rec in ("prim", "char"):
            a = O.slope(qm, q0, qp, bn, G, rec)
            b = O.slope(qp, q0, qm, bn, G, rec)
            assert np.array_equal(a, -b) or np.array_equal(a + b, np.zeros(7)), rec


def test_char_slope_falls_back_where_faces_lose_positivity():
    """A slope that would make a face density non-positive is replaced by the
    primitive minmod slope."""
    q0 = np.array([0.1, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0])
    bn = 0.0
    lam, R, L = O.prim_eigen(q0, bn, G)
    # a strong fast wave on both sides: rho changes by 0.3 per cell
    amp = 0.3 / R[0, 6]
    dm = amp * R[:, 6]
    dm[0] = 0.05         # primitive density difference small on one side
    dp = amp * R[:, 6]
    d = O.slope(q0 - dm, q0, q0 + dp, bn, G, "char")
    prim = O.slope(q0 - dm, q0, q0 + dp, bn, G, "prim")
    lam_, R_, L_ = O.prim_eigen(q0, bn, G)
    ch = [O.minmod(float(L_[k] @ dm), float(L_[k] @ dp)) for k in range(7)]
    raw = R_ @ np.array(ch)
    assert not (q0[0] - 0.5 * abs(raw[0]) > 0)   # the characteristic slope is rejected
    assert np.array_equal(d, prim)


# ---------------------------------------------------------------- slope limiters

def test_limiters_match_their_flux_limiter_functions():
    """In Sweby's form slope = phi(r) b with r = a/b: minmod phi = max(0,
    min(r, 1)); monotonised central phi = max(0, min(2r, (1 + r)/2, 2));
    van Leer phi = (r + |r|)/(1 + |r|).  All three lie in the TVD region
    0 <= phi <= min(2r, 2) and have phi(1) = 1."""
    rng = np.random.default_rng(61)
    phis = {
        "minmod": lambda r: max(0.0, min(r, 1.0)),
        "mc": lambda r: max(0.0, min(2 * r, 0.5 * (1 + r), 2.0)),
        "vanleer": lambda r: (r + abs(r)) / (1 + abs(r)),
    }
    for _ in range(2000):
        b = rng.choice([-1, 1]) * 10 ** rng.uniform(-3, 3)
        r = rng.uniform(-3, 5)
        a = r * b
        for name, phi in phis.items():
            s = O.limit(a, b, name)
            assert s == pytest.approx(phi(r) * b, rel=1e-13, abs=1e-300), (name, r)
            ph = s / b
            assert -1e-15 <= ph <= min(2 * max(r, 0), 2) + 1e-12, (name, r)
    for name in phis:
        for d in (1e-3, -2.5, 7.0):
            assert O.limit(d, d, name) == pytest.approx(d, rel=1e-15)


def test_limiters_symmetric_and_odd():
    rng = np.random.default_rng(62)
    for _ in range(1000):
        a, b = rng.normal(size=2) * 10 ** rng.uniform(-3, 3, 2)
        for name in ("minmod", "mc", "vanleer"):
            s = O.limit(a, b, name)
            assert s == O.limit(b, a, name)
            assert -s == O.limit(-a, -b, name)
            assert (s == 0.0) == (a * b <= 0.0)


# ---------------------------------------------------------------- upwind CT

def _hll_1d(fl, fr, ul, ur, ap, am):
    """HLL flux with right- / left-going bounds ap, am >= 0 (written out)."""
    return (ap * fl + am * fr - ap * am * (ur - ul)) / (ap + am)


def test_uct_hll_reduces_to_hll_along_each_axis():
    """Corner states that do not change along b: the upwind-CT EMF is minus
    the HLL flux along a of the b-field (flux of B_b along a: v_a B_b - v_b
    B_a = -E_c), whatever the b speed bounds; likewise along b for states
    that do not change along a (flux of B_a along b: E_c)."""
    rng = np.random.default_rng(71)
    for _ in range(500):
        va_lo, va_hi, vb_lo, vb_hi = rng.normal(size=4)
        bb_lo, bb_hi, ba = rng.normal(size=3)
        ap, am, bp, bm = rng.uniform(0.05, 3.0, 4)
        e = O.uct_hll([va_lo, va_hi, va_lo, va_hi], [vb_lo, vb_hi, vb_lo, vb_hi], [ba, ba],
                      [bb_lo, bb_hi], [ap, am, bp, bm])
        fl = va_lo * bb_lo - vb_lo * ba
        fr = va_hi * bb_hi - vb_hi * ba
        assert e == pytest.approx(-_hll_1d(fl, fr, bb_lo, bb_hi, ap, am), rel=1e-12, abs=1e-13)
        # along b: states vary with sb only
        ba_lo, ba_hi, bbv = rng.normal(size=3)
        e = O.uct_hll([va_lo, va_lo, va_hi, va_hi], [vb_lo, vb_lo, vb_hi, vb_hi], [ba_lo, ba_hi],
                      [bbv, bbv], [ap, am, bp, bm])
        gl = vb_lo * ba_lo - va_lo * bbv
        gr = vb_hi * ba_hi - va_hi * bbv
        assert e == pytest.approx(_hll_1d(gl, gr, ba_lo, ba_hi, bp, bm), rel=1e-12, abs=1e-13)


def test_uct_hll_upwind_uniform_and_mirror():
    rng = np.random.default_rng(72)
    for _ in range(500):
        va, vb = rng.normal(size=4), rng.normal(size=4)
        ba, bb = rng.normal(size=2), rng.normal(size=2)
        al = rng.uniform(0.05, 3.0, 4)
        # supersonic towards +a and +b: the lower-lower state alone
        e = O.uct_hll(va, vb, ba, bb, [al[0], 0.0, al[2], 0.0])
        assert e == pytest.approx(vb[0] * ba[0] - va[0] * bb[0], rel=1e-13, abs=1e-14)
        # towards -a and -b: the upper-upper state alone
        e = O.uct_hll(va, vb, ba, bb, [0.0, al[1], 0.0, al[3]])
        assert e == pytest.approx(vb[3] * ba[1] - va[3] * bb[1], rel=1e-13, abs=1e-14)
        # one state everywhere: the cell EMF
        e = O.uct_hll([va[0]] * 4, [vb[0]] * 4, [ba[0]] * 2, [bb[0]] * 2, al)
        assert e == pytest.approx(vb[0] * ba[0] - va[0] * bb[0], rel=1e-13, abs=1e-14)
        # mirror a -> -a: lower and upper sides along a trade places, v_a and
        # B_b change sign, the two a bounds swap; E_c is unchanged
        e = O.uct_hll(va, vb, ba, bb, al)
        m = [1, 0, 3, 2]
        em = O.uct_hll(-va[m], vb[m], ba, -bb[::-1], [al[1], al[0], al[2], al[3]])
        assert em == pytest.approx(e, rel=1e-12, abs=1e-13)
        # mirror b -> -b
        m = [2, 3, 0, 1]
        em = O.uct_hll(va[m], -vb[m], -ba[::-1], bb, [al[0], al[1], al[3], al[2]])
        assert em == pytest.approx(e, rel=1e-12, abs=1e-13)
