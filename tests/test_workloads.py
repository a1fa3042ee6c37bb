"""The synthetic inputs: discretely divergence-free face fields, periodic
faces that repeat, positive density and pressure, and the symmetry the 2D
Riemann problem is built with."""
import numpy as np
import pytest

from paper_2606_12753_amd import workloads as W


def divb(spec, bface):
    dx = spec.dx
    return ((bface[0][:, :, 1:] - bface[0][:, :, :-1]) / dx[0]
            + (bface[1][:, 1:, :] - bface[1][:, :-1, :]) / dx[1]
            + (bface[2][1:, :, :] - bface[2][:-1, :, :]) / dx[2])


@pytest.mark.parametrize("wl", [W.orszag_tang_3d(n=24), W.riemann_2d(n=40), W.orszag_tang_2d(n=32),
                                W.blast_3d(n=16), W.random_smooth(n=(9, 7, 5), seed=3),
                                W.kelvin_helmholtz(nx=24, ny=12, nz=12)],
                         ids=lambda w: w.name)
def test_inputs_are_physical_and_divergence_free(wl):
    for spec, st in zip(wl.boxes, wl.states):
        bmax = max(float(np.max(np.abs(b))) for b in st.bface)
        assert float(np.max(np.abs(divb(spec, st.bface)))) * min(spec.dx) <= 1e-14 * max(bmax, 1)
        for d in range(3):
            if spec.bc[d] == W.PERIODIC:
                sl0 = [slice(None)] * 3
                sl1 = [slice(None)] * 3
                sl0[2 - d], sl1[2 - d] = 0, -1
                assert np.array_equal(st.bface[d][tuple(sl0)], st.bface[d][tuple(sl1)])
        rho, mx, my, mz, en = st.cons
        assert np.all(rho > 0) and np.all(np.isfinite(en))


def test_riemann_2d_quadrants_and_mirror():
    wl = W.riemann_2d(n=40)
    spec, st = wl.boxes[0], wl.states[0]
    assert wl.meta == {"rk": 3, "solver": "hll"}
    rho, mx, my, mz, en = (c[0] for c in st.cons)
    assert np.array_equal(rho, rho.T) and np.array_equal(mx, my.T) and np.array_equal(en, en.T)
    assert set(np.unique(rho)) == {0.5, 1.0}
    assert np.all(mz == 0.0)


def test_orszag_tang_3d_varies_along_every_axis():
    """The 3D stand-in shifts the vortex's phase along z, so the state
    varies along every axis (m_x along y and z, m_y along x and z)."""
    wl = W.orszag_tang_3d(n=16)
    rho, mx, my, mz, en = wl.states[0].cons
    assert wl.meta == {"rk": 3}
    for arr, axes in ((mx, (0, 1)), (my, (0, 2))):     # array axes (z, y, x)
        for ax in range(3):
            varies = np.max(np.abs(np.diff(arr, axis=ax))) > 0
            assert varies == (ax in axes), ax
    assert np.all(mz == 0.0)
