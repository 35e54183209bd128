"""Host-side checks of the injector analysis (no device): on analytic
fields the ring analysis returns the amplitude it was given, the flux
integral returns the injected flux, and the potential combines pressure and
the local-capacitance term as documented."""
import numpy as np

from paper_1804_02418_amd import validation as V


def _grid(nx=400, ny=200, centre=(199.5, -0.5)):
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    dx, dy = x - centre[0], y - centre[1]
    r = np.hypot(dx, dy)
    th = np.arctan2(dx, dy)  # from +y
    return r, th, dx


def test_collapse_recovers_amplitude_despite_background():
    centre = (199.5, -0.5)
    r, th, dx = _grid(centre=centre)
    A = 3.7e-4
    y = r * np.cos(th) - 0.5
    phi = A * np.cos(2 * th) / r ** 2 + 2.5e-6 + 1e-8 * dx - 3e-9 * y  # smooth backgrounds
    rings = V.collapse(phi, centre, [30, 50, 80])
    for g in rings:
        assert abs(g["A"] / A - 1) < 2e-3, g
        assert g["misfit"] < 5e-3, g


def test_collapse_sees_a_wrong_law():
    centre = (199.5, -0.5)
    r, th, _ = _grid(centre=centre)
    phi = 1e-3 * np.cos(2 * th) / r  # 1/r instead of 1/r^2: r^2 Phi does not collapse
    amps = [g["A"] for g in V.collapse(phi, centre, [30, 60, 90])]
    assert amps[-1] / amps[0] > 2.5


def test_injected_flux_of_a_stokes_source():
    centre = (199.5, -0.5)
    r, th, _ = _grid(centre=centre)
    Q = 2e-4
    vr = 2 * Q / np.pi * np.cos(th) ** 2 / np.maximum(r, 1e-9)
    fields = {"vx": vr * np.sin(th), "vy": vr * np.cos(th), "n": np.full(r.shape, 1.5)}
    q = V.injected_flux(fields, centre, 40.0, 1.5)
    assert abs(q / Q - 1) < 2e-3


def test_potential_terms():
    f = {"eps": np.array([2 * 1.5 * 1.25 + 1e-6]), "n": np.array([1.5 + 2e-7])}
    phi_inf = V.potential(f, 1.5, 1.25, np.inf)
    assert np.allclose(phi_inf, 5.0 * 0.5e-6 / 1.5, rtol=1e-9)
    phi10 = V.potential(f, 1.5, 1.25, 10.0)
    assert np.allclose(phi10 - phi_inf, 2e-8, rtol=1e-6)
