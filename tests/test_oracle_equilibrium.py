"""Pins of the oracle's equilibrium, moments and Landau solve (CPU only).

* Appendix B against a direct numerical projection of the exact
  Maxwell-Juttner distribution (Eq. ``maxwell-juttner``) onto Appendix A.
* Appendix C's printed closed form against the oracle's sum over k.
* Quadrature moments of f^eq up to third order against the closed-form
  Maxwell-Juttner tensors of a massless 2-D gas (Eqs. ``mj-first-moment``,
  ``mj-second-moment`` and the third moment).
* The Landau frame against LAPACK's eigenvectors.
"""
import numpy as np
import pytest

import oracle
from oracle import appendix

ETA = np.diag([1.0, -1.0, -1.0])


def _states():
    return [(1.0, 1.0, 0.0, 0.0), (1.5, 1.25, 1e-5, 0.0), (0.7, 0.8, 0.2, -0.1),
            (2.0, 1.3, -0.3, 0.25), (1.1, 0.95, 0.0, 0.4)]


def _mj_projection(n, T, vx, vy, nang=2048, nrad=24):
    """a_k = integral f_MJ J_k dp/p0, f_MJ = n/(2 pi T^2) exp(-p.U/T), m = 0.

    On the shell dp/p0 = dp0 dtheta.  For each angle the radial integral of
    exp(-A p) times a cubic in p is done exactly by Gauss-Laguerre; the
    periodic angular integral by the trapezoidal rule (spectrally accurate).
    """
    U = oracle.four_velocity(vx, vy)
    x, wl = np.polynomial.laguerre.laggauss(nrad)
    th = 2 * np.pi * np.arange(nang) / nang
    c, s = np.cos(th), np.sin(th)
    A = (U[0] - U[1] * c - U[2] * s) / T  # exp(-p A)
    p = x[None, :] / A[:, None]
    p0, px, py = p, p * c[:, None], p * s[:, None]
    Jv = appendix.evaluate(p0, px, py)  # (nang, nrad, 16)
    pref = n / (2 * np.pi * T * T)
    integrand = Jv * (wl[None, :, None] / A[:, None, None])
    return pref * integrand.sum(axis=1).sum(axis=0) * (2 * np.pi / nang)


@pytest.mark.parametrize("state", _states())
def test_appendix_b_is_the_maxwell_juttner_projection(state):
    n, T, vx, vy = state
    a_exact = _mj_projection(n, T, vx, vy)
    a_oracle = oracle.projections(n, T, oracle.four_velocity(vx, vy))
    assert np.abs(a_exact - a_oracle).max() < 1e-12 * max(1.0, np.abs(a_exact).max()), (a_exact, a_oracle)


def _appendix_c(w, p0, px, py, n, T, U):
    """Closed form of Appendix C, transcribed as printed (u = 4-velocity)."""
    u0, ux, uy = U
    t = (1 / 6 * T**3 * ux * (px**3 - 3 * p0**2 * px / 4) * (-3 * u0**2 + 4 * ux**2 + 3)
         + 1 / 24 * py * T**3 * uy * (p0**2 - 4 * px**2) * (u0**2 - 4 * ux**2 - 1)
         + 1 / 4 * T**2 * (p0**2 - 2 * px**2) * (u0**2 - 2 * ux**2 - 1)
         + 1 / 8 * (-2 * p0**2 + (p0 - 5) * px**2 + 9 * p0 - 3) * (T * u0 - 1)
         * (T * (5 * T * ux**2 + T - 2 * u0) + 1)
         + 1 / 24 * (4 * p0**3 - 30 * p0**2 - 3 * (p0 - 5) * px**2 + 45 * p0 - 15) * (T * u0 - 1)
         * (T**2 * (4 * u0**2 - 3 * (ux**2 + 1)) - 2 * T * u0 + 1)
         + (p0 - 5) * px * py * T**2 * ux * uy * (T * u0 - 1)
         + 1 / 8 * (p0 - 6) * (p0 - 2) * px * T * ux * (T**2 * (5 * u0**2 - 1) - 8 * T * u0 + 4)
         + (p0 - 3) * px * T * ux * (T * u0 - 1)
         + 1 / 8 * (p0 - 6) * (p0 - 2) * py * T * uy * (T**2 * (5 * u0**2 - 1) - 8 * T * u0 + 4)
         + (p0 - 3) * py * T * uy * (T * u0 - 1)
         + 1 / 4 * ((p0 - 4) * p0 + 2) * (T**2 * (3 * u0**2 - 1) - 4 * T * u0 + 2)
         + (p0 - 1) * (T * u0 - 1) + px * py * T**2 * ux * uy + px * T * ux + py * T * uy + 1)
    return w * n / T * t


@pytest.mark.parametrize("state", _states())
def test_appendix_c_closed_form_matches(state):
    n, T, vx, vy = state
    st = oracle.stencil()
    U = oracle.four_velocity(vx, vy)
    ref = _appendix_c(st.w, st.p0, st.px, st.py, n, T, U)
    got = st.feq(n, T, U)
    assert np.abs(ref - got).max() < 5e-14 * np.abs(ref).max()


@pytest.mark.parametrize("state", _states())
def test_feq_moments_up_to_third_order(state):
    n, T, vx, vy = state
    st = oracle.stencil()
    U = oracle.four_velocity(vx, vy)
    f = st.feq(n, T, U)
    P = np.stack([st.p0, st.px, st.py])  # (3, 48)
    assert abs(f.sum() - n / T) < 1e-14 * n / T
    np.testing.assert_allclose(P @ f, n * U, rtol=0, atol=1e-14 * n * U[0])
    T2 = np.einsum("ai,bi,i->ab", P, P, f)
    np.testing.assert_allclose(T2, n * T * (3 * np.outer(U, U) - ETA), rtol=0, atol=2e-14 * n * T * U[0] ** 2 * 3)
    T3 = np.einsum("ai,bi,ci,i->abc", P, P, P, f)
    ref3 = 15 * np.einsum("a,b,c->abc", U, U, U)
    ref3 -= 3 * (np.einsum("ab,c->abc", ETA, U) + np.einsum("ac,b->abc", ETA, U) + np.einsum("bc,a->abc", ETA, U))
    ref3 *= n * T * T
    np.testing.assert_allclose(T3, ref3, rtol=0, atol=1e-13 * np.abs(ref3).max())


@pytest.mark.parametrize("state", _states())
def test_recovery_round_trip(state):
    n, T, vx, vy = state
    st = oracle.stencil()
    U = oracle.four_velocity(vx, vy)
    n2, T2, eps2, U2 = st.macro(st.feq(n, T, U))
    assert abs(n2 - n) < 1e-14 * n and abs(T2 - T) < 1e-14 * T
    assert abs(eps2 - 2 * n * T) < 1e-14 * n * T
    np.testing.assert_allclose(U2, U, rtol=0, atol=2e-15 * U[0])


def test_landau_frame_matches_lapack():
    st = oracle.stencil()
    rng = np.random.default_rng(1804_02418)
    P = np.stack([st.p0, st.px, st.py])
    worst_e = worst_u = 0.0
    checked = 0
    for _ in range(4000):
        v = rng.uniform(0, 0.9)
        phi = rng.uniform(0, 2 * np.pi)
        n, T = rng.uniform(0.5, 2.0), rng.uniform(0.5, 1.5)
        U = oracle.four_velocity(v * np.cos(phi), v * np.sin(phi))
        f = st.feq(n, T, U) * (1 + rng.uniform(-0.2, 0.2, 48))
        if f.min() < 0:  # the order-3 expansion can go negative at large |v|
            continue
        checked += 1
        Tm = np.einsum("ai,bi,i->ab", P, P, f)
        eps, Uo = oracle.landau(Tm)
        M = Tm @ ETA
        lam, vec = np.linalg.eig(M)
        timelike = [k for k in range(3) if abs(lam[k].imag) < 1e-12
                    and vec[0, k].real ** 2 - vec[1, k].real ** 2 - vec[2, k].real ** 2 > 0]
        assert len(timelike) == 1
        k = timelike[0]
        ul = vec[:, k].real
        ul = ul * np.sign(ul[0]) / np.sqrt(ul[0] ** 2 - ul[1] ** 2 - ul[2] ** 2)
        assert lam[k].real == pytest.approx(max(lam.real))
        worst_e = max(worst_e, abs(eps - lam[k].real) / abs(lam[k].real))
        worst_u = max(worst_u, np.abs(Uo - ul).max() / ul[0])
    assert checked > 1000, checked
    assert worst_e < 1e-13 and worst_u < 1e-13, (worst_e, worst_u)


def test_landau_rejects_tensor_without_timelike_frame():
    # energy flux larger than the energy density: no timelike eigenvector
    Tm = np.array([[1.0, 1.2, 0.0], [1.2, 1.0, 0.0], [0.0, 0.0, 0.5]])
    with pytest.raises(ArithmeticError):
        oracle.landau(Tm)
