"""Pins of the oracle's collision and forcing term (CPU only).

* Collision invariants: N^0, T^00, T^0x, T^0y are unchanged by the
  relaxation of Eq. ``discrete-rbe`` (the Anderson-Witting collision conserves
  the time components; Nx, Ny and the spatial stresses relax).
* Forcing term (Sec. 2.4): its number, energy and momentum sources equal the
  continuum values 0, F . (n U_s) and F^k n U^0.
* The projections b^(k) the oracle builds from C_j a are checked against a
  direct evaluation of the definition: the momentum derivative of the order-3
  equilibrium expansion (complex-step, exact to round-off) projected onto
  Appendix A by exact quadrature (Gauss-Laguerre x trapezoid on the shell).
"""
import numpy as np
import pytest

import oracle
from oracle import appendix

STATES = [(1.0, 1.0, 0.0, 0.0), (1.3, 0.9, 0.1, -0.05), (0.8, 1.2, -0.3, 0.2), (1.5, 1.25, 1e-5, 0.0)]


def _P(st):
    return np.stack([st.p0, st.px, st.py])


def _time_components(st, f):
    P = _P(st)
    N = P @ f
    T = np.einsum("ai,bi,i->ab", P, P, f)
    return N, T


@pytest.mark.parametrize("state", STATES)
@pytest.mark.parametrize("tau", [0.55, 0.8, 1.0, 2.0])
def test_collision_conserves_time_components(state, tau):
    n, T, vx, vy = state
    st = oracle.stencil()
    rng = np.random.default_rng(7)
    f = st.feq(n, T, oracle.four_velocity(vx, vy)) * (1 + 0.1 * rng.uniform(-1, 1, 48))
    g = st.collide(f, tau)
    N1, T1 = _time_components(st, f)
    N2, T2 = _time_components(st, g)
    assert abs(N2[0] - N1[0]) <= 1e-14 * N1[0]
    np.testing.assert_allclose(T2[0], T1[0], rtol=0, atol=1e-14 * T1[0, 0])
    # Nx is not a collision invariant: it relaxes towards n U^x
    assert abs(N2[1] - N1[1]) > 1e-6 * N1[0]


@pytest.mark.parametrize("state", STATES)
def test_equilibrium_is_collision_fixed_point(state):
    n, T, vx, vy = state
    st = oracle.stencil()
    f = st.feq(n, T, oracle.four_velocity(vx, vy))
    np.testing.assert_allclose(st.collide(f, 0.8), f, rtol=0, atol=1e-15 * f.max() * 4)


@pytest.mark.parametrize("state", STATES)
@pytest.mark.parametrize("F", [(1e-5, 0.0), (0.02, -0.01), (0.0, 3e-3)])
def test_force_sources_are_exact(state, F):
    n, T, vx, vy = state
    st = oracle.stencil()
    U = oracle.four_velocity(vx, vy)
    Fi = st.force_term(n, T, U, *F)
    N, Tm = _time_components(st, Fi)
    scale = abs(F[0]) + abs(F[1])
    assert abs(N[0]) < 1e-15 * n * scale * 10
    assert abs(Tm[0, 0] - (F[0] * n * U[1] + F[1] * n * U[2])) < 2e-15 * n * U[0] * scale * 10
    assert abs(Tm[0, 1] - F[0] * n * U[0]) < 2e-15 * n * U[0] * scale * 10
    assert abs(Tm[0, 2] - F[1] * n * U[0]) < 2e-15 * n * U[0] * scale * 10


def _direct_b(a, axis, nang=64, nrad=12):
    """b^(k)_j = integral (d/dp^j f^eq_N) J_k dp/p0 with f^eq_N = omega sum a_m J_m."""
    x, wl = np.polynomial.laguerre.laggauss(nrad)
    th = 2 * np.pi * np.arange(nang) / nang
    p = x[None, :] * np.ones((nang, 1))
    px, py = p * np.cos(th)[:, None], p * np.sin(th)[:, None]
    h = 1e-20

    def feqN(qx, qy):
        q0 = np.sqrt(qx * qx + qy * qy)
        return np.exp(-q0) / (2 * np.pi) * (appendix.evaluate_complex(q0, qx, qy) @ a)

    if axis == "x":
        d = feqN(px + 1j * h, py + 0j).imag / h
    else:
        d = feqN(px + 0j, py + 1j * h).imag / h
    Jv = appendix.evaluate(p, px, py)
    # dp/p0 = dp0 dtheta on the shell; exp(-p) carried inside d, so undo the
    # Laguerre weight factor exp(-x).
    integrand = d[:, :, None] * Jv * (wl * np.exp(x))[None, :, None]
    return integrand.sum(axis=(0, 1)) * (2 * np.pi / nang)


@pytest.mark.parametrize("state", STATES)
def test_force_projection_matches_direct_derivative(state):
    n, T, vx, vy = state
    a = oracle.projections(n, T, oracle.four_velocity(vx, vy))
    Cx, Cy = appendix.force_matrices()
    for axis, C in (("x", Cx), ("y", Cy)):
        ref = _direct_b(a, axis)
        assert np.abs(C @ a - ref).max() < 1e-12 * max(1.0, np.abs(ref).max()), (axis, C @ a, ref)


@pytest.mark.parametrize("state", STATES)
def test_force_term_uses_the_projection(state):
    n, T, vx, vy = state
    st = oracle.stencil()
    U = oracle.four_velocity(vx, vy)
    a = oracle.projections(n, T, U)
    F = (0.01, -0.02)
    b = F[0] * _direct_b(a, "x") + F[1] * _direct_b(a, "y")
    ref = -st.w * (st.J @ b)
    np.testing.assert_allclose(st.force_term(n, T, U, *F), ref, rtol=0, atol=1e-15 * np.abs(ref).max() * 50)


def test_relaxation_factor_is_shell_independent():
    """p_i^mu U_mu / (p^0_i tau) = gamma (1 - nhat_i . v) / tau, the same on all four shells.

    The perturbation w_i J^(3)_000(p_i) is orthogonal to every moment of order
    <= 2, so it leaves N, T^ab, the Landau frame and f^eq unchanged and is
    relaxed by exactly the factor omega_i.
    """
    st = oracle.stencil()
    U = oracle.four_velocity(0.3, -0.2)
    f = st.feq(1.0, 1.0, U)
    delta = 1e-3 * st.w * st.J[:, 9]
    tau = 0.9
    g = st.collide(f + delta, tau)
    omega = (f + delta - g) / delta
    om = omega.reshape(12, 4)
    np.testing.assert_allclose(om, om[:, :1] * np.ones((1, 4)), rtol=1e-10)
    nh = np.array(oracle.quadrature.DIRECTIONS, dtype=float) / 5.0
    np.testing.assert_allclose(om[:, 0], (U[0] - nh @ U[1:]) / tau, rtol=1e-10)
