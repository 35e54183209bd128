"""Pins of the oracle's local-capacitance force (Sec. 3, Eq. lca), CPU only.

Reading: phi = -e n / C_g gives each carrier the force -(e^2 / C_g) grad n
(e = 1), added to the drive; grad n is the central difference of the
density of the previous state (of f(0) for the first collision); a
neighbour off the lattice or solid takes the site's own density.

* Bookkeeping written out independently with numpy: per step, the total
  momentum T^0k grows by sum_x F^k(x) n(x) U^0(x) and N^0 is unchanged,
  with F from the previous density -- this fixes the sign, the factor 1/C_g,
  the half of the central difference and the one-step lag.
* Sound speed: the force adds n0 / C_g to the pressure gradient of the
  linearised momentum equation, so c_s^2 = c^2/2 + c n0 / (3 T0 C_g) in
  sites^2/step^2 with c = 5 sites/step (eps = 2 n T, enthalpy 3 n T).
* Closed box: N^0 and T^00 are conserved with the force on.
* C_g = infinity is the plain step.
"""
import numpy as np
import pytest

import oracle


def _st():
    return oracle.stencil()


def _smooth(nx, ny, amp=2e-2, seed=5):
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:ny, 0:nx]
    ph = rng.uniform(0, 2 * np.pi, 4)
    n = 1 + amp * np.sin(2 * np.pi * x / nx + ph[0]) * np.cos(2 * np.pi * 2 * y / ny + ph[1])
    T = 1 + amp * np.cos(2 * np.pi * x / nx + ph[2])
    vx = amp * np.sin(2 * np.pi * y / ny + ph[3])
    vy = amp * np.cos(2 * np.pi * x / nx)
    return n, T, vx, vy


def _grad_periodic(n):
    gx = 0.5 * (np.roll(n, -1, axis=1) - np.roll(n, 1, axis=1))
    gy = 0.5 * (np.roll(n, -1, axis=0) - np.roll(n, 1, axis=0))
    return gx, gy


@pytest.mark.parametrize("cg", [0.5, 10.0])
def test_momentum_bookkeeping_uses_previous_density(cg):
    drive = (1e-3, -2e-3)
    L = oracle.Lattice(_st(), 20, 16, periodic_x=True, periodic_y=True, tau=0.9, F=drive, cg=cg)
    L.init_fields(*_smooth(20, 16))
    n_prev = L.fields()["n"]  # the first collision takes the density of f(0)
    for _ in range(3):
        fl = L.fields()
        g = 1.0 / np.sqrt(1 - fl["vx"] ** 2 - fl["vy"] ** 2)
        gx, gy = _grad_periodic(n_prev)
        Fx = drive[0] - gx / cg
        Fy = drive[1] - gy / cg
        t0 = L.totals()
        L.run(1)
        t1 = L.totals()
        scale = t0["T00"] * 1e-14
        assert abs(t1["N0"] - t0["N0"]) < scale
        assert abs((t1["T0x"] - t0["T0x"]) - (Fx * fl["n"] * g).sum()) < scale
        assert abs((t1["T0y"] - t0["T0y"]) - (Fy * fl["n"] * g).sum()) < scale
        assert abs((t1["T00"] - t0["T00"]) - ((Fx * fl["vx"] + Fy * fl["vy"]) * fl["n"] * g).sum()) < scale
        n_prev = fl["n"]


def test_bookkeeping_distinguishes_lag():
    """The same bookkeeping with the current density instead of the previous
    one fails: the lag is visible at this amplitude."""
    cg = 0.5
    L = oracle.Lattice(_st(), 20, 16, periodic_x=True, periodic_y=True, tau=0.9, cg=cg)
    L.init_fields(*_smooth(20, 16, amp=5e-2))
    L.run(1)
    fl = L.fields()
    g = 1.0 / np.sqrt(1 - fl["vx"] ** 2 - fl["vy"] ** 2)
    t0 = L.totals()
    L.run(1)
    t1 = L.totals()
    gx, _ = _grad_periodic(fl["n"])
    wrong = (-gx / cg * fl["n"] * g).sum()
    assert abs((t1["T0x"] - t0["T0x"]) - wrong) > 1e3 * t0["T00"] * 1e-14


@pytest.mark.parametrize("cg", [1.0, 0.5])
def test_sound_speed_with_capacitance(cg):
    Lx, n0, T0 = 128, 1.0, 1.0
    L = oracle.Lattice(_st(), Lx, 2, periodic_x=True, periodic_y=True, tau=0.6, cg=cg)
    x = np.ones((2, 1)) * np.arange(Lx)[None, :]
    L.init_fields(n0 + 1e-5 * np.cos(2 * np.pi * x / Lx), T0, 0.0, 0.0)
    ph = 2 * np.pi * np.arange(Lx) / Lx
    amps = []
    for _ in range(120):
        eps = L.fields()["eps"].mean(axis=0)
        amps.append(2.0 / Lx * (eps * np.cos(ph)).sum())
        L.run(1)
    amps = np.array(amps)
    zc = [t + amps[t] / (amps[t] - amps[t + 1]) for t in range(len(amps) - 1) if amps[t] * amps[t + 1] < 0]
    cs = Lx / (2 * np.mean(np.diff(zc)))
    c = 5.0
    expected = np.sqrt(c * c / 2 + c * n0 / (3 * T0 * cg))
    assert abs(cs / expected - 1) < 0.005, (cs, expected)
    # the plain gas would be 12.5% / 6.5% slower: the test tells them apart
    assert abs(cs / (c / np.sqrt(2)) - 1) > 0.05


def test_closed_box_conserves_number_and_energy():
    L = oracle.Lattice(_st(), 18, 14, tau=0.8, cg=2.0)
    L.init_fields(*_smooth(18, 14, amp=3e-2))
    t0 = L.totals()
    L.run(30)
    t1 = L.totals()
    assert abs(t1["N0"] / t0["N0"] - 1) < 1e-13
    # the force does work sum F.N; in a closed box at rest on average it is small
    # but not zero: check number only strictly, energy to the size of that work
    assert abs(t1["T00"] / t0["T00"] - 1) < 1e-5


def test_infinite_capacitance_is_plain_step():
    w = dict(tau=0.9, F=(1e-3, 0.0))
    A = oracle.Lattice(_st(), 12, 10, periodic_x=True, **w)
    B = oracle.Lattice(_st(), 12, 10, periodic_x=True, cg=np.inf, **w)
    for L in (A, B):
        L.init_fields(*_smooth(12, 10))
        L.run(5)
    assert np.array_equal(A.f, B.f)
