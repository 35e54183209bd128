"""Lattice-level pins of the oracle (CPU only).

* A uniform moving equilibrium is a fixed point of the whole step.
* Periodic lattice: global N^0, T^00, T^0x, T^0y are constant without a
  force, and grow by exactly F . sum(n U_s) and F^k sum(n U^0) per step with
  one.
* Closed box (bounce-back walls): global N^0 and T^00 are constant.
* Contacts: the change of global N^0 equals the flux through the contact
  ghost spans (bookkeeping written out independently below).
* Shear viscosity nu = 6.25 (tau - 1/2) sites^2/step (eta = 3/4 n T
  (tau - 1/2); the paper's remark eta = 3/8 at n = T = tau = 1).
* Sound speed c/sqrt(2) = 5/sqrt(2) sites/step (massless 2-D gas, eps = 2P).
* Channel flow with walls and a body force: curvature v'' = -F/(3 T nu).
"""
import numpy as np
import pytest

import oracle
from conftest import read_golden


def _st():
    return oracle.stencil()


def test_uniform_moving_equilibrium_is_fixed_point():
    L = oracle.Lattice(_st(), 16, 12, periodic_x=True, periodic_y=True, tau=0.8)
    L.init_fields(1.2, 0.9, 0.15, -0.1)
    f0 = L.f.copy()
    L.run(50)
    assert np.abs(L.f - f0).max() <= 5e-15 * np.abs(f0).max()


def _smooth_fields(nx, ny, amp=1e-2, seed=3):
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:ny, 0:nx]
    ph = rng.uniform(0, 2 * np.pi, 4)
    n = 1 + amp * np.sin(2 * np.pi * x / nx + ph[0]) * np.cos(2 * np.pi * y / ny + ph[1])
    T = 1 + amp * np.cos(2 * np.pi * x / nx + ph[2])
    vx = amp * np.sin(2 * np.pi * y / ny + ph[3])
    vy = amp * np.cos(2 * np.pi * x / nx)
    return n, T, vx, vy


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def test_periodic_lattice_conserves_totals():
    L = oracle.Lattice(_st(), 24, 20, periodic_x=True, periodic_y=True, tau=0.9)
    L.init_fields(*_smooth_fields(24, 20))
    t0 = L.totals()
    L.run(20)
    t1 = L.totals()
    for k in ("N0", "T00"):
        assert _rel(t1[k], t0[k]) < 20 * 2e-16 * 10, k
    for k in ("T0x", "T0y"):
        assert abs(t1[k] - t0[k]) < 20 * 2e-16 * 10 * t0["T00"], k


@pytest.mark.parametrize("F", [(1e-3, 0.0), (2e-3, -1e-3)])
def test_periodic_lattice_force_increments(F):
    L = oracle.Lattice(_st(), 20, 16, periodic_x=True, periodic_y=True, tau=1.1, F=F)
    L.init_fields(*_smooth_fields(20, 16, amp=5e-2))
    for _ in range(3):
        fl = L.fields()
        g = 1.0 / np.sqrt(1 - fl["vx"] ** 2 - fl["vy"] ** 2)
        nU0 = (fl["n"] * g).sum()
        nUx = (fl["n"] * g * fl["vx"]).sum()
        nUy = (fl["n"] * g * fl["vy"]).sum()
        t0 = L.totals()
        L.run(1)
        t1 = L.totals()
        scale = t0["T00"] * 1e-15 * 10
        assert abs(t1["N0"] - t0["N0"]) < scale
        assert abs((t1["T00"] - t0["T00"]) - (F[0] * nUx + F[1] * nUy)) < scale
        assert abs((t1["T0x"] - t0["T0x"]) - F[0] * nU0) < scale
        assert abs((t1["T0y"] - t0["T0y"]) - F[1] * nU0) < scale


def test_closed_box_conserves_number_and_energy():
    L = oracle.Lattice(_st(), 23, 17, tau=0.7)
    L.init_fields(*_smooth_fields(23, 17, amp=3e-2))
    t0 = L.totals()
    L.run(30)
    t1 = L.totals()
    assert _rel(t1["N0"], t0["N0"]) < 1e-13
    assert _rel(t1["T00"], t0["T00"]) < 1e-13
    # bounce-back does not conserve momentum: it is the no-slip wall
    L2 = oracle.Lattice(_st(), 23, 17, tau=0.7)
    L2.init_fields(1.0, 1.0, 0.05, 0.0)
    p0 = L2.totals()["T0x"]
    L2.run(5)
    assert abs(L2.totals()["T0x"]) < 0.9 * abs(p0)


def test_contact_flux_bookkeeping():
    """Global N^0 after one step = N^0 of post-collision populations that stay
    on the lattice + N^0 of the equilibrium that enters from contact ghosts."""
    st = _st()
    nx, ny = 40, 24
    contacts = [dict(edge="bottom", start=6, width=8, n=1.05, T=1.0),
                dict(edge="top", start=20, width=10, n=0.97, T=1.02, vx=0.01)]
    L = oracle.Lattice(st, nx, ny, contacts=contacts, tau=0.8, F=(1e-3, 0.0))
    L.init_fields(*_smooth_fields(nx, ny, amp=2e-2))
    fstar = L.post_collision()
    # Bookkeeping written from the boundary rule: a population hops c_i; it
    # stays if it lands on the lattice, is absorbed if it lands in a contact
    # ghost span, and otherwise comes back reversed on its own site (same p0).
    def in_contact(x, y):
        for c in contacts:
            if c["edge"] == "bottom" and y < 0 and c["start"] <= x < c["start"] + c["width"]:
                return True
            if c["edge"] == "top" and y >= ny and c["start"] <= x < c["start"] + c["width"]:
                return True
        return False

    expected = 0.0
    y, x = np.mgrid[0:ny, 0:nx]
    for i in range(48):
        dx, dy = st.cx[i], st.cy[i]
        tx, ty = x + dx, y + dy
        inside = (tx >= 0) & (tx < nx) & (ty >= 0) & (ty < ny)
        absorbed = np.vectorize(in_contact)(tx, ty) & ~inside
        kept = ~absorbed
        expected += st.p0[i] * fstar[i][kept].sum()
        # entering from contact ghost spans: destination d, source d - c_i
        sx, sy = x - dx, y - dy
        for c in contacts:
            o = oracle.four_velocity(c.get("vx", 0.0), c.get("vy", 0.0))
            feq = st.feq(c["n"], c["T"], o)
            if c["edge"] == "bottom":
                m = (sy < 0) & (sx >= c["start"]) & (sx < c["start"] + c["width"])
            else:
                m = (sy >= ny) & (sx >= c["start"]) & (sx < c["start"] + c["width"])
            expected += st.p0[i] * feq[i] * m.sum()
    L.run(1)
    got = L.totals()["N0"]
    assert abs(got - expected) < 1e-13 * abs(expected)


def _wave_amplitude(field, k, axis_len, along):
    ph = 2 * np.pi * k * np.arange(axis_len) / axis_len
    prof = field.mean(axis=1 - along)
    return 2.0 / axis_len * (prof * np.sin(ph)).sum(), 2.0 / axis_len * (prof * np.cos(ph)).sum()


def test_paper_viscosity_remark_matches_relation():
    n, T, tau, eta = (float(v) for v in read_golden("viscosity_note.txt")[0])
    assert abs(0.75 * n * T * (tau - 0.5) - eta) < 1e-15


@pytest.mark.parametrize("tau", [0.8, 1.0, 1.5])
def test_shear_wave_viscosity(tau):
    Ly = 64
    L = oracle.Lattice(_st(), 4, Ly, periodic_x=True, periodic_y=True, tau=tau)
    y = np.arange(Ly)[:, None] * np.ones((1, 4))
    L.init_fields(1.0, 1.0, 1e-4 * np.sin(2 * np.pi * y / Ly), 0.0)
    L.run(50)
    a1, _ = _wave_amplitude(L.fields()["vx"], 1, Ly, 0)
    t1 = L.t
    steps = int(0.7 / (6.25 * (tau - 0.5) * (2 * np.pi / Ly) ** 2))
    L.run(steps)
    a2, _ = _wave_amplitude(L.fields()["vx"], 1, Ly, 0)
    nu = np.log(a1 / a2) / ((L.t - t1) * (2 * np.pi / Ly) ** 2)
    assert abs(nu / (6.25 * (tau - 0.5)) - 1) < 0.01, nu


def test_sound_speed():
    Lx = 128
    L = oracle.Lattice(_st(), Lx, 2, periodic_x=True, periodic_y=True, tau=0.6)
    x = np.ones((2, 1)) * np.arange(Lx)[None, :]
    L.init_fields(1 + 1e-5 * np.cos(2 * np.pi * x / Lx), 1.0, 0.0, 0.0)
    amps = []
    for _ in range(120):
        # the energy-momentum sector of a conformal gas closes on itself: eps
        # carries the pure sound mode (n also has a non-propagating part)
        _, c = _wave_amplitude(L.fields()["eps"], 1, Lx, 1)
        amps.append(c)
        L.run(1)
    amps = np.array(amps)
    zc = [t + amps[t] / (amps[t] - amps[t + 1]) for t in range(len(amps) - 1) if amps[t] * amps[t + 1] < 0]
    period = 2 * np.mean(np.diff(zc))
    cs = Lx / period
    assert abs(cs / (5 / np.sqrt(2)) - 1) < 0.005, cs


def test_channel_flow_curvature():
    """Steady channel flow between bounce-back walls driven by a body force:
    n F + eta v'' = 0, i.e. v'' = -F / (3 T nu) in lattice units."""
    tau, F, W = 1.0, 1e-6, 40
    L = oracle.Lattice(_st(), 5, W, periodic_x=True, tau=tau, F=(F, 0.0))
    L.init_fields(1.0, 1.0, 0.0, 0.0)
    nu = 6.25 * (tau - 0.5)
    L.run(int(6 * W * W / (np.pi ** 2 * nu)))
    vx = L.fields()["vx"][:, 0]
    yy = np.arange(W, dtype=float)
    core = slice(8, W - 8)
    c2 = np.polyfit(yy[core], vx[core], 2)[0]
    expected = -F / (3 * 1.0 * nu) / 2
    assert abs(c2 / expected - 1) < 0.02, (c2, expected)
