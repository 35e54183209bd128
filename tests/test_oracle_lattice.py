"""Lattice-level pins of the oracle (CPU only).

* A uniform moving equilibrium is a fixed point of the whole step.
* Periodic lattice: global N^0, T^00, T^0x, T^0y are constant without a
  force, and grow by exactly F . sum(n U_s) and F^k sum(n U^0) per step with
  one.
* Closed box (bounce-back walls): global N^0 and T^00 are constant.
* Contacts: the change of global N^0 equals the flux through the contact
  ghost spans (bookkeeping written out independently below), on every edge
  and with spans that reach the corners.
* Solid masks: a closed box with an interior obstacle keeps N^0 and T^00.
* A quarter turn of the whole problem gives the turned flow (ties the four
  edges' boundary handling together); corner sources bounce back.
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


# ---- solid masks, side contacts and corners (Sec. 3, Fig. `geom` caption;
# readings R11 and R12: bounce-back from solid or off-lattice sources,
# contacts as ghost spans, corner sources are walls) ----

def test_closed_box_with_solid_block_conserves_number_and_energy():
    """Bounce-back from solid sites is an on-site reversal (R11): every
    post-collision population lands exactly once, so a closed box with an
    interior obstacle keeps global N^0 and T^00 to round-off."""
    nx, ny = 29, 21
    solid = np.zeros((ny, nx), dtype=np.uint8)
    solid[7:13, 9:15] = 1          # a block thicker than one hop
    solid[3, 20:27] = 1            # a one-site-thick wall that hops jump over
    L = oracle.Lattice(_st(), nx, ny, solid=solid, tau=0.7)
    n, T, vx, vy = _smooth_fields(nx, ny, amp=3e-2)
    L.init_fields(n, T, vx + 0.02, vy)
    fluid = solid == 0

    def tot():
        f = L.f[:, fluid]
        return float(_st().p0 @ f.sum(axis=1)), float((_st().p0 ** 2) @ f.sum(axis=1))

    n0, e0 = tot()
    f_solid = L.f[:, solid == 1].copy()
    L.run(25)
    n1, e1 = tot()
    assert _rel(n1, n0) < 1e-13 and _rel(e1, e0) < 1e-13, (n1 - n0, e1 - e0)
    # solid sites are not updated
    assert np.array_equal(L.f[:, solid == 1], f_solid)


def _contact_hit(c, tx, ty, nx, ny):
    """Is off-lattice point (tx, ty) in the ghost span of contact c?  The span
    runs along its edge only: a point off the lattice in both axes (a
    corner) is in no span."""
    s, e = c["start"], c["start"] + c["width"]
    if c["edge"] == "bottom":
        return (ty < 0) & (tx >= s) & (tx < e)
    if c["edge"] == "top":
        return (ty >= ny) & (tx >= s) & (tx < e)
    if c["edge"] == "left":
        return (tx < 0) & (ty >= s) & (ty < e)
    return (tx >= nx) & (ty >= s) & (ty < e)


@pytest.mark.parametrize("layout", ["sides", "corners"])
def test_contact_flux_bookkeeping_every_edge(layout):
    """Global N^0 after one step = N^0 of the post-collision populations that
    do not land in a contact span + N^0 of the contact equilibria pulled in,
    with contacts on the left and right edges (and spans that reach the
    corners)."""
    st = _st()
    nx, ny = 36, 30
    if layout == "sides":
        contacts = [dict(edge="left", start=6, width=9, n=1.04, T=1.0, vy=0.01),
                    dict(edge="right", start=14, width=11, n=0.98, T=1.03, vx=-0.01)]
    else:
        contacts = [dict(edge="left", start=0, width=8, n=1.03, T=1.0),
                    dict(edge="bottom", start=0, width=10, n=0.97, T=1.02, vx=0.01),
                    dict(edge="right", start=ny - 7, width=7, n=1.01, T=0.99),
                    dict(edge="top", start=nx - 9, width=9, n=1.02, T=1.0, vy=-0.01)]
    L = oracle.Lattice(st, nx, ny, contacts=contacts, tau=0.8, F=(1e-3, -5e-4))
    L.init_fields(*_smooth_fields(nx, ny, amp=2e-2))
    fstar = L.post_collision()
    y, x = np.mgrid[0:ny, 0:nx]
    expected = 0.0
    for i in range(48):
        dx, dy = st.cx[i], st.cy[i]
        tx, ty = x + dx, y + dy
        absorbed = np.zeros_like(x, dtype=bool)
        for c in contacts:
            absorbed |= _contact_hit(c, tx, ty, nx, ny)
        expected += st.p0[i] * fstar[i][~absorbed].sum()
        sx, sy = x - dx, y - dy
        for c in contacts:
            feq = st.feq(c["n"], c["T"], oracle.four_velocity(c.get("vx", 0.0), c.get("vy", 0.0)))
            expected += st.p0[i] * feq[i] * _contact_hit(c, sx, sy, nx, ny).sum()
    L.run(1)
    got = L.totals()["N0"]
    assert abs(got - expected) < 1e-13 * abs(expected)


def _rotate_cw(a):
    """Scalar field on an nx x ny lattice -> the ny x nx lattice rotated by 90
    degrees clockwise: the site (x, y) goes to (x', y') = (y, nx - 1 - x)."""
    ny, nx = a.shape
    out = np.empty((nx, ny), dtype=a.dtype)
    y, x = np.mgrid[0:ny, 0:nx]
    out[nx - 1 - x, y] = a
    return out


def test_rotated_lattice_runs_the_rotated_flow():
    """The stencil maps to itself under a quarter turn ((cx, cy) -> (cy, -cx)
    keeps each weight family), so a run rotated by 90 degrees clockwise --
    bottom contacts onto the left edge, left onto top, top onto right,
    velocities and drive rotated as vectors -- gives the rotated fields.
    Ties the left/right/top boundary handling to the bottom one."""
    st = _st()
    nx, ny = 34, 26
    contacts = [dict(edge="bottom", start=3, width=10, n=1.03, T=1.0, vx=0.004, vy=0.002),
                dict(edge="bottom", start=22, width=9, n=0.98, T=1.01),
                dict(edge="left", start=0, width=7, n=1.01, T=0.99, vy=-0.003),
                dict(edge="top", start=20, width=14, n=1.0, T=1.02)]
    F = (2e-4, -1e-4)
    n, T, vx, vy = _smooth_fields(nx, ny, amp=2e-2, seed=11)
    A = oracle.Lattice(st, nx, ny, contacts=contacts, tau=0.9, F=F)
    A.init_fields(n, T, vx, vy)
    A.run(12)
    fa = A.fields()
    # clockwise quarter turn: a vector (ax, ay) becomes (ay, -ax); edges map
    # bottom -> left (position along the edge: x -> y' = nx - 1 - x),
    # left -> top (y -> x' = y), top -> right, right -> bottom
    rot = []
    for c in contacts:
        s, w_ = c["start"], c["width"]
        if c["edge"] == "bottom":
            e, s2 = "left", nx - s - w_
        elif c["edge"] == "top":
            e, s2 = "right", nx - s - w_
        elif c["edge"] == "left":
            e, s2 = "top", s
        else:
            e, s2 = "bottom", s
        rot.append(dict(c, edge=e, start=s2, vx=c.get("vy", 0.0), vy=-c.get("vx", 0.0)))
    B = oracle.Lattice(st, ny, nx, contacts=rot, tau=0.9, F=(F[1], -F[0]))
    B.init_fields(_rotate_cw(n), _rotate_cw(T), _rotate_cw(vy), _rotate_cw(-vx))
    B.run(12)
    fb = B.fields()
    assert np.abs(fb["n"] - _rotate_cw(fa["n"])).max() < 1e-13
    umax = np.hypot(fa["vx"], fa["vy"]).max()
    assert np.abs(fb["vx"] - _rotate_cw(fa["vy"])).max() < 1e-12 * umax
    assert np.abs(fb["vy"] - _rotate_cw(-fa["vx"])).max() < 1e-12 * umax
    # the same run with the sides swapped wrongly (left contact reflected onto
    # the bottom instead) does not match: the test sees the edge mapping
    bad = [dict(r, edge="bottom") if r["edge"] == "top" else r for r in rot]
    C = oracle.Lattice(st, ny, nx, contacts=bad, tau=0.9, F=(F[1], -F[0]))
    C.init_fields(_rotate_cw(n), _rotate_cw(T), _rotate_cw(vy), _rotate_cw(-vx))
    C.run(12)
    assert np.abs(C.fields()["n"] - _rotate_cw(fa["n"])).max() > 1e-8


def test_corner_sources_bounce_back_and_spans_pull_equilibria():
    """Streaming alone on arbitrary post-collision values: at a site next to a
    corner whose two edges both carry contact spans, a population whose
    source lies off the lattice in both axes comes back reversed from the
    site itself (R12: corners are walls), one whose source lies in a span
    takes that contact's equilibrium, and the rest are pulled."""
    st = _st()
    nx, ny = 20, 18
    contacts = [dict(edge="bottom", start=0, width=12, n=1.05, T=1.0),
                dict(edge="left", start=0, width=12, n=0.95, T=1.02, vx=0.01)]
    L = oracle.Lattice(st, nx, ny, contacts=contacts)
    rng = np.random.default_rng(4)
    fstar = rng.uniform(0.5, 1.5, size=(48, ny, nx))
    fnew = L.stream(fstar)
    feq_b = st.feq(1.05, 1.0, oracle.four_velocity(0.0, 0.0))
    feq_l = st.feq(0.95, 1.02, oracle.four_velocity(0.01, 0.0))
    kinds = {"corner": 0, "bottom": 0, "left": 0, "pull": 0}
    for (x, y) in [(0, 0), (1, 2), (3, 3), (4, 1), (2, 4)]:
        for i in range(48):
            sx, sy = x - st.cx[i], y - st.cy[i]
            got = fnew[i, y, x]
            if sx < 0 and sy < 0:
                assert got == fstar[st.opp[i], y, x], (x, y, i)
                kinds["corner"] += 1
            elif sy < 0:
                assert got == feq_b[i], (x, y, i)
                kinds["bottom"] += 1
            elif sx < 0:
                assert got == feq_l[i], (x, y, i)
                kinds["left"] += 1
            else:
                assert got == fstar[i, sy, sx], (x, y, i)
                kinds["pull"] += 1
    assert min(kinds.values()) > 0, kinds


def test_long_double_build_solves_the_same_problem():
    """The oracle built with long double arithmetic (the reference that
    measures the float64 build's rounding floor) runs the same discrete
    problem on the same float64 constants: on a run with walls, contacts and
    a drive its fields agree with the float64 build to round-off, and differ
    from it (it is a different evaluation)."""
    sd = oracle.stencil()
    sl = oracle.stencil(long_double=True)
    assert sl.real == np.longdouble and oracle.lib(True).orc_real_bytes() == 16
    nx, ny = 30, 22
    contacts = [dict(edge="bottom", start=4, width=8, n=1.03, T=1.0), dict(edge="right", start=5, width=9, n=0.98)]
    out = []
    for st in (sd, sl):
        L = oracle.Lattice(st, nx, ny, contacts=contacts, tau=0.8, F=(1e-4, 2e-5))
        L.init_fields(*_smooth_fields(nx, ny, amp=2e-2))
        L.run(20)
        out.append(L.fields())
    umax = float(np.hypot(out[1]["vx"], out[1]["vy"]).max())
    assert float(np.abs(out[0]["n"] - out[1]["n"]).max()) < 1e-14
    du = float(np.hypot(out[0]["vx"] - out[1]["vx"], out[0]["vy"] - out[1]["vy"]).max())
    assert 0.0 < du < 1e-13 * umax
