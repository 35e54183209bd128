"""Pins of the oracle's quadrature search (Sec. 2.3), CPU only.

* Moments of the rest Maxwell-Juttner weight: massless values (a+b+c)! times
  the angular mean (b-1)!!(c-1)!!/(b+c)!!; massive values from the
  one-dimensional law e^{-(p0 - m)} on [m, inf): <p0> = 1 + m,
  <p0^2> = m^2 + 2m + 2, <px^2> = (<p0^2> - m^2)/2 = 1 + m; odd moments vanish.
* The polished massless quadrature of the paper satisfies every monomial
  condition of degree <= 6 (a second, independent route to Eq. orthonormal).
* The paper's claim for mbar = 5 (Fig. stencil, left): the 45-vector stencil
  carries a third-order quadrature with non-negative weights.  The stored
  solution (written by tests/golden/make_quadrature_search.py from the
  oracle) solves all conditions, is positive, and its v0 is where the
  smallest weight peaks (moving v0 by 1e-4 either way makes a weight negative).
* The massless solutions form a family: a second member (stored by the same
  script, solved from the printed values with the fourth shell moved to
  1.0) satisfies every condition, has positive weights and differs from the
  paper's quadrature.
"""
import math

import numpy as np
import pytest

from conftest import read_golden
from oracle import quadrature as OQ
from oracle import quadrature_search as Q


def _dfact(n):
    return 1 if n <= 0 else n * _dfact(n - 2)


@pytest.mark.parametrize("a,b,c", [(0, 0, 0), (2, 0, 0), (1, 2, 0), (0, 2, 2), (0, 4, 2), (3, 0, 2), (0, 1, 0), (1, 3, 1)])
def test_massless_moments(a, b, c):
    exact = 0.0 if (b % 2 or c % 2) else math.factorial(a + b + c) * _dfact(b - 1) * _dfact(c - 1) / _dfact(b + c)
    assert abs(Q.mj_moment(0.0, a, b, c) - exact) <= 1e-12 * max(1.0, exact)


@pytest.mark.parametrize("m", [0.5, 5.0, 12.0])
def test_massive_moments(m):
    assert abs(Q.mj_moment(m, 0, 0, 0) - 1) < 1e-13
    assert abs(Q.mj_moment(m, 1, 0, 0) - (1 + m)) < 1e-12 * (1 + m)
    assert abs(Q.mj_moment(m, 2, 0, 0) - (m * m + 2 * m + 2)) < 1e-12 * m * m
    assert abs(Q.mj_moment(m, 0, 2, 0) - (1 + m)) < 1e-12 * (1 + m)
    assert abs(Q.mj_moment(m, 0, 0, 2) - (1 + m)) < 1e-12 * (1 + m)
    assert Q.mj_moment(m, 1, 1, 0) == pytest.approx(0.0, abs=1e-14)


def test_polished_massless_quadrature_solves_all_conditions():
    t = OQ.node_table()
    w, p0, px, py = (np.asarray(t[k], dtype=np.float64) for k in ("w", "p0", "px", "py"))
    assert Q.moment_residual(0.0, p0, px, py, w, order=3) < 1e-13


def _golden_m5():
    rows = read_golden("m5_quadrature.txt")
    mbar, v0, wmin, res = (float(x) for x in rows[0])
    orbits = [((int(r[0]), int(r[1])), int(r[2]), float(r[3])) for r in rows[1:]]
    return mbar, v0, wmin, orbits


def test_m5_stencil_has_a_nonnegative_third_order_quadrature():
    mbar, v0, wmin, orbits = _golden_m5()
    vec = Q.full_symmetric(Q.M5_ORBIT_REPS)
    assert len(vec) == 45 and sum(n for _, n, _ in orbits) == 45
    orbs, w, res = Q.orbit_weights_mp(mbar, v0, vec)
    assert res < 1e-25
    assert min(w) > 0 and abs(min(w) - wmin) < 1e-12
    for (rep, n, wk), orb, wo in zip(orbits, orbs, w):
        assert orb[0] == rep and len(orb) == n and abs(wo - wk) <= 1e-10 * max(wk, 1e-3)
    # the same weights, node by node, solve every condition in double precision too
    p0, px, py = Q.massive_nodes(mbar, v0, vec)
    wn = np.array([wk for orb, wk in zip(orbs, w) for _ in orb])
    order_nodes = [v for orb in orbs for v in orb]
    idx = [vec.index(v) for v in order_nodes]
    assert Q.moment_residual(mbar, p0[idx], px[idx], py[idx], wn, order=3) < 1e-9
    # the window is narrow: a step of 1e-4 in v0 either way turns a weight negative
    for dv in (-1e-4, 1e-4):
        assert min(Q.orbit_weights_mp(mbar, v0 + dv, vec)[1]) < 0


def read_family_member():
    rows = read_golden("m0_family_member.txt")
    w1, w2, p0 = ([float(v) for v in rows[k]] for k in range(3))
    return w1, w2, p0


def test_second_massless_family_member():
    w1, w2, p0 = read_family_member()
    t = OQ.node_table(shells=(w1, w2, p0))
    w, q0, px, py = (np.asarray(t[k], dtype=np.float64) for k in ("w", "p0", "px", "py"))
    assert Q.moment_residual(0.0, q0, px, py, w, order=3) < 1e-13
    assert min(w1 + w2) > 0 and min(p0) > 0
    ref = OQ.shell_tables()[2]
    assert max(abs(a - b) for a, b in zip(p0, ref)) > 1e-3
