"""Oracle side: quadratures on prescribed nodes (Sec. 2.3), the search the
paper describes for new stencils and masses.

Test infrastructure only (see ``oracle/__init__.py``).

Definition (Sec. 2.3, Eq. ``orthonormal``): weights w_i >= 0 on nodes p_i
such that sum_i w_i J_l(p_i) J_k(p_i) = delta_lk for the polynomials up to
the chosen order N.  The products J_l J_k span the polynomials of degree
<= 2N on the mass shell, so the conditions are the exactness of

    sum_i w_i M(p_i) = <M>   for every monomial M = p0^a px^b py^c, a+b+c <= 2N,

with <M> the moment of the rest Maxwell-Juttner weight omega(p0) ~
exp(-p0 / T0) (T0 = 1, mass mbar = m / T0) over d^2p / p0, normalised to
<1> = 1 (Eq. ``mj-poly-weighting-factor``).

* ``mj_moment``: <M> by numerical integration of that definition (mpmath
  quadrature in the angle and in p0 over [mbar, inf)).
* ``massive_nodes``: the nodes of Eq. ``discrete-quadri-momentum`` and
  Eq. ``discrete-p0``: p_i = p0_i (1, v0 n_i), p0_i = mbar gamma_i,
  gamma_i = 1 / sqrt(1 - v0^2 |n_i|^2).
* ``node_weights``: the weights of a node set from all the monomial
  conditions (one weight per node, no symmetry assumed; least squares,
  minimum norm) and the largest violation relative to the moment's scale.
* ``moment_residual``: the largest violation for given weights.
"""
from __future__ import annotations

import functools
import math

import mpmath as mp
import numpy as np

# Sec. 2.3, Fig. `stencil` (left): the 45-component stencil printed for mbar = 5.
M5_ORBIT_REPS = ((0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2), (3, 0), (3, 2), (3, 3), (4, 0))


def full_symmetric(reps):
    """The (+-x, +-y)_FS closure of representative vectors: all sign changes
    and the exchange of x and y, without repeats, in a fixed order."""
    out = []
    for x, y in reps:
        for v in ((x, y), (-x, y), (x, -y), (-x, -y), (y, x), (-y, x), (y, -x), (-y, -x)):
            if v not in out:
                out.append(v)
    return out


def monomials(order: int):
    """Exponents (a, b, c) of p0^a px^b py^c with a + b + c <= 2 * order."""
    top = 2 * order
    return [(a, b, c) for a in range(top + 1) for b in range(top + 1 - a) for c in range(top + 1 - a - b)]


@functools.lru_cache(maxsize=None)
def mj_moment(mbar: float, a: int, b: int, c: int, dps: int = 30) -> float:
    """<p0^a px^b py^c> under omega ~ exp(-p0) on the shell p0^2 = mbar^2 + p^2,
    normalised by <1>, by numerical integration of the definition: with
    d^2p / p0 = dp0 dtheta (p dp = p0 dp0),
        <M> = int dtheta int_mbar^inf dp0 e^{-p0} p0^a (p cos)^b (p sin)^c
              / (2 pi int_mbar^inf e^{-p0} dp0),   p = sqrt(p0^2 - mbar^2)."""
    with mp.workdps(dps):
        m = mp.mpf(mbar)

        def radial(k):
            f = lambda p0: mp.exp(-(p0 - m)) * p0 ** a * (p0 * p0 - m * m) ** (mp.mpf(k) / 2)
            return mp.quad(f, [m, m + 10, m + 40, mp.inf])

        ang = mp.quad(lambda t: mp.cos(t) ** b * mp.sin(t) ** c, [0, mp.pi / 2, mp.pi, 3 * mp.pi / 2, 2 * mp.pi])
        norm = 2 * mp.pi * mp.quad(lambda p0: mp.exp(-(p0 - m)), [m, m + 10, mp.inf])
        return float(ang * radial(b + c) / norm)


def massive_nodes(mbar: float, v0: float, vectors):
    """(p0, px, py) arrays of Eq. discrete-quadri-momentum with Eq. discrete-p0."""
    n = np.asarray(vectors, dtype=np.float64)
    v = v0 * np.hypot(n[:, 0], n[:, 1])
    if np.any(v >= 1.0):
        raise ValueError("v0 |n_i| must stay below 1")
    p0 = mbar / np.sqrt(1.0 - v * v)
    return p0, p0 * v0 * n[:, 0], p0 * v0 * n[:, 1]


def _system(mbar, p0, px, py, order):
    mons = monomials(order)
    A = np.array([p0 ** a * px ** b * py ** c for (a, b, c) in mons])
    rhs = np.array([mj_moment(float(mbar), a, b, c) for (a, b, c) in mons])
    # each condition divided by the size of its moment (at least 1), so that
    # the high moments do not swamp the low ones
    scale = np.maximum(np.abs(rhs), 1.0)
    return A / scale[:, None], rhs / scale


def node_weights(mbar, p0, px, py, order=3):
    """Minimum-norm least-squares weights of all monomial conditions and the
    largest scaled violation."""
    A, rhs = _system(mbar, p0, px, py, order)
    w, *_ = np.linalg.lstsq(A, rhs, rcond=None)
    return w, float(np.abs(A @ w - rhs).max())


def moment_residual(mbar, p0, px, py, w, order=3):
    A, rhs = _system(mbar, p0, px, py, order)
    return float(np.abs(A @ np.asarray(w) - rhs).max())


def orbits(vectors):
    """Partition of a full-symmetric stencil into (+-x, +-y)_FS orbits (lists of vectors)."""
    left = list(vectors)
    out = []
    while left:
        orb = [v for v in full_symmetric([left[0]]) if v in left]
        if len(orb) != len(full_symmetric([left[0]])):
            raise ValueError("stencil is not closed under the symmetries of the square")
        out.append(orb)
        left = [v for v in left if v not in orb]
    return out


def orbit_weights_mp(mbar, v0, vectors, order=3, dps=40):
    """Weights of a full-symmetric massive stencil in extended precision: the
    conditions are invariant under the symmetries of the square, so a
    solution can be averaged over them and one weight per orbit suffices.
    All monomial conditions of degree <= 2 * order (scaled as in
    node_weights) are solved by least squares.  Returns the
    orbits, their weights (per node of the orbit) and the residual norm."""
    orbs = orbits(vectors)
    mons = monomials(order)
    with mp.workdps(dps):
        m = mp.mpf(mbar)
        v0m = mp.mpf(v0)
        A = mp.matrix(len(mons), len(orbs))
        rhs = mp.matrix(len(mons), 1)
        nodes = []
        for orb in orbs:
            pts = []
            for x, y in orb:
                v = v0m * mp.sqrt(x * x + y * y)
                p0 = m / mp.sqrt(1 - v * v)
                pts.append((p0, p0 * v0m * x, p0 * v0m * y))
            nodes.append(pts)
        for r, (a, b, c) in enumerate(mons):
            mom = mp.mpf(mj_moment(float(mbar), a, b, c, dps=dps + 5))
            sc = max(abs(mom), mp.mpf(1))
            rhs[r] = mom / sc
            for k, pts in enumerate(nodes):
                A[r, k] = sum(p0 ** a * px ** b * py ** c for (p0, px, py) in pts) / sc
        # normal equations: the system has full column rank and a condition
        # number far below 10^dps, so squaring it loses nothing that matters
        w = mp.lu_solve(A.T * A, A.T * rhs)
        res = mp.norm(A * w - rhs)
        return orbs, [float(x) for x in w], float(res)


def scan_massive(mbar, vectors, order=3, v0_grid=None):
    """(v0, smallest weight, residual) over a grid of v0 in (0, 1/max|n|)."""
    rmax = max(math.hypot(x, y) for x, y in vectors)
    grid = v0_grid if v0_grid is not None else np.linspace(0.02 / rmax, 0.999 / rmax, 400)
    out = []
    for v0 in grid:
        w, res = node_weights(mbar, *massive_nodes(mbar, v0, vectors), order)
        out.append((float(v0), float(w.min()), res))
    return out
