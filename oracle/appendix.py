"""Oracle side: Appendix A polynomials and the force projection matrices.

Test infrastructure only (see ``oracle/__init__.py``).

* ``polynomials()`` transcribes the 16 orthonormal polynomials J^(k) of
  Appendix A (m = 0, third order) as sympy expressions in (p0, px, py), in
  the order the appendix lists them.
* ``inner(g)`` is the weighted average <g> = integral of omega g dp/p0 with
  the rest-frame weight omega = exp(-p0)/(2 pi) (Eq. ``mj-poly-weighting-
  factor``, T0 = 1).  On the massless shell p = p0 (1, cos t, sin t) and
  dp/p0 = dp0 dt, so it is (1/2pi) times a double integral over p0 >= 0 and
  t in [0, 2pi).  The angle is integrated first: the force terms below carry
  a factor 1/p0 that is only integrable after the angular mean removes it.
* ``force_matrices()`` gives C_x, C_y with b_j = C_j a (Sec. 2.4, forcing
  scheme): b^(k)_j is the projection of the momentum derivative of the
  equilibrium onto J^(k).  Integrating by parts on the shell,
      b^(k)_j = - integral f^eq [ d_j J_k - J_k p^j / p0^2 ] dp/p0,
  where d_j is the on-shell derivative d/dp^j + (p^j/p0) d/dp0.  With f^eq
  replaced by its order-3 expansion omega sum_m a_m J_m (Eq.
  ``feq-expansion``), b_j = C_j a with
      C_j[k, m] = - < J_m ( d_j J_k - J_k p^j / p0^2 ) >.
"""
from __future__ import annotations

import functools

import numpy as np
import sympy as sp

P0, PX, PY = sp.symbols("p0 px py")
_R, _C, _S = sp.symbols("r c s")  # shell radius and direction cosines (on-shell form)

NAMES = ("0", "1_0", "1_x", "1_y", "2_00", "2_0x", "2_0y", "2_xx", "2_xy",
         "3_000", "3_xxx", "3_00x", "3_0xx", "3_00y", "3_xxy", "3_0xy")


@functools.lru_cache(maxsize=1)
def polynomials():
    """Appendix A, third-order 2-D relativistic orthonormal polynomials (m = 0)."""
    r3, r15, r6, r10 = sp.sqrt(3), sp.sqrt(15), sp.sqrt(6), sp.sqrt(10)
    half = sp.Rational(1, 2)
    s53 = sp.sqrt(sp.Rational(5, 3))
    s23 = sp.sqrt(sp.Rational(2, 3))
    s25 = sp.sqrt(sp.Rational(2, 5))
    p0, px, py = P0, PX, PY
    return (
        sp.Integer(1),
        p0 - 1,
        px,
        py,
        half * p0**2 - 2 * p0 + 1,
        p0 * px / r3 - r3 * px,
        p0 * py / r3 - r3 * py,
        px**2 / r3 - p0**2 / (2 * r3),
        px * py / r3,
        p0**3 / 6 - sp.Rational(3, 2) * p0**2 + 3 * p0 - 1,
        -p0 * px + px**3 / 6 + sp.Rational(3, 2) * px,
        p0**2 * px / r15 - s53 * p0 * px - px**3 / (2 * r15) + r15 / 2 * px,
        -p0**3 / (2 * r15) + half * s53 * p0**2 + p0 * px**2 / r15 - s53 * px**2,
        p0**2 * py / (2 * r6) - 2 * s23 * p0 * py + r6 * py,
        sp.Rational(1, 3) * s25 * px**2 * py - p0**2 * py / (6 * r10),
        p0 * px * py / r15 - s53 * px * py,
    )


def _angular_mean(b: int, c: int) -> sp.Expr:
    if b % 2 or c % 2:
        return sp.Integer(0)
    k, l = b // 2, c // 2
    return sp.gamma(k + sp.Rational(1, 2)) * sp.gamma(l + sp.Rational(1, 2)) / (sp.pi * sp.gamma(k + l + 1))


def inner(expr) -> sp.Expr:
    """<expr> under omega dp/p0 on the massless shell, angle first (exact)."""
    on_shell = sp.expand(sp.sympify(expr).subs({P0: _R, PX: _R * _C, PY: _R * _S}, simultaneous=True))
    # Laurent terms r^e c^b s^c: collect the angular mean of each power of r.
    by_power: dict[int, sp.Expr] = {}
    for term in sp.Add.make_args(on_shell):
        coeff, mono = term.as_coeff_Mul()
        powers = mono.as_powers_dict()
        e = int(powers.get(_R, 0))
        b = int(powers.get(_C, 0))
        c = int(powers.get(_S, 0))
        rest = mono / (_R**e * _C**b * _S**c)
        by_power[e] = by_power.get(e, 0) + coeff * rest * _angular_mean(b, c)
    total = sp.Integer(0)
    for e, ang in by_power.items():
        ang = sp.nsimplify(sp.simplify(ang)) if ang != 0 else ang
        if ang == 0:
            continue
        if e < 0:
            raise ValueError(f"non-integrable r^{e} term survives the angular mean: {ang}")
        total += ang * sp.factorial(e)
    return sp.simplify(total)


def shell_derivative(expr, axis: str) -> sp.Expr:
    """On-shell derivative d/dp^j of expr(p0(p), px, py), p0 = |p| (m = 0)."""
    pj = PX if axis == "x" else PY
    return sp.diff(expr, pj) + sp.diff(expr, P0) * pj / P0


@functools.lru_cache(maxsize=1)
def force_matrices():
    """(C_x, C_y) as float64 16x16 arrays, exact entries rounded once."""
    J = polynomials()
    mats = []
    for axis in ("x", "y"):
        pj = PX if axis == "x" else PY
        C = np.zeros((16, 16))
        for k in range(16):
            g = shell_derivative(J[k], axis) - J[k] * pj / P0**2
            for m in range(16):
                C[k, m] = float(-inner(J[m] * g))
        mats.append(C)
    return mats[0], mats[1]


@functools.lru_cache(maxsize=1)
def _lambdified():
    J = polynomials()
    return [sp.lambdify((P0, PX, PY), e, "numpy") for e in J]


def evaluate(p0, px, py) -> np.ndarray:
    """J_k at arrays of momenta; shape (..., 16), float64."""
    p0 = np.asarray(p0, dtype=np.float64)
    px = np.asarray(px, dtype=np.float64)
    py = np.asarray(py, dtype=np.float64)
    out = [np.broadcast_to(np.asarray(f(p0, px, py), dtype=np.float64), p0.shape) for f in _lambdified()]
    return np.stack(out, axis=-1)


def node_J_table(nodes: dict) -> np.ndarray:
    """48 x 16 table J_k(p_i) at the quadrature nodes."""
    return evaluate(np.array(nodes["p0"]), np.array(nodes["px"]), np.array(nodes["py"]))


def evaluate_complex(p0, px, py) -> np.ndarray:
    """J_k at complex momenta (for complex-step derivatives); shape (..., 16)."""
    p0 = np.asarray(p0, dtype=np.complex128)
    px = np.asarray(px, dtype=np.complex128)
    py = np.asarray(py, dtype=np.complex128)
    out = [np.broadcast_to(np.asarray(f(p0, px, py), dtype=np.complex128), p0.shape) for f in _lambdified()]
    return np.stack(out, axis=-1)
