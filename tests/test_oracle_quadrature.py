"""Pins of the oracle's quadrature and Appendix A polynomials (CPU only).

Each check compares the oracle with something the paper or the mathematics
fixes: the printed weights (Sec. 2.3), the 48-component count, the exact
continuum moments of the rest-frame weight, and orthonormality (Eq.
``orthonormal``).
"""
import math

import numpy as np
import pytest
import sympy as sp

import oracle
from oracle import appendix, quadrature
from conftest import read_golden


def test_printed_values_match_golden_fixture():
    rows = read_golden("printed_quadrature.txt")
    w1, w2, p0 = quadrature.printed_values()
    for j, row in enumerate(rows):
        assert int(row[0]) == j + 1
        assert float(row[1]) == w1[j] and float(row[2]) == w2[j] and float(row[3]) == p0[j]


def test_stencil_has_48_components_of_radius_5():
    quadrature.check_directions()
    nodes = quadrature.node_table()
    assert len(nodes["w"]) == 48
    pairs = {(cx, cy) for cx, cy in zip(nodes["cx"], nodes["cy"])}
    expected = {(sx * a, sy * b) for a, b in ((3, 4), (4, 3)) for sx in (1, -1) for sy in (1, -1)}
    expected |= {(5, 0), (-5, 0), (0, 5), (0, -5)}
    assert pairs == expected
    # opposite populations: reversed hop, same shell and weight
    for i, o in enumerate(nodes["opp"]):
        assert (nodes["cx"][o], nodes["cy"][o]) == (-nodes["cx"][i], -nodes["cy"][i])
        assert nodes["p0"][o] == nodes["p0"][i] and nodes["w"][o] == nodes["w"][i]


def test_polish_stays_within_print_truncation():
    q = quadrature.polished()
    w1, w2, p0 = quadrature.printed_values()
    printed = w1 + w2 + p0
    polished = [float(v) for v in q["w1"] + q["w2"] + q["p0"]]
    for a, b in zip(printed, polished):
        # printed values are truncated after 12 decimals
        assert abs(a - b) <= 1.1e-12
        assert b > 0.0
    assert q["residual"] < 1e-40
    assert q["residual_printed"] > 1e-7  # the print alone does not satisfy the conditions


def test_solution_set_is_rank_deficient():
    q = quadrature.polished()
    assert q["rank"] == 10
    s = sorted(q["singular_values"], reverse=True)
    assert s[9] > 1e-2 and s[10] < 1e-30


def test_monomial_moments_in_float64():
    """All 84 monomial conditions of degree <= 6 hold in float64 to round-off."""
    nodes = quadrature.node_table()
    p0 = np.array(nodes["p0"])
    ux = np.array(nodes["cx"]) / 5.0
    uy = np.array(nodes["cy"]) / 5.0
    w = np.array(nodes["w"])
    for deg in range(7):
        for a in range(deg + 1):
            for b in range(deg - a + 1):
                c = deg - a - b
                disc = float(np.sum(w * p0**deg * ux**b * uy**c))
                exact = float(quadrature.continuum_moment(a, b, c))
                assert abs(disc - exact) <= 4e-15 * max(1.0, math.factorial(deg)), (a, b, c, disc, exact)


def test_appendix_a_continuum_orthonormality_exact():
    J = appendix.polynomials()
    for a in range(16):
        for b in range(a, 16):
            val = appendix.inner(J[a] * J[b])
            assert sp.simplify(val - (1 if a == b else 0)) == 0, (appendix.NAMES[a], appendix.NAMES[b], val)


@pytest.mark.parametrize("use_printed,tol_lo,tol_hi", [(False, 0.0, 2e-15), (True, 1e-10, 1e-7)])
def test_discrete_gram_is_identity(use_printed, tol_lo, tol_hi):
    """Eq. orthonormal on the lattice: sum_i w_i J_l(p_i) J_k(p_i) = delta_lk."""
    st = oracle.stencil(use_printed)
    G = (st.J * st.w[:, None]).T @ st.J
    err = np.abs(G - np.eye(16)).max()
    assert tol_lo <= err <= tol_hi, err


def test_weights_sum_to_one_and_first_moments():
    st = oracle.stencil()
    assert abs(st.w.sum() - 1.0) < 1e-15
    assert abs((st.w * st.p0).sum() - 1.0) < 1e-15
    assert abs((st.w * st.px).sum()) < 1e-16 and abs((st.w * st.py).sum()) < 1e-16
