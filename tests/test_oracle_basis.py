"""Pins of the oracle's 1D ingredients against closed forms and exact polynomial algebra.

GLL nodes/weights and the nodal derivative matrix enter the paper through Eq.
numerical_integ (nodes double as quadrature points) and Eq. deriv_u (derivatives as
sums of basis derivatives at the nodes).
"""
import math

import numpy as np
import numpy.polynomial.polynomial as P
import pytest

from oracle import gll


def test_gll_p4_closed_form():
    # Textbook closed form for 5 Lobatto points.
    x, w = gll.gll(4)
    s = math.sqrt(3.0 / 7.0)
    np.testing.assert_allclose(x, [-1, -s, 0, s, 1], atol=1e-15)
    np.testing.assert_allclose(w, [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10], rtol=1e-14)


def test_gll_p5_closed_form():
    x, w = gll.gll(5)
    a = math.sqrt(1.0 / 3.0 + 2.0 * math.sqrt(7.0) / 21.0)
    b = math.sqrt(1.0 / 3.0 - 2.0 * math.sqrt(7.0) / 21.0)
    np.testing.assert_allclose(x, [-1, -a, -b, b, a, 1], atol=1e-15)
    wa = (14.0 - math.sqrt(7.0)) / 30.0
    wb = (14.0 + math.sqrt(7.0)) / 30.0
    np.testing.assert_allclose(w, [1 / 15, wa, wb, wb, wa, 1 / 15], rtol=1e-14)


@pytest.mark.parametrize("p", range(1, 13))
def test_gll_quadrature_exact_to_degree_2p_minus_1(p):
    x, w = gll.gll(p)
    assert abs(w.sum() - 2.0) < 1e-14
    for k in range(2 * p):
        exact = (1.0 - (-1.0) ** (k + 1)) / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 1e-13, k
    # and not exact for degree 2p (Lobatto quadrature has degree of exactness 2p-1)
    k = 2 * p
    assert abs(np.dot(w, x ** k) - 2.0 / (k + 1)) > 1e-9


@pytest.mark.parametrize("p", range(1, 11))
def test_derivative_matrix_exact_on_polynomials(p):
    x, _ = gll.gll(p)
    D = gll.derivative_matrix(p)
    np.testing.assert_allclose(D @ np.ones(p + 1), 0.0, atol=1e-13)
    for k in range(1, p + 1):
        np.testing.assert_allclose(D @ x ** k, k * x ** (k - 1), atol=2e-12 * p * p)


def _lagrange_polys(x):
    """Lagrange cardinal polynomials built independently with numpy.polynomial."""
    out = []
    for j in range(len(x)):
        roots = np.delete(x, j)
        c = P.polyfromroots(roots)
        out.append(c / P.polyval(x[j], c))
    return out


@pytest.mark.parametrize("p", [2, 4, 5, 7])
def test_stiffness_1d_matches_exact_integral(p):
    """D^T W D is the exact 1D stiffness: int_{-1}^{1} l_i' l_j' (degree 2p-2 <= 2p-1)."""
    x, w = gll.gll(p)
    D = gll.derivative_matrix(p)
    S = D.T @ np.diag(w) @ D
    L = _lagrange_polys(x)
    exact = np.empty((p + 1, p + 1))
    for i in range(p + 1):
        for j in range(p + 1):
            prod = P.polymul(P.polyder(L[i]), P.polyder(L[j]))
            integ = P.polyint(prod)
            exact[i, j] = P.polyval(1.0, integ) - P.polyval(-1.0, integ)
    np.testing.assert_allclose(S, exact, atol=1e-11 * np.abs(exact).max())


def test_lagrange_values_cardinal():
    p = 5
    x, _ = gll.gll(p)
    np.testing.assert_allclose(gll.lagrange_values(p, x, x), np.eye(p + 1), atol=1e-14)
