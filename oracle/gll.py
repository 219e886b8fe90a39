"""Gauss-Lobatto-Legendre nodes, weights and derivative matrix on [-1, 1].

The paper's local nodes double as quadrature points (Sec. 4.2, Eq. numerical_integ) and
derivatives of u are sums of basis derivatives at those nodes (Eq. deriv_u). On the
tensor-product quadrilateral used here the 1D ingredients are the p+1 GLL points, their
quadrature weights and D[i, j] = l_j'(xi_i), the derivative of the j-th Lagrange
polynomial at node i. The paper's triangle nodes (Blyth-Pozrikidis) are not used.
"""
from __future__ import annotations

import numpy as np


def legendre(p: int, x):
    """P_p(x) and P_{p-1}(x) by the three-term (Bonnet) recurrence."""
    x = np.asarray(x, dtype=np.float64)
    pm1 = np.ones_like(x)
    if p == 0:
        return pm1, np.zeros_like(x)
    pk = x.copy()
    for k in range(1, p):
        pm1, pk = pk, ((2 * k + 1) * x * pk - k * pm1) / (k + 1)
    return pk, pm1


def gll(p: int):
    """Return (nodes xi[0..p] ascending, weights w[0..p]).

    Interior nodes are the roots of P_p'. Newton's method on P_p' starts from the
    Chebyshev-Gauss-Lobatto points -cos(pi i / p); P_p' and P_p'' come from the
    identities (1 - x^2) P_p' = p (P_{p-1} - x P_p) and the Legendre equation
    (1 - x^2) P_p'' = 2 x P_p' - p (p + 1) P_p. Weights: w_i = 2 / (p (p+1) P_p(xi_i)^2).
    """
    if p < 1:
        raise ValueError("p >= 1 required")
    x = -np.cos(np.pi * np.arange(p + 1) / p)
    for _ in range(100):
        xi = x[1:-1]
        P, Pm1 = legendre(p, xi)
        d1 = p * (Pm1 - xi * P) / (1.0 - xi * xi)
        d2 = (2.0 * xi * d1 - p * (p + 1) * P) / (1.0 - xi * xi)
        step = d1 / d2
        x[1:-1] = xi - step
        if np.max(np.abs(step), initial=0.0) < 1e-16:
            break
    x[0], x[-1] = -1.0, 1.0
    # enforce the exact symmetry xi_{p-i} = -xi_i
    x = 0.5 * (x - x[::-1])
    if p % 2 == 0:
        x[p // 2] = 0.0
    P, _ = legendre(p, x)
    w = 2.0 / (p * (p + 1) * P * P)
    return x, w


def derivative_matrix(p: int, x=None):
    """D[i, j] = l_j'(x_i) for the Lagrange basis on the GLL nodes.

    Off-diagonal: (P_p(x_i) / P_p(x_j)) / (x_i - x_j). The diagonal is minus the
    off-diagonal row sum, so derivatives of constants vanish to rounding.
    """
    if x is None:
        x, _ = gll(p)
    P, _ = legendre(p, x)
    n = p + 1
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i != j:
                D[i, j] = (P[i] / P[j]) / (x[i] - x[j])
        D[i, i] = -np.sum(D[i, :])
    return D


def lagrange_values(p: int, x_nodes, t):
    """Values l_j(t) of the Lagrange basis on ``x_nodes`` at points ``t`` -> [len(t), p+1]."""
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    n = p + 1
    out = np.ones((t.size, n))
    for j in range(n):
        for k in range(n):
            if k != j:
                out[:, j] *= (t - x_nodes[k]) / (x_nodes[j] - x_nodes[k])
    return out
