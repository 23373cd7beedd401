"""Gauss-Lobatto-Legendre points, weights and 1D element operators.

Follows Sec. III.A: the element basis is the tensor product of 1D Lagrange
polynomials through the Gauss-Lobatto points, and every integral is taken
with the Gauss-Lobatto rule on the same points (the quadrature formula of
that section).  Reference interval [-1, 1].

Test infrastructure only (see ``oracle/__init__``).
"""
import numpy as np
from numpy.polynomial import legendre as npleg


def gll(p):
    """Return (xi, w): the p+1 Gauss-Lobatto nodes (ascending) and weights.

    Interior nodes are the roots of P_p'(x); weights are 2/(p(p+1)P_p(x)^2).
    """
    if p < 1:
        raise ValueError("p >= 1")
    cp = np.zeros(p + 1)
    cp[p] = 1.0
    if p == 1:
        inner = np.zeros(0)
    else:
        inner = np.sort(np.real(npleg.legroots(npleg.legder(cp))))
    xi = np.concatenate([[-1.0], inner, [1.0]])
    pv = npleg.legval(xi, cp)
    w = 2.0 / (p * (p + 1) * pv ** 2)
    return xi, w


def lagrange_eval(xi, x):
    """L[a, j] = l_a(x_j): the Lagrange basis through nodes xi at points x."""
    x = np.atleast_1d(np.asarray(x, dtype=float))
    n = len(xi)
    L = np.ones((n, len(x)))
    for a in range(n):
        for b in range(n):
            if b != a:
                L[a] *= (x - xi[b]) / (xi[a] - xi[b])
    return L


def lagrange_deriv(xi, x):
    """dL[a, j] = l_a'(x_j), by the product rule (no barycentric tricks)."""
    x = np.atleast_1d(np.asarray(x, dtype=float))
    n = len(xi)
    dL = np.zeros((n, len(x)))
    for a in range(n):
        for c in range(n):
            if c == a:
                continue
            term = np.ones(len(x)) / (xi[a] - xi[c])
            for b in range(n):
                if b != a and b != c:
                    term = term * (x - xi[b]) / (xi[a] - xi[b])
            dL[a] += term
    return dL


def operators_1d(p):
    """Return (xi, w, D, A): D[a, b] = l_b'(xi_a) and A = D^T diag(w) D.

    A is the reference 1D stiffness integrated with the GLL rule, which is
    exact for the degree 2p-2 integrand; diag(w) is the lumped 1D mass.
    """
    xi, w = gll(p)
    D = lagrange_deriv(xi, xi).T
    A = D.T @ np.diag(w) @ D
    return xi, w, D, A
