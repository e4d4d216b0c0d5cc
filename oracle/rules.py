"""1D quadrature rules and Lagrange interpolation on them (FP64).

Test infrastructure of the oracle.  Nodes and weights are returned in extended precision
(long double); the discretisation's tables are built from them in extended precision, so a
table's last-bit rounding cannot leak the large mean pressure into the residual.
Rules used by the discretisation:
  GL(n)   Gauss-Lobatto, n points including both ends, exact to degree 2n-3
  LGR(n)  left Gauss-Radau, n points including -1 but not +1, exact to degree 2n-2
  LG(n)   Gauss-Legendre, n interior points, exact to degree 2n-1
The node sets are the tensor-product building blocks of the element nodes (paper
Sec. 2: element-local polynomials of degree N; the tensor-product operators of
Sec. 1).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg


def legendre(k: int, x):
    """P_k(x)."""
    c = np.zeros(k + 1)
    c[k] = 1.0
    return npleg.legval(np.asarray(x, dtype=float), c)


def _legendre_ld(k, x):
    """P_k(x) and P_k'(x) in extended precision (three-term recurrence)."""
    x = np.asarray(x, dtype=np.longdouble)
    p0, p1 = np.ones_like(x), x.copy()
    d0, d1 = np.zeros_like(x), np.ones_like(x)
    if k == 0:
        return p0, d0
    for j in range(1, k):
        p2 = ((2 * j + 1) * x * p1 - j * p0) / (j + 1)
        d2 = d0 + (2 * j + 1) * p1
        p0, p1, d0, d1 = p1, p2, d1, d2
    return p1, d1


def _newton_ld(x0, f, iters=8):
    """Polish roots with Newton steps in extended precision; returns long double roots."""
    x = np.asarray(x0, dtype=np.longdouble)
    for _ in range(iters):
        v, d = f(x)
        x = x - v / d
    return x


def gauss_lobatto(n: int):
    """n-point Gauss-Lobatto rule: nodes -1, +1 and the roots of P'_{n-1};
    weights 2 / (N (N+1) P_N(x)^2), N = n-1.  Roots from the companion matrix, polished and
    weighted in extended precision."""
    if n < 2:
        raise ValueError("Gauss-Lobatto needs n >= 2")
    N = n - 1
    cN = np.zeros(N + 1)
    cN[N] = 1.0
    interior = np.sort(np.real(npleg.legroots(npleg.legder(cN)))) if N >= 2 else np.array([])

    def f(x):  # P'_N and P''_N via (1-x^2) P_N'' = 2x P_N' - N(N+1) P_N
        p, d = _legendre_ld(N, x)
        return d, (2 * x * d - N * (N + 1) * p) / (1 - x * x)

    xi = _newton_ld(interior, f) if interior.size else np.array([], dtype=np.longdouble)
    x = np.concatenate([[np.longdouble(-1)], xi, [np.longdouble(1)]])
    pN, _ = _legendre_ld(N, x)
    w = 2 / (N * (N + 1) * pN * pN)
    return x, w


def gauss_radau_left(n: int):
    """n-point left Gauss-Radau rule: -1 and the roots of (P_{n-1}+P_n)/(1+x);
    weights 2/n^2 at -1 and (1-x)/(n^2 P_{n-1}(x)^2) elsewhere (polished and weighted in
    extended precision)."""
    if n < 1:
        raise ValueError("Gauss-Radau needs n >= 1")
    c = np.zeros(n + 1)
    c[n - 1] = 1.0
    c[n] = 1.0
    r = np.sort(np.real(npleg.legroots(c)))[1:]

    def f(x):
        a, da = _legendre_ld(n, x)
        b, db = _legendre_ld(n - 1, x)
        return a + b, da + db

    xr = _newton_ld(r, f) if r.size else np.array([], dtype=np.longdouble)
    x = np.concatenate([[np.longdouble(-1)], xr])
    w = np.empty(n, dtype=np.longdouble)
    w[0] = np.longdouble(2) / (n * n)
    pm, _ = _legendre_ld(n - 1, x[1:])
    w[1:] = (1 - x[1:]) / (n * n * pm * pm)
    return x, w


def gauss_legendre(n: int):
    """n-point Gauss-Legendre rule: library nodes, polished and weighted
    (2 / ((1-x^2) P_n'(x)^2)) in extended precision."""
    x, _ = npleg.leggauss(n)
    xl = _newton_ld(x, lambda t: _legendre_ld(n, t))
    _, d = _legendre_ld(n, xl)
    w = 2 / ((1 - xl * xl) * d * d)
    return xl, w


RULES = {"GL": gauss_lobatto, "LGR": gauss_radau_left, "LG": gauss_legendre}


def lagrange_eval(xn, x):
    """L[p, j] = l_j(x_p) for the Lagrange basis on nodes xn (product formula)."""
    xn = np.asarray(xn)
    x = np.atleast_1d(np.asarray(x))
    dt = np.result_type(xn, x, np.float64)
    n = xn.size
    L = np.ones((x.size, n), dtype=dt)
    for j in range(n):
        for m in range(n):
            if m != j:
                L[:, j] *= (x - xn[m]) / (xn[j] - xn[m])
    return L


def lagrange_deriv_eval(xn, x):
    """dL[p, j] = l_j'(x_p), from the product rule applied to the product formula."""
    xn = np.asarray(xn)
    x = np.atleast_1d(np.asarray(x))
    dt = np.result_type(xn, x, np.float64)
    n = xn.size
    dL = np.zeros((x.size, n), dtype=dt)
    for j in range(n):
        for k in range(n):
            if k == j:
                continue
            term = np.full(x.size, 1 / (xn[j] - xn[k]), dtype=dt)
            for m in range(n):
                if m != j and m != k:
                    term *= (x - xn[m]) / (xn[j] - xn[m])
            dL[:, j] += term
    return dL


def derivative_matrix(xn):
    """D[i, j] = l_j'(x_i)."""
    return lagrange_deriv_eval(xn, xn)
