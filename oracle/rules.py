"""1D quadrature rules and Lagrange interpolation on them (FP64).

Test infrastructure of the oracle.  Rules used by the discretisation:
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


def _polish(roots, f, df, iters=3):
    x = np.array(roots, dtype=float)
    for _ in range(iters):
        d = df(x)
        ok = d != 0
        x[ok] = x[ok] - f(x[ok]) / d[ok]
    return x


def gauss_lobatto(n: int):
    """n-point Gauss-Lobatto rule: nodes -1, +1 and the roots of P'_{n-1};
    weights 2 / (N (N+1) P_N(x)^2), N = n-1."""
    if n < 2:
        raise ValueError("Gauss-Lobatto needs n >= 2")
    N = n - 1
    cN = np.zeros(N + 1)
    cN[N] = 1.0
    d1 = npleg.legder(cN)
    d2 = npleg.legder(cN, 2)
    interior = np.sort(np.real(npleg.legroots(d1))) if N >= 2 else np.array([])
    interior = _polish(interior, lambda x: npleg.legval(x, d1), lambda x: npleg.legval(x, d2))
    x = np.concatenate([[-1.0], interior, [1.0]])
    w = 2.0 / (N * (N + 1) * legendre(N, x) ** 2)
    return x, w


def gauss_radau_left(n: int):
    """n-point left Gauss-Radau rule: -1 and the roots of (P_{n-1}+P_n)/(1+x);
    weights 2/n^2 at -1 and (1-x)/(n^2 P_{n-1}(x)^2) elsewhere."""
    if n < 1:
        raise ValueError("Gauss-Radau needs n >= 1")
    c = np.zeros(n + 1)
    c[n - 1] = 1.0
    c[n] = 1.0
    r = np.sort(np.real(npleg.legroots(c)))
    dc = npleg.legder(c)
    r = _polish(r[1:], lambda x: npleg.legval(x, c), lambda x: npleg.legval(x, dc))
    x = np.concatenate([[-1.0], r])
    w = np.empty(n)
    w[0] = 2.0 / n ** 2
    w[1:] = (1.0 - x[1:]) / (n ** 2 * legendre(n - 1, x[1:]) ** 2)
    return x, w


def gauss_legendre(n: int):
    """n-point Gauss-Legendre rule (library routine)."""
    x, w = npleg.leggauss(n)
    return np.asarray(x, float), np.asarray(w, float)


RULES = {"GL": gauss_lobatto, "LGR": gauss_radau_left, "LG": gauss_legendre}


def lagrange_eval(xn, x):
    """L[p, j] = l_j(x_p) for the Lagrange basis on nodes xn (product formula)."""
    xn = np.asarray(xn, float)
    x = np.atleast_1d(np.asarray(x, float))
    n = xn.size
    L = np.ones((x.size, n))
    for j in range(n):
        for m in range(n):
            if m != j:
                L[:, j] *= (x - xn[m]) / (xn[j] - xn[m])
    return L


def lagrange_deriv_eval(xn, x):
    """dL[p, j] = l_j'(x_p), from the product rule applied to the product formula."""
    xn = np.asarray(xn, float)
    x = np.atleast_1d(np.asarray(x, float))
    n = xn.size
    dL = np.zeros((x.size, n))
    for j in range(n):
        for k in range(n):
            if k == j:
                continue
            term = np.full(x.size, 1.0 / (xn[j] - xn[k]))
            for m in range(n):
                if m != j and m != k:
                    term *= (x - xn[m]) / (xn[j] - xn[m])
            dL[:, j] += term
    return dL


def derivative_matrix(xn):
    """D[i, j] = l_j'(x_i)."""
    return lagrange_deriv_eval(xn, xn)
