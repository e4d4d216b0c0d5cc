"""Orthonormal modal bases of the collapsed element types (FP64).

Test infrastructure of the oracle.  Modal time stepping (paper Sec. 2, Algorithm 1)
evolves the coefficients of a modal basis phi; the generalised Vandermonde matrix is
V[k, j] = phi_j(eta_k).  The paper does not fix the basis; the reading taken here is the
collapsed-coordinate Jacobi (Dubiner-type) family in the element's cube coordinates eta:

  tet      P_p(e1) ((1-e2)/2)^p P_q^(2p+1,0)(e2) ((1-e3)/2)^(p+q) P_r^(2p+2q+2,0)(e3),  p+q+r <= N
  prism    P_p(e1) P_q(e2) ((1-e3)/2)^p P_r^(2p+1,0)(e3),                       p,q <= N, p+r <= N
  pyramid  P_p(e1) P_q(e2) ((1-e3)/2)^m P_r^(2m+2,0)(e3), m = max(p,q),        p,q <= N, r <= N-m

enumerated with p outermost and r fastest, each scaled to unit norm in the L2 product
of the reference element (geometry.REF_CORNERS); the norm is computed numerically with a
Gauss-Legendre rule that is exact for the integrand.  Jacobi polynomials come from their
three-term recurrence and everything is evaluated in extended precision (long double).
"""
from __future__ import annotations

import numpy as np
from . import geometry, rules

HEX, PRISM, PYR, TET = geometry.HEX, geometry.PRISM, geometry.PYR, geometry.TET


def modes(etype: int, N: int):
    out = []
    if etype == TET:
        for p in range(N + 1):
            for q in range(N + 1 - p):
                for r in range(N + 1 - p - q):
                    out.append((p, q, r))
    elif etype == PRISM:
        for p in range(N + 1):
            for q in range(N + 1):
                for r in range(N + 1 - p):
                    out.append((p, q, r))
    elif etype == PYR:
        for p in range(N + 1):
            for q in range(N + 1):
                for r in range(N + 1 - max(p, q)):
                    out.append((p, q, r))
    else:
        raise ValueError("hexahedra are nodal")
    return out


def n_modes(etype: int, N: int) -> int:
    return len(modes(etype, N))


def _jac(k, alpha, x):
    """P_k^(alpha,0)(x) by the standard three-term recurrence, in the precision of x."""
    x = np.asarray(x)
    p0 = np.ones_like(x)
    if k == 0:
        return p0
    a = alpha
    p1 = ((a + 2) * x + a) / 2
    for n in range(2, k + 1):
        c = 2 * n + a
        a1 = 2 * n * (n + a) * (c - 2)
        a2 = (c - 1) * (c * (c - 2) * x + a * a)
        a3 = 2 * (n + a - 1) * (n - 1) * c
        p0, p1 = p1, (a2 * p1 - a3 * p0) / a1
    return p1


def psi_raw(etype: int, N: int, eta):
    """Unscaled basis values B[p, j] at points eta[p]."""
    eta = np.atleast_2d(np.asarray(eta, dtype=np.longdouble))
    a, b, c = eta[:, 0], eta[:, 1], eta[:, 2]
    ms = modes(etype, N)
    B = np.empty((eta.shape[0], len(ms)), dtype=np.longdouble)
    for j, (p, q, r) in enumerate(ms):
        if etype == TET:
            B[:, j] = (_jac(p, 0.0, a) * ((1 - b) / 2) ** p * _jac(q, 2 * p + 1.0, b)
                       * ((1 - c) / 2) ** (p + q) * _jac(r, 2 * p + 2 * q + 2.0, c))
        elif etype == PRISM:
            B[:, j] = (_jac(p, 0.0, a) * _jac(q, 0.0, b) * ((1 - c) / 2) ** p
                       * _jac(r, 2 * p + 1.0, c))
        else:
            m = max(p, q)
            B[:, j] = (_jac(p, 0.0, a) * _jac(q, 0.0, b) * ((1 - c) / 2) ** m
                       * _jac(r, 2 * m + 2.0, c))
    return B


def exact_rule(nq: int):
    """nq^3 Gauss-Legendre rule on the reference cube."""
    x, w = rules.gauss_legendre(nq)
    l, j, i = np.meshgrid(np.arange(nq), np.arange(nq), np.arange(nq), indexing="ij")
    eta = np.stack([x[i.ravel()], x[j.ravel()], x[l.ravel()]], axis=1)
    return eta, w[i.ravel()] * w[j.ravel()] * w[l.ravel()]


def reference_gram(etype: int, N: int, scaled=True):
    """Gram matrix of the basis in the reference-element L2 product (exact quadrature)."""
    eta, w = exact_rule(N + 3)
    J, _ = geometry.metrics(geometry.REF_CORNERS[etype], eta)
    B = psi(etype, N, eta) if scaled else psi_raw(etype, N, eta)
    return B.T @ (B * (w * J)[:, None])


_NORM_CACHE: dict = {}


def _norms(etype: int, N: int):
    key = (etype, N)
    if key not in _NORM_CACHE:
        eta, w = exact_rule(N + 3)
        J, _ = geometry.metrics(geometry.REF_CORNERS[etype], eta)
        B = psi_raw(etype, N, eta)
        _NORM_CACHE[key] = np.sqrt(np.einsum("pj,p->j", B * B, w * J))
    return _NORM_CACHE[key]


def psi(etype: int, N: int, eta):
    """Orthonormal basis values phi_j(eta_p)."""
    return psi_raw(etype, N, eta) / _norms(etype, N)[None, :]
