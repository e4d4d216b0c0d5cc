"""Element geometry: degenerate trilinear hexahedra, volume nodes, metrics (FP64).

Test infrastructure of the oracle.  Every element is x(eta) = sum_c N_c(eta) X_c over the
eight corners of the reference cube, with collapsed corners repeated (paper Sec. 2: the
mapping x = chi(xi) to the reference element, and the Duffy transform of prisms, pyramids
and tetrahedra to the unit hexahedron).  Metrics follow the contravariant form of Eq. (1):
J = det(dx/deta), a^a = dx/deta_{a+1} x dx/deta_{a+2} (= J grad_x eta_a).
"""
from __future__ import annotations

import numpy as np

from . import rules

HEX, PRISM, PYR, TET = 0, 1, 2, 3

# volume node families, 1-D rule per direction (eta1, eta2, eta3):
#   "R1"  Gauss-Lobatto where the direction does not collapse, left Gauss-Radau (contains -1,
#         omits the collapsed end +1) where it does; the discretisation of the hot path
#   "LG"  Gauss-Legendre in every direction (the Legendre-Gauss family of Sec. 2), kept to
#         measure what the R1 rules cost in accuracy on the collapsed types
NODE_FAMILIES = {
    "R1": {
        HEX: ("GL", "GL", "GL"),
        PRISM: ("GL", "GL", "LGR"),
        PYR: ("GL", "GL", "LGR"),
        TET: ("GL", "LGR", "LGR"),
    },
    "LG": {t: ("LG", "LG", "LG") for t in (HEX, PRISM, PYR, TET)},
}
NODE_RULES = NODE_FAMILIES["R1"]

# reference elements (xi space) as degenerate hexahedra; their L2 product defines the
# orthonormal modal bases
_T = {
    "t0": (-1, -1, -1), "t1": (1, -1, -1), "t2": (-1, 1, -1), "t3": (-1, -1, 1),
}
REF_CORNERS = {
    HEX: np.array([[2 * (c & 1) - 1, 2 * ((c >> 1) & 1) - 1, 2 * ((c >> 2) & 1) - 1]
                   for c in range(8)], dtype=float),
    # prism vertices v0..v5 with corners (v0, v1, v3, v4, v2, v2, v5, v5)
    PRISM: np.array([(-1, -1, -1), (1, -1, -1), (-1, 1, -1), (1, 1, -1),
                     (-1, -1, 1), (-1, -1, 1), (-1, 1, 1), (-1, 1, 1)], dtype=float),
    # pyramid base b0..b3 (lexicographic) and apex
    PYR: np.array([(-1, -1, -1), (1, -1, -1), (-1, 1, -1), (1, 1, -1),
                   (-1, -1, 1), (-1, -1, 1), (-1, -1, 1), (-1, -1, 1)], dtype=float),
    # tet corners (v0, v1, v2, v2, v3, v3, v3, v3)
    TET: np.array([_T["t0"], _T["t1"], _T["t2"], _T["t2"],
                   _T["t3"], _T["t3"], _T["t3"], _T["t3"]], dtype=float),
}


_RULE_CACHE: dict = {}


def node_rules(etype: int, n: int, family: str = "R1"):
    """1-D (nodes, weights) per direction; computed once per (type, n, family), returned as
    copies."""
    key = (int(etype), int(n), family)
    if key not in _RULE_CACHE:
        _RULE_CACHE[key] = [rules.RULES[name](n) for name in NODE_FAMILIES[family][etype]]
    return [(x.copy(), w.copy()) for x, w in _RULE_CACHE[key]]


def volume_nodes(etype: int, n: int, family: str = "R1"):
    """Tensor-product nodes eta[k] and weights w[k], k = i + n*j + n*n*l."""
    (x1, w1), (x2, w2), (x3, w3) = node_rules(etype, n, family)
    l, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    i, j, l = i.ravel(), j.ravel(), l.ravel()
    eta = np.stack([x1[i], x2[j], x3[l]], axis=1)
    w = w1[i] * w2[j] * w3[l]
    return eta, w  # long double


def lagrange3d(etype: int, n: int, eta, family: str = "R1"):
    """L[p, k] = l_k(eta_p): tensor-product Lagrange basis on the element's volume nodes."""
    eta = np.atleast_2d(eta)
    r = node_rules(etype, n, family)
    L1 = rules.lagrange_eval(r[0][0], eta[:, 0])
    L2 = rules.lagrange_eval(r[1][0], eta[:, 1])
    L3 = rules.lagrange_eval(r[2][0], eta[:, 2])
    out = np.einsum("pl,pj,pi->plji", L3, L2, L1)
    return out.reshape(eta.shape[0], n ** 3)


def lagrange3d_grad(etype: int, n: int, eta, family: str = "R1"):
    """G[p, k, a] = d l_k / d eta_a at eta_p."""
    eta = np.atleast_2d(eta)
    r = node_rules(etype, n, family)
    L = [rules.lagrange_eval(r[a][0], eta[:, a]) for a in range(3)]
    dL = [rules.lagrange_deriv_eval(r[a][0], eta[:, a]) for a in range(3)]
    P = eta.shape[0]
    G = np.empty((P, n ** 3, 3), dtype=np.result_type(eta, np.longdouble))
    G[:, :, 0] = np.einsum("pl,pj,pi->plji", L[2], L[1], dL[0]).reshape(P, -1)
    G[:, :, 1] = np.einsum("pl,pj,pi->plji", L[2], dL[1], L[0]).reshape(P, -1)
    G[:, :, 2] = np.einsum("pl,pj,pi->plji", dL[2], L[1], L[0]).reshape(P, -1)
    return G


def shape(eta):
    """Trilinear shape functions N[p, c] = prod_a (1 + s_a eta_a)/2, s_a = +-1 from bit a of c."""
    eta = np.atleast_2d(eta)
    out = np.ones((eta.shape[0], 8), dtype=eta.dtype)
    for c in range(8):
        for a in range(3):
            s = 1.0 if (c >> a) & 1 else -1.0
            out[:, c] *= 0.5 * (1.0 + s * eta[:, a])
    return out


def dshape(eta):
    """dN[p, c, a] = d N_c / d eta_a."""
    eta = np.atleast_2d(eta)
    out = np.ones((eta.shape[0], 8, 3), dtype=eta.dtype)
    for c in range(8):
        for a in range(3):
            for b in range(3):
                s = 1.0 if (c >> b) & 1 else -1.0
                if a == b:
                    out[:, c, a] *= 0.5 * s
                else:
                    out[:, c, a] *= 0.5 * (1.0 + s * eta[:, b])
    return out


def map_points(corners, eta):
    return shape(eta) @ corners


def jacobian(corners, eta):
    """X[p, c, a] = d x_c / d eta_a."""
    return np.einsum("pka,kc->pca", dshape(eta), corners)


def metrics(corners, eta):
    """J[p] = det(dx/deta) and contravariant vectors acon[p, a, :] = x_{eta_{a+1}} x x_{eta_{a+2}},
    evaluated in extended precision (long double) for the given FP64 corners."""
    ld = np.longdouble
    X = jacobian(np.asarray(corners, ld), np.asarray(eta, ld))
    cols = [X[:, :, a] for a in range(3)]
    acon = np.stack([np.cross(cols[1], cols[2]), np.cross(cols[2], cols[0]),
                     np.cross(cols[0], cols[1])], axis=1)
    J = np.einsum("pc,pc->p", cols[0], acon[:, 0, :])
    return J, acon


def inverse_map(corners, x, plane, tol=1e-15, maxit=60):
    """Reference coordinates of points x that lie on the face plane eta_a = +-1 of an element,
    plane = (a, side).  The two free coordinates are found by Gauss-Newton on x(eta) = x with
    eta_a held fixed; the face map is regular even where the element collapses (the collapsed
    edge of a prism lies on its side faces).  The iteration runs in extended precision
    (long double) on extended-precision points and returns long double coordinates."""
    ld = np.longdouble
    x = np.atleast_2d(np.asarray(x, dtype=ld))
    corners = np.asarray(corners, dtype=ld)
    a, side = plane
    free = [b for b in range(3) if b != a]
    eta = np.zeros(x.shape, dtype=ld)
    eta[:, a] = ld(1) if side else ld(-1)
    polish = 2  # iterations kept after the step drops below tol
    for _ in range(maxit):
        res = shape(eta) @ corners - x
        X = np.einsum("pka,kc->pca", dshape(eta), corners)[:, :, free]   # (P, 3, 2)
        A00 = np.einsum("pc,pc->p", X[:, :, 0], X[:, :, 0])
        A01 = np.einsum("pc,pc->p", X[:, :, 0], X[:, :, 1])
        A11 = np.einsum("pc,pc->p", X[:, :, 1], X[:, :, 1])
        g0 = np.einsum("pc,pc->p", X[:, :, 0], res)
        g1 = np.einsum("pc,pc->p", X[:, :, 1], res)
        det = A00 * A11 - A01 * A01
        d0 = (A11 * g0 - A01 * g1) / det
        d1 = (A00 * g1 - A01 * g0) / det
        eta[:, free[0]] -= d0
        eta[:, free[1]] -= d1
        if max(np.max(np.abs(d0)), np.max(np.abs(d1))) < tol:
            polish -= 1
            if polish < 0:
                break
    scale = max(1.0, float(np.max(np.abs(corners))))
    err = float(np.max(np.abs(shape(eta) @ corners - x)))
    if err > 1e-14 * scale:
        raise RuntimeError(f"inverse map did not converge (residual {err:.3e})")
    return eta
