"""Faces of a periodic mixed mesh: matching, canonical face points, per-side coordinates.

Test infrastructure of the oracle.  Elements couple only through the numerical flux on
shared faces (paper Sec. 3; Eq. (1) second term); faces may be non-conforming (Sec. 2).

Faces are found from shared global vertex-id sets: two element faces with the same id set
are a conforming face; a quadrilateral face left over is matched by the two triangles of
the neighbouring cell that cover it (a mortar), and each triangle half becomes a face of
its own on which the quadrilateral side evaluates its polynomial.

Face points are defined from vertex ids only, so periodic images agree:
  quad  A = smallest id, B and D its two edge neighbours (B < D);
        P(s,t) = A + (1+s)/2 (B-A) + (1+t)/2 (D-A), s,t on the Gauss-Lobatto points
  tri   A < B < C by id, collapse at C;
        P(s,t) = A (1-s)(1-t)/4 + B (1+s)(1-t)/4 + C (1+t)/2, s,t on the Gauss-Legendre points
Point p = i_s + n*i_t.  Weighted area elements ws_p = w_s w_t |dP/ds x dP/dt| and the unit
normal are taken from the face geometry of side L (the smaller element index) and the
normal points from L to R.  Each side's reference coordinates eta of the points come from
inverting that element's own map.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import geometry, rules


@dataclasses.dataclass
class Face:
    kind: str              # "quad" or "tri"
    ids: tuple             # canonical vertex ids (A, B, D) or (A, B, C)
    eL: int
    eR: int
    planeL: tuple          # (axis, side) of the face in each element's reference cube
    planeR: tuple
    mortar: bool
    # geometry (filled by FaceGeometry)
    normal: np.ndarray = None
    ws: np.ndarray = None
    etaL: np.ndarray = None
    etaR: np.ndarray = None


def element_planes(corner_ids):
    """Faces of one element: list of (axis, side, slots[2][2], distinct id count)."""
    out = []
    for a in range(3):
        b, c = [x for x in range(3) if x != a]
        for s in range(2):
            slots = np.empty((2, 2), dtype=int)
            for u in range(2):
                for v in range(2):
                    slots[u, v] = (s << a) | (u << b) | (v << c)
            ids = {int(corner_ids[k]) for k in slots.ravel()}
            if len(ids) >= 3:
                out.append((a, s, slots, len(ids)))
    return out


def build_faces(mesh):
    """Match element faces of a periodic mesh; returns the list of Face records."""
    quads, tris = {}, {}
    plane_info = {}
    for e in range(mesh.n_elems):
        cid = mesh.elem_corner[e]
        for (a, s, slots, nd) in element_planes(cid):
            key = frozenset(int(cid[k]) for k in slots.ravel())
            plane_info[(e, a, s)] = slots
            (quads if nd == 4 else tris).setdefault(key, []).append((e, (a, s)))
    faces = []

    def quad_frame(e, plane, key):
        slots = plane_info[(e,) + plane]
        cid = mesh.elem_corner[e]
        pos = {int(cid[slots[u, v]]): (u, v) for u in range(2) for v in range(2)}
        A = min(key)
        u, v = pos[A]
        nb = sorted([int(cid[slots[1 - u, v]]), int(cid[slots[u, 1 - v]])])
        return (A, nb[0], nb[1])

    leftover_quads = []
    for key, sides in quads.items():
        if len(sides) == 2:
            (e0, p0), (e1, p1) = sorted(sides)
            faces.append(Face("quad", quad_frame(e0, p0, key), e0, e1, p0, p1, False))
        elif len(sides) == 1:
            leftover_quads.append((key, sides[0]))
        else:
            raise ValueError("non-manifold quadrilateral face")
    used_tris = set()
    for key, sides in tris.items():
        if len(sides) == 2:
            (e0, p0), (e1, p1) = sorted(sides)
            faces.append(Face("tri", tuple(sorted(key)), e0, e1, p0, p1, False))
            used_tris.add(key)
        elif len(sides) > 2:
            raise ValueError("non-manifold triangular face")
    for key, (eq, pq) in leftover_quads:
        ids = sorted(key)
        halves = []
        for drop in ids:
            tk = frozenset(i for i in ids if i != drop)
            if tk in tris and len(tris[tk]) == 1 and tk not in used_tris:
                halves.append(tk)
        if len(halves) != 2 or len(halves[0] | halves[1]) != 4:
            raise ValueError("unmatched quadrilateral face")
        for tk in halves:
            et, pt = tris[tk][0]
            used_tris.add(tk)
            (e0, p0), (e1, p1) = sorted([(eq, pq), (et, pt)])
            faces.append(Face("tri", tuple(sorted(tk)), e0, e1, p0, p1, True))
    for key, sides in tris.items():
        if key not in used_tris:
            raise ValueError("unmatched triangular face")
    return faces


def face_rule(kind: str, n: int):
    """Canonical parameters (s, t) and weights of the face points."""
    x, w = (rules.gauss_lobatto(n) if kind == "quad" else rules.gauss_legendre(n))
    it, is_ = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    s, t = x[is_.ravel()], x[it.ravel()]
    return s, t, w[is_.ravel()] * w[it.ravel()]


def _vertex_xyz(mesh, e, vid):
    k = int(np.nonzero(mesh.elem_corner[e] == vid)[0][0])
    return mesh.corner_xyz[e, k]


def face_points(kind, XA, XB, XC, s, t):
    """Physical points and |dP/ds x dP/dt| of the canonical parametrisation (in the precision of
    the inputs)."""
    if kind == "quad":
        P = XA[None] + ((1 + s) / 2)[:, None] * (XB - XA)[None] + ((1 + t) / 2)[:, None] * (XC - XA)[None]
        dPs = np.broadcast_to((XB - XA) / 2, P.shape)
        dPt = np.broadcast_to((XC - XA) / 2, P.shape)
    else:
        a = ((1 - s) * (1 - t) / 4)[:, None]
        b = ((1 + s) * (1 - t) / 4)[:, None]
        c = ((1 + t) / 2)[:, None]
        P = a * XA[None] + b * XB[None] + c * XC[None]
        dPs = ((1 - t) / 4)[:, None] * (XB - XA)[None]
        dPt = (-(1 - s) / 4)[:, None] * XA[None] - ((1 + s) / 4)[:, None] * XB[None] + 0.5 * XC[None]
    jac = np.linalg.norm(np.cross(dPs, dPt), axis=1)
    return P, jac


def face_geometry(mesh, f: Face, n: int):
    """Fill normal, ws, etaL, etaR of a face."""
    s, t, wq = face_rule(f.kind, n)
    ld = np.longdouble
    XL = [_vertex_xyz(mesh, f.eL, v) for v in f.ids]
    _, jac = face_points(f.kind, XL[0], XL[1], XL[2], s, t)
    # face points in extended precision for the inversion of each side's map
    P_L, _ = face_points(f.kind, *[np.asarray(X, ld) for X in XL], np.asarray(s, ld), np.asarray(t, ld))
    nrm = np.cross(XL[1] - XL[0], XL[2] - XL[0])
    nrm = nrm / np.linalg.norm(nrm)
    # orient from L to R: away from L's centroid
    cL = mesh.corner_xyz[f.eL].mean(axis=0)
    if np.dot(np.asarray(P_L.mean(axis=0), np.float64) - cL, nrm) < 0:
        nrm = -nrm
    f.normal = nrm
    f.ws = wq * jac
    f.etaL = geometry.inverse_map(mesh.corner_xyz[f.eL], P_L, f.planeL)
    XR = [_vertex_xyz(mesh, f.eR, v) for v in f.ids]
    P_R, _ = face_points(f.kind, *[np.asarray(X, ld) for X in XR], np.asarray(s, ld), np.asarray(t, ld))
    f.etaR = geometry.inverse_map(mesh.corner_xyz[f.eR], P_R, f.planeR)
    return f
