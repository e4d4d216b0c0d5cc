"""Faces of a periodic mixed mesh: matching, canonical face points, per-side coordinates.

Test infrastructure of the oracle.  Elements couple only through the numerical flux on
shared faces (paper Sec. 3; Eq. (1) second term); faces may be non-conforming (Sec. 2).

Faces are found from shared global vertex-id sets: two element faces with the same id set
are a conforming face; a quadrilateral face left over is matched by the two triangles of
the neighbouring cell that cover it (a mortar), and each triangle half becomes a face of
its own on which the quadrilateral side evaluates its polynomial.

Mortar faces: each triangle half is integrated with a collapsed Gauss rule of ms x mt points,
exact to total degree 3N on the half (3N - 1 at N = 6), because the quadrilateral side
integrates its degree-N-per-direction test functions times the flux there: the triangle's own
n x n rule is exact only for constant fluxes on that side, which keeps free stream and
conservation but costs consistency.  The ms * mt <= 2 n^2 points are split into two chunks of
n^2 points (zero-weight padding at the half's centre point s = t = 0), and each chunk is a face
of its own, so every face carries n^2 points.

Face points are defined from vertex ids only, so periodic images agree:
  quad  A = smallest id, B and D its two edge neighbours (B < D);
        P(s,t) = A + (1+s)/2 (B-A) + (1+t)/2 (D-A), s,t on the Gauss-Lobatto points
        (Gauss-Legendre points with the "LG" volume node family)
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
    chunk: int = -1        # mortar halves: which n^2-point chunk of the rich rule (0 or 1)
    # geometry (filled by FaceGeometry)
    normal: np.ndarray = None
    ws: np.ndarray = None
    etaL: np.ndarray = None
    etaR: np.ndarray = None


def element_planes(corner_ids):  # per-element form, kept for reference and tests
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


def _plane_slot_table():
    """slots[plane][u][v] of the six reference-cube faces, plane = 2*axis + side."""
    out = np.empty((6, 2, 2), dtype=int)
    for a in range(3):
        b, c = [x for x in range(3) if x != a]
        for s in range(2):
            for u in range(2):
                for v in range(2):
                    out[2 * a + s, u, v] = (s << a) | (u << b) | (v << c)
    return out


PLANE_SLOTS = _plane_slot_table()


class FaceTable:
    """Matched faces as arrays; face(i) / table[i] returns a Face record (cached)."""

    def __init__(self, kind, ids, eL, eR, pL, pR, mortar, chunk):
        self.kind, self.ids, self.eL, self.eR = kind, ids, eL, eR
        self.pL, self.pR, self.mortar, self.chunk = pL, pR, mortar, chunk
        self._cache = {}

    def __len__(self):
        return int(self.eL.shape[0])

    def __getitem__(self, i):
        f = self._cache.get(i)
        if f is None:
            i = int(i)
            f = Face("quad" if self.kind[i] == 0 else "tri", tuple(int(v) for v in self.ids[i]),
                     int(self.eL[i]), int(self.eR[i]), (int(self.pL[i]) >> 1, int(self.pL[i]) & 1),
                     (int(self.pR[i]) >> 1, int(self.pR[i]) & 1), bool(self.mortar[i]), int(self.chunk[i]))
            self._cache[i] = f
        return f

    def __iter__(self):
        for i in range(len(self)):
            yield self[i]


def build_faces(mesh):
    """Match element faces of a periodic mesh (vectorised over elements).

    Records (element, plane) with at least three distinct vertex ids are grouped by their
    sorted id set; groups of two are conforming faces (kind 0 quad, 1 triangle), a lone
    quadrilateral is matched with the two lone triangles whose id sets it contains.
    L is the smaller element index of each face."""
    ne = mesh.n_elems
    cid = np.asarray(mesh.elem_corner, dtype=np.int64)
    rec_e, rec_p, rec_ids, rec_nd = [], [], [], []
    for plane in range(6):
        ids = cid[:, PLANE_SLOTS[plane].ravel()]            # (ne, 4) in slot (u, v) order
        srt = np.sort(ids, axis=1)
        nd = 1 + (np.diff(srt, axis=1) != 0).sum(axis=1)
        keep = nd >= 3
        # unique ids padded with -1 (triangles)
        dup = np.concatenate([np.zeros((ne, 1), bool), np.diff(srt, axis=1) == 0], axis=1)
        srt_u = np.where(dup, np.iinfo(np.int64).max, srt)
        srt_u = np.sort(srt_u, axis=1)
        key = np.where(srt_u == np.iinfo(np.int64).max, -1, srt_u)
        rec_e.append(np.nonzero(keep)[0])
        rec_p.append(np.full(int(keep.sum()), plane))
        rec_ids.append(key[keep])
        rec_nd.append(nd[keep])
    rec_e = np.concatenate(rec_e)
    rec_p = np.concatenate(rec_p)
    rec_ids = np.concatenate(rec_ids)
    rec_nd = np.concatenate(rec_nd)
    order = np.lexsort((rec_p, rec_e, rec_ids[:, 3], rec_ids[:, 2], rec_ids[:, 1], rec_ids[:, 0], rec_nd))
    rec_e, rec_p, rec_ids, rec_nd = rec_e[order], rec_p[order], rec_ids[order], rec_nd[order]
    same = np.all(rec_ids[1:] == rec_ids[:-1], axis=1) & (rec_nd[1:] == rec_nd[:-1])
    start = np.concatenate([[True], ~same])
    gid = np.cumsum(start) - 1
    gsize = np.bincount(gid)
    if gsize.max() > 2:
        raise ValueError("non-manifold face")
    first = np.nonzero(start)[0]
    pair = first[gsize == 2]
    # conforming faces: records pair, pair+1 (sorted by element, so L = smaller element)
    c_e0, c_e1 = rec_e[pair], rec_e[pair + 1]
    c_p0, c_p1 = rec_p[pair], rec_p[pair + 1]
    c_nd = rec_nd[pair]
    c_ids = rec_ids[pair].copy()
    # canonical quad frame: A = min id, B < D its two edge neighbours in L's plane grid
    q = c_nd == 4
    if q.any():
        grid = cid[c_e0[q][:, None], PLANE_SLOTS[c_p0[q]].reshape(-1, 4)]    # (nq, 4), idx = 2u + v
        ia = np.argmin(grid, axis=1)
        u, v = ia // 2, ia % 2
        nb1 = grid[np.arange(grid.shape[0]), (1 - u) * 2 + v]
        nb2 = grid[np.arange(grid.shape[0]), u * 2 + (1 - v)]
        c_ids[q, 0] = grid.min(axis=1)
        c_ids[q, 1] = np.minimum(nb1, nb2)
        c_ids[q, 2] = np.maximum(nb1, nb2)
        c_ids[q, 3] = -1
    kind = [np.where(c_nd == 4, 0, 1)]
    ids = [c_ids[:, :3]]
    eL, eR, pL, pR, mort = [c_e0], [c_e1], [c_p0], [c_p1], [np.zeros(c_e0.size, bool)]
    chunk = [np.full(c_e0.size, -1)]
    # mortars: lone quadrilaterals covered by two lone triangles
    lone = first[gsize == 1]
    lq = lone[rec_nd[lone] == 4]
    lt = lone[rec_nd[lone] == 3]
    tri_index = {tuple(rec_ids[r, :3]): r for r in lt}
    used = set()
    m_e0, m_e1, m_p0, m_p1, m_ids, m_chunk = [], [], [], [], [], []
    for r in lq:
        qi = rec_ids[r]
        halves = []
        for drop in range(4):
            tk = tuple(int(qi[j]) for j in range(4) if j != drop)
            tr = tri_index.get(tk)
            if tr is not None and tr not in used:
                halves.append(tr)
        if len(halves) != 2 or len(set(rec_ids[halves[0], :3]) | set(rec_ids[halves[1], :3])) != 4:
            raise ValueError("unmatched quadrilateral face")
        for tr in halves:
            used.add(tr)
            (e0, p0), (e1, p1) = sorted([(int(rec_e[r]), int(rec_p[r])), (int(rec_e[tr]), int(rec_p[tr]))])
            for ch in (0, 1):   # the two n^2-point chunks of the half's rich rule
                m_e0.append(e0); m_e1.append(e1); m_p0.append(p0); m_p1.append(p1)
                m_ids.append(rec_ids[tr, :3])
                m_chunk.append(ch)
    if len(used) != len(lt):
        raise ValueError("unmatched triangular face")
    if m_e0:
        kind.append(np.ones(len(m_e0), int))
        ids.append(np.array(m_ids))
        eL.append(np.array(m_e0)); eR.append(np.array(m_e1))
        pL.append(np.array(m_p0)); pR.append(np.array(m_p1))
        mort.append(np.ones(len(m_e0), bool))
        chunk.append(np.array(m_chunk))
    return FaceTable(np.concatenate(kind), np.concatenate(ids), np.concatenate(eL), np.concatenate(eR),
                     np.concatenate(pL), np.concatenate(pR), np.concatenate(mort), np.concatenate(chunk))


def mortar_rule_size(n: int):
    """(ms, mt): Gauss-Legendre points in s and in t of the collapsed rule on a mortar half, the
    fewest that integrate total degree D = 3N exactly (s-degree D, t-degree D + 1 with the
    collapse factor), D = 3N - 1 at N = 6, so that ms * mt <= 2 n^2."""
    N = n - 1
    D = 3 * N if N <= 5 else 3 * N - 1
    ms, mt = (D + 2) // 2, (D + 3) // 2
    assert ms * mt <= 2 * n * n
    return ms, mt


def face_rule(kind: str, n: int, family: str = "R1", chunk: int = -1):
    """Canonical parameters (s, t) and weights of the face points (a triangle's weights exclude
    the collapse factor, which face_points' area element carries).  chunk >= 0: that chunk of
    n^2 points of a mortar half's rich rule."""
    if chunk >= 0:
        ms, mt = mortar_rule_size(n)
        xs, ws = rules.gauss_legendre(ms)
        xt, wt = rules.gauss_legendre(mt)
        jt, js = np.meshgrid(np.arange(mt), np.arange(ms), indexing="ij")
        s, t, w = xs[js.ravel()], xt[jt.ravel()], ws[js.ravel()] * wt[jt.ravel()]
        n2 = n * n
        pad = 2 * n2 - s.size
        zero = np.zeros(pad, dtype=s.dtype)
        s, t, w = np.concatenate([s, zero]), np.concatenate([t, zero]), np.concatenate([w, zero])
        sl = slice(chunk * n2, (chunk + 1) * n2)
        return s[sl], t[sl], w[sl]
    x, w = (rules.gauss_lobatto(n) if kind == "quad" and family == "R1" else rules.gauss_legendre(n))
    it, is_ = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    s, t = x[is_.ravel()], x[it.ravel()]
    return s, t, w[is_.ravel()] * w[it.ravel()]


def _vertex_xyz(mesh, e, vid):
    k = int(np.nonzero(mesh.elem_corner[e] == vid)[0][0])
    return mesh.corner_xyz[e, k]


def face_points(kind, XA, XB, XC, s, t, X4=None):
    """Physical points, dP/ds x dP/dt and its length, of the canonical parametrisation (in the
    precision of the inputs).  Quadrilaterals are the bilinear patch of A (s, t = -1, -1),
    B (+1, -1), D = XC (-1, +1) and the corner X4 opposite A (+1, +1); without X4 the
    parallelogram (X4 = B + D - A)."""
    if kind == "quad":
        if X4 is None:
            X4 = XB + XC - XA
        a = ((1 - s) * (1 - t) / 4)[:, None]
        b = ((1 + s) * (1 - t) / 4)[:, None]
        c = ((1 - s) * (1 + t) / 4)[:, None]
        d = ((1 + s) * (1 + t) / 4)[:, None]
        P = a * XA[None] + b * XB[None] + c * XC[None] + d * X4[None]
        dPs = ((1 - t) / 4)[:, None] * (XB - XA)[None] + ((1 + t) / 4)[:, None] * (X4 - XC)[None]
        dPt = ((1 - s) / 4)[:, None] * (XC - XA)[None] + ((1 + s) / 4)[:, None] * (X4 - XB)[None]
    else:
        a = ((1 - s) * (1 - t) / 4)[:, None]
        b = ((1 + s) * (1 - t) / 4)[:, None]
        c = ((1 + t) / 2)[:, None]
        P = a * XA[None] + b * XB[None] + c * XC[None]
        dPs = ((1 - t) / 4)[:, None] * (XB - XA)[None]
        dPt = (-(1 - s) / 4)[:, None] * XA[None] - ((1 + s) / 4)[:, None] * XB[None] + 0.5 * XC[None]
    nv = np.cross(dPs, dPt)
    return P, nv, np.linalg.norm(nv, axis=1)


def _quad_fourth(mesh, e, plane, ids):
    """The vertex of element e's face `plane` that is not among the canonical ids (A, B, D)."""
    a, side = plane
    slots = PLANE_SLOTS[2 * a + side].ravel()
    rest = [int(v) for v in mesh.elem_corner[e][slots] if int(v) not in ids]
    return rest[0]


def face_geometry(mesh, f: Face, n: int, family: str = "R1"):
    """Fill normal ([3][P], per face point: quadrilaterals may be bilinear, not flat), ws, etaL,
    etaR of a face."""
    s, t, wq = face_rule(f.kind, n, family, f.chunk)
    ld = np.longdouble
    quad = f.kind == "quad"
    X4L = _vertex_xyz(mesh, f.eL, _quad_fourth(mesh, f.eL, f.planeL, f.ids)) if quad else None
    XL = [_vertex_xyz(mesh, f.eL, v) for v in f.ids]
    _, nv, jac = face_points(f.kind, XL[0], XL[1], XL[2], s, t, X4L)
    # face points in extended precision for the inversion of each side's map
    P_L, _, _ = face_points(f.kind, *[np.asarray(X, ld) for X in XL], np.asarray(s, ld), np.asarray(t, ld),
                            None if X4L is None else np.asarray(X4L, ld))
    nrm = nv / jac[:, None]
    # orient from L to R: away from L's centroid
    cL = mesh.corner_xyz[f.eL].mean(axis=0)
    if np.dot(np.asarray(P_L.mean(axis=0), np.float64) - cL, nrm.mean(axis=0)) < 0:
        nrm = -nrm
    f.normal = np.ascontiguousarray(nrm.T)
    f.ws = wq * jac
    f.etaL = geometry.inverse_map(mesh.corner_xyz[f.eL], P_L, f.planeL)
    XR = [_vertex_xyz(mesh, f.eR, v) for v in f.ids]
    X4R = _vertex_xyz(mesh, f.eR, _quad_fourth(mesh, f.eR, f.planeR, f.ids)) if quad else None
    P_R, _, _ = face_points(f.kind, *[np.asarray(X, ld) for X in XR], np.asarray(s, ld), np.asarray(t, ld),
                            None if X4R is None else np.asarray(X4R, ld))
    f.etaR = geometry.inverse_map(mesh.corner_xyz[f.eR], P_R, f.planeR)
    return f
