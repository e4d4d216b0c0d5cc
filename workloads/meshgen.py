"""Periodic mixed hex/prism/pyramid/tet meshes built by splitting the cells of a cube.

Every element is described as a degenerate trilinear hexahedron: eight corners in
lexicographic order c = i + 2j + 4k of the reference cube [-1,1]^3, where collapsed
corners repeat a vertex.  The collapse patterns are

    hex      (c0..c7)                      all distinct
    prism    (v0, v1, v3, v4, v2, v2, v5, v5)   triangle (v0,v1,v2) extruded to (v3,v4,v5)
    pyramid  (b0, b1, b2, b3, a, a, a, a)    base listed lexicographically, apex a
    tet      (v0, v1, v2, v2, v3, v3, v3, v3)

so that the mapping from the reference cube is a collapsed-coordinate (Duffy)
transform followed by an affine map (paper Sec. 2, Duffy transform to the unit
hexahedron).  Cells are split as in the paper's mixed meshes (Sec. 4: hexahedra
split into prisms, pyramids and tetrahedra):

    hex-split      one hexahedron
    prism-split    two prisms, cut by the plane x = y through the cell's min/max corner
    pyramid-split  six pyramids, one per cell face, apex at the cell centre
    tet-split      six Kuhn tetrahedra  0 <= x_s1 <= x_s2 <= x_s3 <= 1

All cut diagonals of cell faces pass through the face's min and max corner, so
triangulated faces of neighbouring cells agree.

Global vertex ids identify periodic images; cell centres get ids after the grid
vertices.  Coordinates are unwrapped per element (each element's corners lie in
one cell), so geometry is periodic-safe.
"""
from __future__ import annotations

import dataclasses
import itertools
import math

import numpy as np

HEX, PRISM, PYR, TET = 0, 1, 2, 3
TYPE_NAMES = ("hex", "prism", "pyramid", "tet")

# cell split kinds share the numbering of the element types they produce
SPLIT_HEX, SPLIT_PRISM, SPLIT_PYR, SPLIT_TET = HEX, PRISM, PYR, TET

CENTER = 8  # local point index of the cell centre (0..7 are the cube corners)


def _local_xyz(lp):
    if lp == CENTER:
        return np.array([0.5, 0.5, 0.5])
    return np.array([lp & 1, (lp >> 1) & 1, (lp >> 2) & 1], dtype=float)


def _det_cols(a, b, c):
    return float(np.linalg.det(np.stack([a, b, c], axis=1)))


def _orient_prism(v):
    v0, v1, v2, v3, v4, v5 = v
    x = [_local_xyz(p) for p in v]
    if _det_cols(x[1] - x[0], x[3] - x[0], x[2] - x[0]) < 0:
        v0, v1, v3, v4 = v1, v0, v4, v3
    return [v0, v1, v3, v4, v2, v2, v5, v5]


def _orient_pyr(b):
    b0, b1, b2, b3 = b
    x0, x1, x2 = _local_xyz(b0), _local_xyz(b1), _local_xyz(b2)
    if _det_cols(x1 - x0, x2 - x0, _local_xyz(CENTER) - x0) < 0:
        b1, b2 = b2, b1
    return [b0, b1, b2, b3, CENTER, CENTER, CENTER, CENTER]


def _orient_tet(v):
    v0, v1, v2, v3 = v
    x = [_local_xyz(p) for p in v]
    if _det_cols(x[1] - x[0], x[2] - x[0], x[3] - x[0]) < 0:
        v0, v1 = v1, v0
    return [v0, v1, v2, v2, v3, v3, v3, v3]


def _split_table():
    """Per split kind: list of (element type, 8 local point indices)."""
    tab = {SPLIT_HEX: [(HEX, list(range(8)))]}
    # prisms: triangles (0,0)-(1,0)-(1,1) and (0,0)-(1,1)-(0,1) of the bottom face, extruded in z
    tab[SPLIT_PRISM] = [
        (PRISM, _orient_prism([0, 1, 3, 4, 5, 7])),
        (PRISM, _orient_prism([0, 3, 2, 4, 7, 6])),
    ]
    pyr = []
    for axis in range(3):
        for side in range(2):
            base = [c for c in range(8) if ((c >> axis) & 1) == side]  # lexicographic order
            pyr.append((PYR, _orient_pyr(base)))
    tab[SPLIT_PYR] = pyr
    tet = []
    for s in itertools.permutations(range(3)):
        v1 = 1 << s[2]
        v2 = v1 | (1 << s[1])
        tet.append((TET, _orient_tet([0, v1, v2, 7])))
    tab[SPLIT_TET] = tet
    return tab


SPLITS = _split_table()
ELEMS_PER_SPLIT = {k: len(v) for k, v in SPLITS.items()}


@dataclasses.dataclass
class Mesh:
    """Mesh tables in generator element order (cell-major)."""
    L: float
    C: int
    cell_kind: np.ndarray      # int8 [C^3]
    elem_type: np.ndarray      # int8 [n_elems]
    elem_cell: np.ndarray      # int32 [n_elems]
    elem_corner: np.ndarray    # int32 [n_elems, 8] global vertex ids
    corner_xyz: np.ndarray     # float64 [n_elems, 8, 3] unwrapped coordinates
    centroid: np.ndarray       # float64 [n_elems, 3] mean of the distinct vertices
    n_vertices: int

    @property
    def n_elems(self):
        return int(self.elem_type.shape[0])

    @property
    def h(self):
        return self.L / self.C

    def type_counts(self):
        return np.bincount(self.elem_type, minlength=4)


def make_mesh(C: int, cell_kind: np.ndarray, L: float = 2.0 * math.pi) -> Mesh:
    """Build the element tables of a periodic C^3-cell cube whose cells are split by `cell_kind`."""
    if C < 3:
        raise ValueError("periodic vertex-id matching needs at least 3 cells per direction")
    cell_kind = np.asarray(cell_kind, dtype=np.int8).reshape(-1)
    assert cell_kind.shape[0] == C ** 3
    h = L / C
    n_cells = C ** 3
    cells = np.arange(n_cells, dtype=np.int64)
    ci, cj, ck = cells % C, (cells // C) % C, cells // (C * C)
    origin = np.stack([ci, cj, ck], axis=1).astype(np.float64) * h

    # local point -> global id / coordinate, for all cells: shape [n_cells, 9]
    gid = np.empty((n_cells, 9), dtype=np.int64)
    lxyz = np.stack([_local_xyz(p) for p in range(9)])  # [9,3]
    for p in range(8):
        a, b, c = p & 1, (p >> 1) & 1, (p >> 2) & 1
        gid[:, p] = (ci + a) % C + C * (((cj + b) % C) + C * ((ck + c) % C))
    gid[:, CENTER] = n_cells + cells

    counts = np.array([ELEMS_PER_SPLIT[int(k)] for k in range(4)])
    per_cell = counts[cell_kind]
    n_elems = int(per_cell.sum())
    elem_type = np.empty(n_elems, dtype=np.int8)
    elem_cell = np.empty(n_elems, dtype=np.int32)
    elem_lp = np.empty((n_elems, 8), dtype=np.int64)
    first = np.concatenate([[0], np.cumsum(per_cell)[:-1]])
    for kind in range(4):
        sel = np.nonzero(cell_kind == kind)[0]
        if sel.size == 0:
            continue
        for j, (etype, lps) in enumerate(SPLITS[kind]):
            idx = first[sel] + j
            elem_type[idx] = etype
            elem_cell[idx] = sel
            elem_lp[idx] = np.array(lps)
    cell_of = elem_cell.astype(np.int64)
    elem_corner = np.take_along_axis(gid[cell_of], elem_lp, axis=1).astype(np.int32)
    corner_xyz = origin[cell_of][:, None, :] + h * lxyz[elem_lp]
    # centroid: mean of the distinct vertices of each element
    nd = np.array([8, 6, 5, 4])[elem_type]
    cen = np.zeros((n_elems, 3))
    for t, pick in ((HEX, range(8)), (PRISM, (0, 1, 4, 2, 3, 6)), (PYR, (0, 1, 2, 3, 4)), (TET, (0, 1, 2, 4))):
        m = elem_type == t
        if m.any():
            cen[m] = corner_xyz[m][:, list(pick), :].sum(axis=1) / len(pick)
    assert np.all(nd > 0)
    return Mesh(L=L, C=C, cell_kind=cell_kind, elem_type=elem_type, elem_cell=elem_cell,
                elem_corner=elem_corner, corner_xyz=corner_xyz, centroid=cen,
                n_vertices=2 * n_cells)


def deformed(mesh: Mesh, amp: float) -> Mesh:
    """The same mesh with every vertex moved by amp * h * (sin ky sin kz, sin kz sin kx,
    sin kx sin ky), k = 2 pi / L (periodic, so images of a vertex move alike): hexahedra become
    trilinear, quadrilateral faces bilinear (not flat) and triangles stay flat.  Meant for meshes
    without quadrilateral-triangle interfaces (a curved quadrilateral has no straight diagonal)."""
    k = 2.0 * math.pi / mesh.L
    h = mesh.L / mesh.C
    x, y, z = mesh.corner_xyz[..., 0], mesh.corner_xyz[..., 1], mesh.corner_xyz[..., 2]
    d = np.stack([np.sin(k * y) * np.sin(k * z), np.sin(k * z) * np.sin(k * x),
                  np.sin(k * x) * np.sin(k * y)], axis=-1)
    xyz = mesh.corner_xyz + amp * h * d
    cen = np.zeros_like(mesh.centroid)
    for t, pick in ((HEX, range(8)), (PRISM, (0, 1, 4, 2, 3, 6)), (PYR, (0, 1, 2, 3, 4)), (TET, (0, 1, 2, 4))):
        m = mesh.elem_type == t
        if m.any():
            cen[m] = xyz[m][:, list(pick), :].sum(axis=1) / len(pick)
    return dataclasses.replace(mesh, corner_xyz=xyz, centroid=cen)


def motion(mesh: Mesh, amp: float) -> np.ndarray:
    """Corner displacements d [n_elems][8][3] of a mesh motion x(t) = x0 + d sin(omega t):
    amp * h * (sin k(y+z), sin k(z+x), sin k(x+y)), k = 2 pi / L, at each corner's position x0
    (periodic, so images of a vertex move alike)."""
    k = 2.0 * math.pi / mesh.L
    h = mesh.L / mesh.C
    x, y, z = mesh.corner_xyz[..., 0], mesh.corner_xyz[..., 1], mesh.corner_xyz[..., 2]
    return amp * h * np.stack([np.sin(k * (y + z)), np.sin(k * (z + x)), np.sin(k * (x + y))], axis=-1)


# ---------------------------------------------------------------------------------------------
# cell-type placement for the five workloads
# ---------------------------------------------------------------------------------------------

def _kinds_from_counts(rng, n, counts):
    kinds = np.empty(n, dtype=np.int8)
    perm = rng.permutation(n)
    off = 0
    for k, c in enumerate(counts):
        kinds[perm[off:off + c]] = k
        off += c
    assert off == n
    return kinds


def cell_kinds_config(cfg: int, seed: int = 0, C: int | None = None):
    """Seeded cell split kinds of workload `cfg` (1, 2, 4 or 5)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if cfg == 1:
        C = 4 if C is None else C
        n = C ** 3
        counts = [n // 2, n // 4, n // 8, n - n // 2 - n // 4 - n // 8]
        return C, _kinds_from_counts(rng, n, counts)
    if cfg == 2:
        C = 48 if C is None else C
        B = 4
        nb = C // B
        blocks = _kinds_from_counts(rng, nb ** 3, [nb ** 3 // 4] * 4)
        cells = np.arange(C ** 3)
        ci, cj, ck = cells % C, (cells // C) % C, cells // (C * C)
        bid = ci // B + nb * ((cj // B) + nb * (ck // B))
        return C, blocks[bid].astype(np.int8)
    if cfg == 4:
        C = 24 if C is None else C
        n = C ** 3
        return C, _kinds_from_counts(rng, n, [n // 4] * 4)
    if cfg == 5:
        C = 64 if C is None else C
        n = C ** 3
        centre = rng.uniform(0.3, 0.7, size=3)  # in units of L
        cells = np.arange(n)
        cc = (np.stack([cells % C, (cells // C) % C, cells // (C * C)], axis=1) + 0.5) / C
        inside = np.linalg.norm(cc - centre, axis=1) < 0.3
        p_in = np.array([1, 1, 1, 27]) / 30.0     # 90 % tet-split, rest equally
        p_out = np.array([27, 1, 1, 1]) / 30.0    # 90 % hex, rest equally
        u = rng.uniform(size=n)
        cdf_in, cdf_out = np.cumsum(p_in), np.cumsum(p_out)
        k_in = np.searchsorted(cdf_in, u, side="right")
        k_out = np.searchsorted(cdf_out, u, side="right")
        kinds = np.where(inside, k_in, k_out).clip(0, 3).astype(np.int8)
        return C, kinds
    raise ValueError(f"no cell placement for workload {cfg}")


def config_mesh(cfg: int, seed: int = 0, C: int | None = None) -> Mesh:
    C, kinds = cell_kinds_config(cfg, seed, C)
    return make_mesh(C, kinds)


CONFIGS = {
    1: dict(name="euler_mixed_4c_N3", C=4, N=3, equations="euler", steps=10, cfl=0.5),
    2: dict(name="ns_mixed_48c_N4", C=48, N=4, equations="ns", steps=100, cfl=0.5),
    3: dict(name="euler_batched_64meshes", C=None, N=None, equations="euler", steps=50, cfl=0.5),
    4: dict(name="ns_mixed_24c_N3_adjoint", C=24, N=3, equations="ns", steps=20, cfl=0.5),
    5: dict(name="ns_sphere_64c_N5", C=64, N=5, equations="ns", steps=50, cfl=0.5),
}


def config_params(cfg: int):
    c = dict(CONFIGS[cfg])
    c.update(gamma=1.4, mu=1.0 / 1600.0, Pr=0.71, R=1.0, mach=0.1)
    return c


def batched_configs(n_meshes: int = 64, seed: int = 0, max_edge: int = 32, min_edge: int = 8):
    """Per-mesh (edge, N, cell kinds) of the batched workload: edge ~ U{min_edge..max_edge},
    type fractions ~ Dirichlet(1,1,1,1), N ~ U{2..6}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n_meshes):
        C = int(rng.integers(min_edge, max_edge + 1))
        frac = rng.dirichlet(np.ones(4))
        N = int(rng.integers(2, 7))
        kinds = rng.choice(4, size=C ** 3, p=frac).astype(np.int8)
        out.append(dict(index=i, C=C, N=N, fractions=frac, kinds=kinds))
    return out


# ---------------------------------------------------------------------------------------------
# initial state inputs
# ---------------------------------------------------------------------------------------------

def tgv_primitive(x, y, z, gamma=1.4, mach=0.1, xp=np):
    """Taylor-Green initial field: rho = 1, u = sin x cos y cos z, v = -cos x sin y cos z,
    w = 0, p = 1/(gamma Ma^2) + (cos 2x + cos 2y)(cos 2z + 2)/16.  `xp` is the array module
    (numpy, or torch for device tensors)."""
    rho = x * 0.0 + 1.0
    u = xp.sin(x) * xp.cos(y) * xp.cos(z)
    v = -xp.cos(x) * xp.sin(y) * xp.cos(z)
    w = x * 0.0
    p = 1.0 / (gamma * mach * mach) + (xp.cos(2 * x) + xp.cos(2 * y)) * (xp.cos(2 * z) + 2.0) / 16.0
    return rho, u, v, w, p


def density_wave_primitive(x, y, z, t=0.0, u0=0.5, amp=0.2, p0=1.0, xp=np):
    """Exact Euler solution: density wave advected by a constant velocity (u0,u0,u0)."""
    rho = 1.0 + amp * xp.sin(x + y + z - 3.0 * u0 * t)
    u = x * 0.0 + u0
    return rho, u, u * 1.0, u * 1.0, x * 0.0 + p0


def node_noise(seed: int, n_nodes: int, elems, amp: float = 1e-3, n_vars: int = 5):
    """Uniform noise U(-amp, amp) per element, variable and volume node.

    The full stream is laid out as [element][variable][node] in generator element
    order; the values of element e start at draw e*n_vars*n_nodes of a PCG64(seed)
    stream, so any subset of elements can be produced without the others.
    Returns float64 [len(elems), n_vars, n_nodes].
    """
    elems = np.asarray(elems, dtype=np.int64).reshape(-1)
    out = np.empty((elems.size, n_vars, n_nodes))
    per = n_vars * n_nodes
    if elems.size == 0:
        return out
    # contiguous runs share one generator
    order = np.argsort(elems, kind="stable")
    se = elems[order]
    run_start = 0
    while run_start < se.size:
        run_end = run_start + 1
        while run_end < se.size and se[run_end] == se[run_end - 1] + 1:
            run_end += 1
        bg = np.random.PCG64(seed)
        bg.advance(int(se[run_start]) * per)
        g = np.random.Generator(bg)
        vals = g.uniform(-amp, amp, size=(run_end - run_start, n_vars, n_nodes))
        out[order[run_start:run_end]] = vals
        run_start = run_end
    return out


def time_step(mesh: Mesh, N: int, cfl: float = 0.5, gamma: float = 1.4, mach: float = 0.1):
    """dt = CFL * min_e l_e / ((2N+1) * S), with l_e = 6 |e| / |boundary of e| of the split
    shapes (hex h, prism 3h/(3+sqrt 2), pyramid and Kuhn tet h/(1+sqrt 2)) and S an upper
    bound of |u| + c of the Taylor-Green initial field (|u| <= 1, p <= p0 + 3/8, rho = 1)."""
    h = mesh.h
    ell = {HEX: h, PRISM: 3.0 * h / (3.0 + math.sqrt(2.0)),
           PYR: h / (1.0 + math.sqrt(2.0)), TET: h / (1.0 + math.sqrt(2.0))}
    present = [t for t in range(4) if mesh.type_counts()[t] > 0]
    lmin = min(ell[t] for t in present)
    pmax = 1.0 / (gamma * mach * mach) + 3.0 / 8.0
    S = 1.0 + math.sqrt(gamma * pmax)
    return cfl * lmin / ((2 * N + 1) * S)


def stored_dofs(etype: int, N: int) -> int:
    """Stored values per variable of an element: (N+1)^3 nodal values for hexahedra, the
    number of modes of the collapsed types (tet n(n+1)(n+2)/6, prism n^2(n+1)/2, pyramid
    n(n+1)(2n+1)/6 with n = N+1)."""
    n = N + 1
    return {HEX: n ** 3, PRISM: n * n * (n + 1) // 2, PYR: n * (n + 1) * (2 * n + 1) // 6,
            TET: n * (n + 1) * (n + 2) // 6}[int(etype)]


def coefficient_state(mesh: Mesh, N: int, seed: int = 2, amp: float = 1e-3, gamma: float = 1.4,
                      mach: float = 0.1):
    """A valid state given directly in the stored variables, for meshes too large to project
    an initial field element by element: per element the conservative Taylor-Green state at
    its centroid, c(e), as every nodal value of a hexahedron and as the first (constant-mode)
    coefficient of the other types, plus seeded uniform noise U(-amp, amp) on every stored
    value (first modes included).  Layout: input element order, per element [5][ndof].
    Returns (U, offsets)."""
    ndof = np.array([stored_dofs(t, N) for t in range(4)])[mesh.elem_type]
    off = np.concatenate([[0], np.cumsum(5 * ndof)]).astype(np.int64)
    g = np.random.Generator(np.random.PCG64(seed))
    U = g.uniform(-amp, amp, size=int(off[-1]))
    c = mesh.centroid
    rho, u, v, w, p = tgv_primitive(c[:, 0], c[:, 1], c[:, 2], gamma=gamma, mach=mach)
    cons = np.stack([rho, rho * u, rho * v, rho * w,
                     p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)], axis=1)  # [e][5]
    # per (element, variable) block: hexahedra get c(e) on every value, the other types on
    # the first value only
    block_len = np.repeat(ndof, 5)
    block_start = (off[:-1, None] + np.arange(5)[None, :] * ndof[:, None]).ravel()
    is_hex = np.repeat(mesh.elem_type == HEX, 5)
    vals = cons.ravel()
    U[block_start[~is_hex]] += vals[~is_hex]
    hex_entries = np.repeat(is_hex, block_len)
    U[hex_entries] += np.repeat(vals[is_hex], block_len[is_hex])
    return U, off
