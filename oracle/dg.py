"""Plain FP64 residual R(U) of modal-time-stepping DGSEM on mixed meshes, and LSERK4.

Test infrastructure of the oracle.  Written element by element and face by face from the
paper's statement of the method, with no operator factorisation:

* weak form, paper Eq. (1): for every test function l_k of the element's nodal tensor
  basis,  int J q_t l_k = int F . grad_xi l_k  -  oint (F.n)* l_k dS, with the volume
  integral evaluated by the element's nodal quadrature,
      r_k = sum_m w_m sum_a G^a_m d l_k/d eta_a (eta_m),   G^a = sum_c a^a_c F_c;
* surface term on every face point P:  r_k -= ws_P f*_P l_k(P) on side L (normal L->R)
  and += on side R;
* hexahedra are advanced nodally (lumped mass): dU/dt_k = r_k / (w_k J_k);
* prisms, pyramids and tetrahedra are advanced modally (paper Sec. 2, Algorithm 1):
  dU~/dt = M^-1 V^T r with M = V^T W J V per element, where the surface term is applied
  to the modes directly through phi_j(P) (= V^T of the nodal lift, as phi_j is exactly
  represented by the nodal basis);
* Navier-Stokes: BR1 lifting of (u, v, w, T) in strong form (face value w* = (w_L + w_R)/2,
  with w evaluated from each side's state trace), nodal with lumped mass on hexahedra and
  modal with the element mass matrix on the other types (see _gradients);
  viscous face flux (Fv_L + Fv_R).n / 2 from each side's state and gradient traces;
* time integration by the five-stage fourth-order 2N-storage LSERK scheme (Sec. 2,
  method of lines);
* optional entropy-stable split form of the inviscid volume term (Sec. 2: an SBP-like property
  and Chandrashekar's two-point flux).  Along a node line of direction a whose 1-D rule holds
  both end points (Gauss-Lobatto: Q = W D with Q + Q^T = diag(-1, 0, .., 0, 1)), the weak term
  sum_m Q[m][i] G^a_m is replaced by the flux-differencing form
      sum_m (Q^T - Q)[i][m] F#(q_i, q_m) . (a^a_i + a^a_m) / 2,
  which equals the weak term for a constant state and, for hexahedra, is the entropy-
  conservative SBP split form.  Directions on left Gauss-Radau nodes (collapsing directions of
  prisms, pyramids and tetrahedra, whose boundary operator Q + Q^T is not diagonal) keep the
  weak term; viscous fluxes always do.  The surface flux is local Lax-Friedrichs, or the
  two-point flux itself (entropy conservative) for property tests.

State layout (generator element order): element e owns U[off[e]:off[e+1]], shaped
(5, ndof_e) variable-major; hexahedra hold nodal values at the volume nodes, the other
types the coefficients of basis.psi.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import basis, faces as facemod, geometry, physics, rules

HEX, PRISM, PYR, TET = geometry.HEX, geometry.PRISM, geometry.PYR, geometry.TET

# Residual sums are accumulated in extended precision and the result rounded once to FP64:
# at low Mach number the pressure (~71 at Ma 0.1) cancels between volume and surface terms
# down to O(1) residuals, so FP64 accumulation would add errors far above the problem's own
# FP64 conditioning.  Tables (V, Lagrange values, weights, metrics) stay FP64.
ACC = np.longdouble


def _x(a):
    return np.asarray(a, dtype=ACC)


def set_accumulation(dtype):
    """Select the accumulation precision of the residual sums (np.longdouble by default;
    np.float64 gives the plain FP64 evaluation of the same formulas)."""
    global ACC
    ACC = dtype

# Carpenter & Kennedy (1994) five-stage fourth-order 2N-storage coefficients
LSERK_A = np.array([0.0,
                    -567301805773.0 / 1357537059087.0,
                    -2404267990393.0 / 2016746695238.0,
                    -3550918686646.0 / 2091501179385.0,
                    -1275806237668.0 / 842570457699.0])
LSERK_B = np.array([1432997174477.0 / 9575080441755.0,
                    5161836677717.0 / 13612068292357.0,
                    1720146321549.0 / 2090206949498.0,
                    3134564353537.0 / 4481467310338.0,
                    2277821191437.0 / 14882151754819.0])
LSERK_C = np.array([0.0,
                    1432997174477.0 / 9575080441755.0,
                    2526269341429.0 / 6820363962896.0,
                    2006345519317.0 / 3224310063776.0,
                    2802321613138.0 / 2924317926251.0])


class _ElemFaces:
    """elem_faces[e] -> list of (face index, side) of element e (side 0 = L)."""

    def __init__(self, o):
        self.o = o

    def __getitem__(self, e):
        o = self.o
        a, b = o._ef_ptr[e], o._ef_ptr[e + 1]
        return list(zip(o._ef_face[a:b].tolist(), o._ef_side[a:b].tolist()))

    def __len__(self):
        return self.o.mesh.n_elems


class DGOracle:
    def __init__(self, mesh, N, equations="euler", gamma=1.4, mu=1.0 / 1600.0, Pr=0.71,
                 Rgas=1.0, volume_form="weak", surface_flux="lf", node_family="R1",
                 lifting="strong", corner_velocity=None):
        """node_family: "R1" (the discretisation of the hot path) or "LG" (Gauss-Legendre volume
        and quadrilateral-face points, weak volume form only).  lifting: "strong" or "weak", the
        form of the BR1 lifting (_gradients).  corner_velocity: None, or the velocity of every
        element corner [n_elems][8][3] (a mesh moving with the trilinear interpolation of these):
        residual() is then the moving-mesh form at this instant (weak form, LF flux only)."""
        if equations not in ("euler", "ns"):
            raise ValueError(equations)
        if volume_form not in ("weak", "split") or surface_flux not in ("lf", "ec"):
            raise ValueError((volume_form, surface_flux))
        if node_family not in geometry.NODE_FAMILIES or lifting not in ("strong", "weak"):
            raise ValueError((node_family, lifting))
        if node_family != "R1" and volume_form != "weak":
            raise ValueError("the split form is defined on the R1 nodes only")
        if corner_velocity is not None and (volume_form != "weak" or surface_flux != "lf"):
            raise ValueError("moving meshes take the weak form with the LF flux")
        self.cvel = None if corner_velocity is None else np.asarray(corner_velocity, dtype=np.float64)
        self.volume_form, self.surface_flux = volume_form, surface_flux
        self.family, self.lifting = node_family, lifting
        self.mesh = mesh
        self.N = int(N)
        self.n = self.N + 1
        self.equations = equations
        self.gamma, self.mu, self.Pr, self.Rgas = gamma, mu, Pr, Rgas
        n3 = self.n ** 3
        self.ndof_type = [n3] + [basis.n_modes(t, self.N) for t in (PRISM, PYR, TET)]
        self.ndof = np.array(self.ndof_type)[mesh.elem_type]
        self.offset = np.concatenate([[0], np.cumsum(5 * self.ndof)]).astype(np.int64)
        self.size = int(self.offset[-1])
        # per-type reference data: nodes, weights, basis derivatives at the nodes, V
        self.tref = {}
        for t in range(4):
            eta, w = geometry.volume_nodes(t, self.n, self.family)
            ref = dict(eta=eta, w=w, dL=geometry.lagrange3d_grad(t, self.n, eta, self.family))
            # 1-D operators per direction for the split form: Q = W D, and whether the rule
            # holds both end points
            r1 = geometry.node_rules(t, self.n, self.family)
            ref["Q1"] = [np.asarray(wa, dtype=float)[:, None] * np.asarray(rules.derivative_matrix(xa), dtype=float)
                         for xa, wa in r1]
            ref["w1"] = [np.asarray(wa, dtype=float) for _, wa in r1]
            ref["sbp"] = [name == "GL" for name in geometry.NODE_FAMILIES[self.family][t]]
            if t != HEX:
                ref["V"] = basis.psi(t, self.N, eta)
            self.tref[t] = ref
        self.faces = facemod.build_faces(mesh)
        # element -> (face, side) lists in CSR form
        nf = len(self.faces)
        owner = np.concatenate([self.faces.eL, self.faces.eR])
        fidx = np.concatenate([np.arange(nf), np.arange(nf)])
        side = np.concatenate([np.zeros(nf, int), np.ones(nf, int)])
        o = np.lexsort((side, fidx, owner))
        self._ef_face, self._ef_side = fidx[o], side[o]
        self._ef_ptr = np.concatenate([[0], np.cumsum(np.bincount(owner, minlength=mesh.n_elems))])
        self._geo = {}
        self._fgeo = {}

    # ------------------------------------------------------------------ geometry
    def elem_geo(self, e):
        g = self._geo.get(e)
        if g is None:
            t = int(self.mesh.elem_type[e])
            ref = self.tref[t]
            corners = self.mesh.corner_xyz[e]
            J, acon = geometry.metrics(corners, ref["eta"])
            if np.any(J <= 0):  # noqa: SIM102
                raise ValueError(f"element {e}: non-positive Jacobian at a volume node")
            g = dict(type=t, J=J, acon=acon, x=geometry.map_points(corners, ref["eta"]))
            if self.cvel is not None:
                # grid velocity at the nodes, and dJ/dt by Jacobi's formula: the derivative of
                # det(dx/deta) is sum_a (d xdot / d eta_a) . a^a (a^a the cofactor columns)
                ld = np.longdouble
                g["xdot"] = geometry.map_points(self.cvel[e], ref["eta"])
                Xd = geometry.jacobian(np.asarray(self.cvel[e], ld), np.asarray(ref["eta"], ld))
                g["Jdot"] = np.einsum("pca,pac->p", Xd, acon)
            if t != HEX:
                V = ref["V"]
                M = V.T @ (V * (ref["w"] * J)[:, None])
                g["chol"] = sla.cho_factor(np.asarray(M, dtype=np.float64), lower=True)
            self._geo[e] = g
        return g

    def face_geo(self, fi):
        fg = self._fgeo.get(fi)
        if fg is None:
            f = self.faces[fi]
            facemod.face_geometry(self.mesh, f, self.n, self.family)
            fg = dict(normal=f.normal, ws=f.ws)
            if self.cvel is not None:
                # normal speed of the face points: the face's own parametrisation applied to the
                # velocities of side L's vertices
                cL = self.mesh.elem_corner[f.eL]
                vel = lambda vid: self.cvel[f.eL][int(np.nonzero(cL == vid)[0][0])]  # noqa: E731
                V4 = (vel(facemod._quad_fourth(self.mesh, f.eL, f.planeL, f.ids))
                      if f.kind == "quad" else None)
                s_, t_, _ = facemod.face_rule(f.kind, self.n, self.family, f.chunk)
                Pv, _, _ = facemod.face_points(f.kind, *[vel(v) for v in f.ids], s_, t_, V4)
                fg["vn"] = np.einsum("pc,cp->p", Pv, f.normal)
            for side, e, eta in ((0, f.eL, f.etaL), (1, f.eR, f.etaR)):
                t = int(self.mesh.elem_type[e])
                fg[("lag", side)] = geometry.lagrange3d(t, self.n, eta, self.family)
                if t != HEX:
                    fg[("psi", side)] = basis.psi(t, self.N, eta)
            self._fgeo[fi] = fg
        return fg

    @property
    def elem_faces(self):
        return _ElemFaces(self)

    def neighbours(self, e):
        out = []
        for fi, side in self.elem_faces[e]:
            f = self.faces[fi]
            out.append(f.eR if side == 0 else f.eL)
        return out

    # ------------------------------------------------------------------ state helpers
    def elem_state(self, U, e):
        return U[self.offset[e]:self.offset[e + 1]].reshape(5, -1)

    def nodal(self, U, e):
        """Nodal conservative state (5, n^3) at the volume nodes."""
        t = int(self.mesh.elem_type[e])
        u = _x(self.elem_state(U, e))
        if t == HEX:
            return u
        return u @ _x(self.tref[t]["V"]).T

    def trace(self, U, fi, side):
        """State at the face points, evaluated from the side's own polynomial: (5, P)."""
        f = self.faces[fi]
        e = f.eL if side == 0 else f.eR
        fg = self.face_geo(fi)
        u = _x(self.elem_state(U, e))
        if self.mesh.elem_type[e] == HEX:
            return u @ _x(fg[("lag", side)]).T
        return u @ _x(fg[("psi", side)]).T

    def project(self, e, qnodal):
        """Modal time-stepping projection (Algorithm 1): u~ = M^-1 V^T W J q."""
        t = int(self.mesh.elem_type[e])
        if t == HEX:
            return np.array(qnodal, dtype=float)
        g = self.elem_geo(e)
        ref = self.tref[t]
        rhs = (_x(qnodal) * (ref["w"] * g["J"])[None, :]) @ ref["V"]
        return sla.cho_solve(g["chol"], np.asarray(rhs, dtype=np.float64).T).T

    def initial_state(self, prim_fn, noise_fn=None, elems=None):
        """U with U_e = projection of cons(prim_fn(x)) + noise at the volume nodes.
        `noise_fn(elems)` returns (len(elems), 5, n^3) in generator element order."""
        elems = range(self.mesh.n_elems) if elems is None else elems
        elems = list(elems)
        U = np.full(self.size, np.nan)
        nz = noise_fn(np.array(elems)) if noise_fn is not None else None
        for i, e in enumerate(elems):
            x = self.elem_geo(e)["x"]
            q = physics.primitive_to_conservative(*prim_fn(x[:, 0], x[:, 1], x[:, 2]),
                                                  gamma=self.gamma)
            if nz is not None:
                q = q + nz[i]
            U[self.offset[e]:self.offset[e + 1]] = self.project(e, q).ravel()
        return U

    # ------------------------------------------------------------------ residual
    def _volume(self, q, e, Fv=None):
        g = self.elem_geo(e)
        ref = self.tref[g["type"]]
        F = physics.euler_flux(q, self.gamma)            # (3, 5, K)
        if self.cvel is not None:
            # flux relative to the moving nodes: F - q xdot
            F = F - _x(g["xdot"]).T[:, None, :] * q[None, :, :]
        if Fv is not None:
            F = F - Fv
        G = np.einsum("mac,cvm->avm", _x(g["acon"]), F)   # contravariant flux (3, 5, K)
        return np.einsum("avm,m,mka->vk", G, _x(ref["w"]), _x(ref["dL"]))

    def _volume_split(self, q, e, Fv=None, two_point=None):
        """Volume term with the split form along every Gauss-Lobatto direction (module
        docstring); `two_point(qa, qb, n)` defaults to the Chandrashekar flux."""
        g = self.elem_geo(e)
        ref = self.tref[g["type"]]
        if two_point is None:
            gamma = self.gamma
            two_point = lambda qa, qb, nv: physics.chandrashekar_flux(qa, qb, nv, gamma)  # noqa: E731
        n = self.n
        K = n ** 3
        acon = _x(g["acon"])                                 # (K, 3, 3): a^a_c at the nodes
        F = physics.euler_flux(q, self.gamma)
        r = np.zeros((5, K), dtype=ACC)
        idx = np.arange(K)
        ijk = np.stack([idx % n, (idx // n) % n, idx // (n * n)])
        stride = [1, n, n * n]
        for a in range(3):
            if ref["sbp"][a]:
                # two-point part over every ordered pair (k, m) on a line of direction a
                Q = ref["Q1"][a]
                wperp = _x(ref["w"]) / _x(ref["w1"][a][ijk[a]])
                ks, ms = [], []
                for l in range(n):
                    m = idx + (l - ijk[a]) * stride[a]
                    keep = l != ijk[a]
                    ks.append(idx[keep])
                    ms.append(m[keep])
                ks, ms = np.concatenate(ks), np.concatenate(ms)
                navg = 0.5 * (acon[ks, a, :] + acon[ms, a, :]).T       # (3, pairs)
                Fp = two_point(q[:, ks], q[:, ms], navg)
                coef = _x(Q[ijk[a][ms], ijk[a][ks]] - Q[ijk[a][ks], ijk[a][ms]]) * wperp[ks]
                np.add.at(r.T, ks, (coef * Fp).T)
                if Fv is not None:   # the viscous flux keeps the weak term
                    G = np.einsum("mc,cvm->vm", acon[:, a, :], -Fv)
                    r += np.einsum("vm,m,mk->vk", G, _x(ref["w"]), _x(ref["dL"][:, :, a]))
            else:
                Fa = F if Fv is None else F - Fv
                G = np.einsum("mc,cvm->vm", acon[:, a, :], Fa)
                r += np.einsum("vm,m,mk->vk", G, _x(ref["w"]), _x(ref["dL"][:, :, a]))
        return r

    def _gradients(self, U, e, qtr):
        """BR1 lifted gradients g of the lifting variables w = (u, v, w, T) on element e, with the
        face value w* = (w_L + w_R)/2 (each side's w from its state trace), in strong form
            int g phi J = int grad(w_h) phi J + oint (w* - w_own) n phi dS,
        where w_h interpolates w at the volume nodes (J grad(w_h) = sum_a a^a dw_h/deta_a) and
        w_own is w of the element's own state trace.  Hexahedra: nodal test functions l_k with
        the lumped (nodal) mass, g[s, c, k] at the volume nodes.  Other types: the modal test
        functions phi_j with the mass matrix M = V^T W J V of their time derivative, g~[s, c, j],
        g = V g~ at the nodes.
        The weak form  int g phi J = oint w* n phi dS - int w grad(phi) J  is the same lifting
        wherever the quadrature obeys a discrete Gauss theorem, as on a Gauss-Lobatto hexahedron
        with collocated faces.  The R1 rules of the collapsed types (a Gauss-Radau volume rule,
        Gauss-Lobatto points on quadrilateral faces), and a hexahedron face that meets two
        triangles (whose points are the triangles' own), fall short of it; there the weak form
        misses the gradient of a degree-N field by O(1), while the strong form returns it exactly
        (lifting="weak" keeps the weak form, for that comparison).
        Returns (kind, coefficients), kind "nodal" or "modal"."""
        g = self.elem_geo(e)
        t = g["type"]
        ref = self.tref[t]
        q = self.nodal(U, e)
        wv = physics.lifting_variables(q, self.gamma, self.Rgas)        # (4, K)
        strong = self.lifting == "strong"
        if strong:
            dw = np.einsum("sk,mka->sam", wv, _x(ref["dL"]))               # dw_h/deta_a at node m
            Jg = np.einsum("sam,mac->scm", dw, _x(g["acon"]))              # J grad(w_h) at node m
        else:
            vol = np.einsum("sm,m,mac,mka->sck", wv, _x(ref["w"]), _x(g["acon"]), _x(ref["dL"]))
        key = "lag" if t == HEX else "psi"
        surf = np.zeros((4, 3, self.ndof[e]), dtype=ACC)
        for fi, side in self.elem_faces[e]:
            fg = self.face_geo(fi)
            qL, qR = qtr[fi]
            wL = physics.lifting_variables(qL, self.gamma, self.Rgas)
            wR = physics.lifting_variables(qR, self.gamma, self.Rgas)
            wstar = 0.5 * (wL + wR)
            if strong:
                wstar = wstar - (wL if side == 0 else wR)
            nout = fg["normal"] if side == 0 else -fg["normal"]
            surf += np.einsum("p,sp,cp,pk->sck", _x(fg["ws"]), wstar, _x(nout), _x(fg[(key, side)]))
        if t == HEX:
            wJ = _x(ref["w"] * g["J"])[None, None, :]
            if strong:
                return "nodal", Jg / _x(g["J"])[None, None, :] + surf / wJ
            return "nodal", (surf - vol) / wJ
        if strong:
            rhs = np.einsum("scm,m,mj->scj", Jg, _x(ref["w"]), _x(ref["V"])) + surf
        else:
            rhs = surf - vol @ _x(ref["V"])
        rhs = rhs.reshape(12, -1).astype(np.float64)
        gm = sla.cho_solve(g["chol"], rhs.T).T.reshape(4, 3, -1)
        return "modal", _x(gm)

    def _grad_nodal(self, e, gr):
        kind, c = gr
        if kind == "nodal":
            return c
        return c @ _x(self.tref[int(self.mesh.elem_type[e])]["V"]).T

    def _grad_trace(self, fi, side, gr):
        kind, c = gr
        fg = self.face_geo(fi)
        return c @ _x(fg[("lag" if kind == "nodal" else "psi", side)]).T

    def residual(self, U, elems=None):
        """dU/dt for the elements `elems` (all when None); other entries are NaN."""
        mesh = self.mesh
        S = list(range(mesh.n_elems)) if elems is None else sorted(set(int(e) for e in elems))
        ns = self.equations == "ns"
        if ns:
            Gset = set(S)
            for e in S:
                Gset.update(self.neighbours(e))
            tr_elems = set(Gset)
        else:
            Gset = set()
            tr_elems = set(S)
        face_set = set()
        for e in tr_elems:
            for fi, _ in self.elem_faces[e]:
                face_set.add(fi)
        qtr = {fi: (self.trace(U, fi, 0), self.trace(U, fi, 1)) for fi in sorted(face_set)}
        grads = {e: self._gradients(U, e, qtr) for e in sorted(Gset)} if ns else {}
        out = np.full(self.size, np.nan)
        for e in S:
            g = self.elem_geo(e)
            t = g["type"]
            ref = self.tref[t]
            q = self.nodal(U, e)
            Fv = (physics.viscous_flux(q, self._grad_nodal(e, grads[e]), self.gamma, self.mu,
                                       self.Pr, self.Rgas) if ns else None)
            r = self._volume(q, e, Fv) if self.volume_form == "weak" else self._volume_split(q, e, Fv)
            if self.cvel is not None:
                # the test functions' mass moments change as J does: M du~/dt = r - (dM/dt) u~,
                # dM/dt u~ = V^T W (dJ/dt q) at the nodes (Alg. 1 with a Jacobian that changes)
                r = r - q * _x(ref["w"] * g["Jdot"])[None, :]
            smodal = np.zeros((5, self.ndof[e]), dtype=ACC)
            for fi, side in self.elem_faces[e]:
                fg = self.face_geo(fi)
                f = self.faces[fi]
                qL, qR = qtr[fi]
                if self.cvel is not None:
                    fstar = physics.lax_friedrichs_moving(qL, qR, _x(fg["normal"]), _x(fg["vn"]), self.gamma)
                elif self.surface_flux == "lf":
                    fstar = physics.lax_friedrichs(qL, qR, _x(fg["normal"]), self.gamma)
                else:
                    fstar = physics.chandrashekar_flux(qL, qR, _x(fg["normal"]), self.gamma)
                if ns:
                    gL = self._grad_trace(fi, 0, grads[f.eL])
                    gR = self._grad_trace(fi, 1, grads[f.eR])
                    FvL = physics.viscous_flux(qL, gL, self.gamma, self.mu, self.Pr, self.Rgas)
                    FvR = physics.viscous_flux(qR, gR, self.gamma, self.mu, self.Pr, self.Rgas)
                    fstar = fstar - 0.5 * physics.normal_flux(FvL + FvR, _x(fg["normal"]))
                contrib = fstar * _x(fg["ws"])[None, :]
                sign = -1.0 if side == 0 else 1.0
                if t == HEX:
                    r += sign * (contrib @ _x(fg[("lag", side)]))
                else:
                    smodal += sign * (contrib @ _x(fg[("psi", side)]))
            if t == HEX:
                d = r / _x(ref["w"] * g["J"])[None, :]
            else:
                rhs = (r @ _x(ref["V"]) + smodal).astype(np.float64)
                d = sla.cho_solve(g["chol"], rhs.T).T
            out[self.offset[e]:self.offset[e + 1]] = np.asarray(d, dtype=np.float64).ravel()
        return out

    # ------------------------------------------------------------------ time integration
    def rk_steps(self, U, dt, n_steps, K=None):
        """n_steps of LSERK4: per stage K <- A_s K + R(U), U <- U + dt B_s K (K = 0 at start)."""
        U = np.array(U, dtype=float)
        K = np.zeros_like(U) if K is None else np.array(K, dtype=float)
        for _ in range(n_steps):
            for s in range(5):
                K = LSERK_A[s] * K + self.residual(U)
                U = U + dt * LSERK_B[s] * K
        return U, K

    # ------------------------------------------------------------------ diagnostics
    def integral(self, U):
        """Discrete integral sum_e sum_m w_m J_m q_m of each conservative variable."""
        tot = np.zeros(5)
        for e in range(self.mesh.n_elems):
            g = self.elem_geo(e)
            tot += self.nodal(U, e) @ (self.tref[g["type"]]["w"] * g["J"])
        return tot

    def kinetic_energy(self, U):
        tot = 0.0
        for e in range(self.mesh.n_elems):
            g = self.elem_geo(e)
            q = self.nodal(U, e)
            ke = 0.5 * (q[1] ** 2 + q[2] ** 2 + q[3] ** 2) / q[0]
            tot += float(ke @ (self.tref[g["type"]]["w"] * g["J"]))
        return tot

    def l2_error(self, U, exact_fn, var=0):
        err = 0.0
        for e in range(self.mesh.n_elems):
            g = self.elem_geo(e)
            x = g["x"]
            qe = exact_fn(x[:, 0], x[:, 1], x[:, 2])
            d = self.nodal(U, e)[var] - qe[var]
            err += float((d * d) @ (self.tref[g["type"]]["w"] * g["J"]))
        return np.sqrt(err)
