"""Adjoint of the residual: vector-Jacobian products (dR/dU)^T lam, and through LSERK4.

Test infrastructure of the oracle.  The residual of dg.DGOracle.residual is a composition
of linear element and face operators (nodal evaluation V, traces at the face points,
weak derivatives, lifts, the inverse mass matrix) and pointwise nonlinear functions (the
Euler and viscous fluxes, the Lax-Friedrichs flux, the BR1 lifting variables).  Its
transpose is assembled here step by step in the reverse order of the forward evaluation:
each linear operator is applied transposed and each pointwise function through its
analytic Jacobian (physics.*_jacobian[s]).  The forward residual follows paper Eq. (1) and
Algorithm 1; the adjoint is not in the paper.  Conventions at the non-smooth points: the
maximum wave speed takes the left side on ties and d|x|/dx = sign(x) with sign(0) = 0.

Reverse LSERK4 stage s (forward K <- A_s K + R(U), U <- U + dt B_s K):
    Kbar <- Kbar + dt B_s Ubar;  Ubar <- Ubar + (dR/dU(U_s))^T Kbar;  Kbar <- A_s Kbar.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import dg as dgmod, physics

HEX = dgmod.HEX


def _x(a):
    return np.asarray(a, dtype=dgmod.ACC)


def _ring(ora, elems, depth):
    out = set(elems)
    for _ in range(depth):
        out |= {nb for e in list(out) for nb in ora.neighbours(e)}
    return out


def vjp(ora, U, lam, elems=None):
    """(dR/dU)^T lam for the whole state; with `elems`, only the entries of those elements
    are formed (exactly) and the rest are NaN."""
    mesh = ora.mesh
    ns = ora.equations == "ns"
    gam, mu, Pr, Rg = ora.gamma, ora.mu, ora.Pr, ora.Rgas
    if elems is None:
        out_set = set(range(mesh.n_elems))
        lam_set = sorted(out_set)
    else:
        out_set = set(int(e) for e in elems)
        lam_set = sorted(_ring(ora, out_set, 2 if ns else 1))
    # forward quantities, as in the residual over lam_set
    gset = sorted(_ring(ora, lam_set, 1)) if ns else []
    tr_elems = set(gset) if ns else set(lam_set)
    face_set = sorted({fi for e in tr_elems for fi, _ in ora.elem_faces[e]})
    qtr = {fi: (ora.trace(U, fi, 0), ora.trace(U, fi, 1)) for fi in face_set}
    grads = {e: ora._gradients(U, e, qtr) for e in gset}

    qbar_nodes = {}
    qbar_tr = {}
    cbar = {e: np.zeros_like(grads[e][1]) for e in gset}
    fbar = {}

    def add_tr(fi, side, val):
        acc = qbar_tr.setdefault(fi, [0.0, 0.0])
        acc[side] = acc[side] + val

    # residual of every element of lam_set, reversed
    for e in lam_set:
        g = ora.elem_geo(e)
        t = g["type"]
        ref = ora.tref[t]
        lam_e = np.asarray(lam[ora.offset[e]:ora.offset[e + 1]], dtype=np.float64).reshape(5, -1)
        wJ = _x(ref["w"] * g["J"])
        if t == HEX:
            rbar = _x(lam_e) / wJ[None, :]
            sbar = None
        else:
            # d = M^-1 (r V + s), M symmetric
            sbar = _x(sla.cho_solve(g["chol"], lam_e.T).T)
            rbar = sbar @ _x(ref["V"]).T
        q = ora.nodal(U, e)
        # weak volume term r_k = sum_m w_m sum_a G^a_m dl_k/deta_a(eta_m)
        Gbar = np.einsum("vk,m,mka->avm", rbar, _x(ref["w"]), _x(ref["dL"]))
        Fbar = np.einsum("mac,avm->cvm", _x(g["acon"]), Gbar)
        qb = np.einsum("cvm,cvwm->wm", Fbar, physics.euler_flux_jacobian(q, gam))
        if ns:
            gn = ora._grad_nodal(e, grads[e])
            dq, dgr = physics.viscous_flux_jacobians(q, gn, gam, mu, Pr, Rg)
            qb = qb - np.einsum("cvm,cvwm->wm", Fbar, dq)
            gnbar = -np.einsum("cvm,cvsdm->sdm", Fbar, dgr)
            if grads[e][0] == "nodal":
                cbar[e] = cbar[e] + gnbar
            else:
                cbar[e] = cbar[e] + gnbar @ _x(ref["V"])
        qbar_nodes[e] = qbar_nodes.get(e, 0.0) + qb
        # surface term: r or s gets sign * (f* ws) @ basis-at-face-points
        for fi, side in ora.elem_faces[e]:
            fg = ora.face_geo(fi)
            sign = -1.0 if side == 0 else 1.0
            if t == HEX:
                cb = sign * (rbar @ _x(fg[("lag", side)]).T)
            else:
                cb = sign * (sbar @ _x(fg[("psi", side)]).T)
            fbar[fi] = fbar.get(fi, 0.0) + cb * _x(fg["ws"])[None, :]

    # face fluxes
    for fi in sorted(fbar):
        fb = fbar[fi]
        fg = ora.face_geo(fi)
        f = ora.faces[fi]
        qL, qR = qtr[fi]
        nrm = _x(fg["normal"])
        JL, JR = physics.lax_friedrichs_jacobians(qL, qR, nrm, gam)
        add_tr(fi, 0, np.einsum("vp,vwp->wp", fb, JL))
        add_tr(fi, 1, np.einsum("vp,vwp->wp", fb, JR))
        if ns:
            # f* -= (Fv_L + Fv_R).n / 2
            Fvbar = -0.5 * nrm[:, None, :] * fb[None, :, :]
            for side, es in ((0, f.eL), (1, f.eR)):
                gs = ora._grad_trace(fi, side, grads[es])
                dq, dgr = physics.viscous_flux_jacobians(qtr[fi][side], gs, gam, mu, Pr, Rg)
                add_tr(fi, side, np.einsum("cvp,cvwp->wp", Fvbar, dq))
                gsbar = np.einsum("cvp,cvsdp->sdp", Fvbar, dgr)
                key = "lag" if grads[es][0] == "nodal" else "psi"
                cbar[es] = cbar[es] + gsbar @ _x(fg[(key, side)])

    # BR1 gradients (dg.DGOracle._gradients, strong or weak form)
    strong = ora.lifting == "strong"
    for e in gset:
        cb = cbar[e]
        if not np.any(cb):
            continue
        g = ora.elem_geo(e)
        t = g["type"]
        ref = ora.tref[t]
        if grads[e][0] == "nodal":
            sb = cb / _x(ref["w"] * g["J"])[None, None, :]
            key = "lag"
        else:
            rhs = np.asarray(cb, dtype=np.float64).reshape(12, -1)
            sb = _x(sla.cho_solve(g["chol"], rhs.T).T).reshape(4, 3, -1)
            key = "psi"
        if strong:
            # J grad(w_h)[s, c, m] = sum_a a^a_c(m) sum_k wv[s, k] dl_k/deta_a(eta_m)
            if t == HEX:
                Jgbar = cb / _x(g["J"])[None, None, :]
            else:
                Jgbar = np.einsum("scj,mj,m->scm", sb, _x(ref["V"]), _x(ref["w"]))
            dwbar = np.einsum("scm,mac->sam", Jgbar, _x(g["acon"]))
            wvbar = np.einsum("sam,mka->sk", dwbar, _x(ref["dL"]))
        else:
            vb = -sb if t == HEX else -(sb @ _x(ref["V"]).T)
            # vol[s, c, k] = sum_m wv[s, m] w_m a^a_c(m) dl_k/deta_a(eta_m)
            wvbar = np.einsum("sck,m,mac,mka->sm", vb, _x(ref["w"]), _x(g["acon"]), _x(ref["dL"]))
        q = ora.nodal(U, e)
        qbar_nodes[e] = qbar_nodes.get(e, 0.0) + np.einsum(
            "sm,swm->wm", wvbar, physics.lifting_jacobian(q, gam, Rg))
        for fi, side in ora.elem_faces[e]:
            fg = ora.face_geo(fi)
            nout = _x(fg["normal"]) if side == 0 else -_x(fg["normal"])
            wsbar = np.einsum("p,cp,sck,pk->sp", _x(fg["ws"]), nout, sb, _x(fg[(key, side)]))
            qL, qR = qtr[fi]
            # face value w* = (w_L + w_R)/2, less the own w_own in the strong form
            cL = 0.5 - (1.0 if strong and side == 0 else 0.0)
            cR = 0.5 - (1.0 if strong and side == 1 else 0.0)
            add_tr(fi, 0, cL * np.einsum("sp,swp->wp", wsbar, physics.lifting_jacobian(qL, gam, Rg)))
            add_tr(fi, 1, cR * np.einsum("sp,swp->wp", wsbar, physics.lifting_jacobian(qR, gam, Rg)))

    # traces and nodal values back to the stored coefficients
    acc = {}
    for e, qb in qbar_nodes.items():
        t = int(mesh.elem_type[e])
        acc[e] = acc.get(e, 0.0) + (qb if t == HEX else qb @ _x(ora.tref[t]["V"]))
    for fi, sides in qbar_tr.items():
        f = ora.faces[fi]
        fg = ora.face_geo(fi)
        for side, es in ((0, f.eL), (1, f.eR)):
            b = sides[side]
            if np.isscalar(b):
                continue
            key = "lag" if mesh.elem_type[es] == HEX else "psi"
            acc[es] = acc.get(es, 0.0) + b @ _x(fg[(key, side)])
    out = np.full(ora.size, np.nan)
    for e in out_set:
        val = acc.get(e)
        a, b = ora.offset[e], ora.offset[e + 1]
        out[a:b] = 0.0 if val is None else np.asarray(val, dtype=np.float64).ravel()
    return out


def kinetic_energy_grad(ora, U):
    """d/dU of dg.DGOracle.kinetic_energy: E = sum_e sum_m w_m J_m |rho u|^2 / (2 rho)."""
    out = np.zeros(ora.size)
    for e in range(ora.mesh.n_elems):
        g = ora.elem_geo(e)
        t = g["type"]
        ref = ora.tref[t]
        q = ora.nodal(U, e)
        m2 = q[1] ** 2 + q[2] ** 2 + q[3] ** 2
        qb = np.zeros_like(q)
        qb[0] = -0.5 * m2 / q[0] ** 2
        qb[1:4] = q[1:4] / q[0]
        qb = qb * _x(ref["w"] * g["J"])[None, :]
        ub = qb if t == HEX else qb @ _x(ref["V"])
        out[ora.offset[e]:ora.offset[e + 1]] = np.asarray(ub, dtype=np.float64).ravel()
    return out


def rk_vjp(ora, U0, dt, n_steps, Ubar):
    """Gradient with respect to U0 of <Ubar, U_n> where U_n is U0 after n_steps of LSERK4
    (K = 0 at the start of every step), by the reverse stage recursion; every stage state
    is kept."""
    A, B = dgmod.LSERK_A, dgmod.LSERK_B
    states = []
    U = np.array(U0, dtype=float)
    K = np.zeros_like(U)
    for _ in range(n_steps):
        K[:] = 0.0
        for s in range(5):
            states.append(U.copy())
            K = A[s] * K + ora.residual(U)
            U = U + dt * B[s] * K
    Ub = np.array(Ubar, dtype=float)
    Kb = np.zeros_like(Ub)
    for i in reversed(range(len(states))):
        s = i % 5
        Kb = Kb + dt * B[s] * Ub
        Ub = Ub + vjp(ora, states[i], Kb)
        Kb = A[s] * Kb
    return Ub
