"""Compressible Euler and Navier-Stokes-Fourier fluxes (FP64).

Test infrastructure of the oracle.  Conservative variables q = (rho, rho u, rho v, rho w,
rho E); ideal gas p = (gamma-1)(rho E - rho |u|^2 / 2).  The paper's solver integrates the
compressible Navier-Stokes-Fourier equations (Sec. 2).  Arrays carry the variable on the
first axis and any number of trailing point axes.
"""
from __future__ import annotations

import numpy as np


def pressure(q, gamma):
    rho = q[0]
    ke = 0.5 * (q[1] ** 2 + q[2] ** 2 + q[3] ** 2) / rho
    return (gamma - 1.0) * (q[4] - ke)


def euler_flux(q, gamma):
    """F[c, v, ...]: Cartesian component c of the inviscid flux of variable v."""
    rho = q[0]
    u = q[1:4] / rho
    p = pressure(q, gamma)
    F = np.empty((3, 5) + q.shape[1:], dtype=q.dtype)
    for c in range(3):
        F[c, 0] = q[1 + c]
        for i in range(3):
            F[c, 1 + i] = q[1 + i] * u[c]
        F[c, 1 + c] = F[c, 1 + c] + p
        F[c, 4] = (q[4] + p) * u[c]
    return F


def normal_flux(F, nrm):
    return F[0] * nrm[0] + F[1] * nrm[1] + F[2] * nrm[2]


def lax_friedrichs(qL, qR, nrm, gamma):
    """Local Lax-Friedrichs (Rusanov) flux
    f* = (F(qL) + F(qR)).n / 2 - lambda (qR - qL) / 2,
    lambda = max(|uL.n| + cL, |uR.n| + cR), c = sqrt(gamma p / rho)."""
    FL = normal_flux(euler_flux(qL, gamma), nrm)
    FR = normal_flux(euler_flux(qR, gamma), nrm)
    unL = (qL[1] * nrm[0] + qL[2] * nrm[1] + qL[3] * nrm[2]) / qL[0]
    unR = (qR[1] * nrm[0] + qR[2] * nrm[1] + qR[3] * nrm[2]) / qR[0]
    cL = np.sqrt(gamma * pressure(qL, gamma) / qL[0])
    cR = np.sqrt(gamma * pressure(qR, gamma) / qR[0])
    lam = np.maximum(np.abs(unL) + cL, np.abs(unR) + cR)
    return 0.5 * (FL + FR) - 0.5 * lam * (qR - qL)


def lax_friedrichs_moving(qL, qR, nrm, vn, gamma):
    """Local Lax-Friedrichs flux through a face moving with normal speed vn = xdot . n (the
    flux relative to the moving face, F - q xdot, in the arbitrary Lagrangian-Eulerian form):
    f* = (F(qL) + F(qR)).n / 2 - vn (qL + qR) / 2 - lambda (qR - qL) / 2,
    lambda = max(|uL.n - vn| + cL, |uR.n - vn| + cR).  vn = 0 is lax_friedrichs."""
    FL = normal_flux(euler_flux(qL, gamma), nrm)
    FR = normal_flux(euler_flux(qR, gamma), nrm)
    unL = (qL[1] * nrm[0] + qL[2] * nrm[1] + qL[3] * nrm[2]) / qL[0]
    unR = (qR[1] * nrm[0] + qR[2] * nrm[1] + qR[3] * nrm[2]) / qR[0]
    cL = np.sqrt(gamma * pressure(qL, gamma) / qL[0])
    cR = np.sqrt(gamma * pressure(qR, gamma) / qR[0])
    lam = np.maximum(np.abs(unL - vn) + cL, np.abs(unR - vn) + cR)
    return 0.5 * (FL + FR) - 0.5 * vn * (qL + qR) - 0.5 * lam * (qR - qL)


def lifting_variables(q, gamma, Rgas):
    """BR1 lifting variables (u, v, w, T) with T = p / (rho R)."""
    rho = q[0]
    out = np.empty((4,) + q.shape[1:], dtype=q.dtype)
    out[0:3] = q[1:4] / rho
    out[3] = pressure(q, gamma) / (rho * Rgas)
    return out


def viscous_flux(q, grad, gamma, mu, Pr, Rgas):
    """Fv[c, v, ...] from the state and the gradients grad[s, c, ...] of (u, v, w, T):
    tau = mu (grad u + grad u^T - 2/3 div u I), heat flux -kappa grad T,
    kappa = mu c_p / Pr, c_p = gamma R / (gamma - 1)."""
    u = q[1:4] / q[0]
    div = grad[0, 0] + grad[1, 1] + grad[2, 2]
    kappa = mu * gamma * Rgas / ((gamma - 1.0) * Pr)
    Fv = np.zeros((3, 5) + q.shape[1:], dtype=np.result_type(q, grad))
    for c in range(3):
        for i in range(3):
            tau = mu * (grad[i, c] + grad[c, i])
            if i == c:
                tau = tau - mu * (2.0 / 3.0) * div
            Fv[c, 1 + i] = tau
        Fv[c, 4] = u[0] * Fv[c, 1] + u[1] * Fv[c, 2] + u[2] * Fv[c, 3] + kappa * grad[3, c]
    return Fv


def primitive_to_conservative(rho, u, v, w, p, gamma):
    q = np.empty((5,) + np.shape(rho))
    q[0] = rho
    q[1] = rho * u
    q[2] = rho * v
    q[3] = rho * w
    q[4] = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return q


# ---------------------------------------------------------------------------------------
# Pointwise Jacobians for the adjoint (vector-Jacobian products of the residual).  Each
# returns the derivative array with the input variable on the axis named in the docstring;
# all follow from the chain rule on the definitions above.

def _dpressure(q, gamma):
    """dp/dq[w, ...]: ( (g-1)|u|^2/2, -(g-1)u, -(g-1)v, -(g-1)w, g-1 )."""
    rho = q[0]
    u = q[1:4] / rho
    g1 = gamma - 1.0
    d = np.empty_like(q)
    d[0] = 0.5 * g1 * (u[0] ** 2 + u[1] ** 2 + u[2] ** 2)
    d[1:4] = -g1 * u
    d[4] = g1
    return d


def _dvelocity(q):
    """du_c/dq[w]: array (3, 5, ...)."""
    rho = q[0]
    d = np.zeros((3,) + q.shape, dtype=q.dtype)
    for c in range(3):
        d[c, 0] = -q[1 + c] / (rho * rho)
        d[c, 1 + c] = 1.0 / rho
    return d


def euler_flux_jacobian(q, gamma):
    """dF[c, v, w, ...] = d F[c, v] / d q[w]."""
    rho = q[0]
    u = q[1:4] / rho
    p = pressure(q, gamma)
    dp = _dpressure(q, gamma)
    du = _dvelocity(q)
    one = np.ones_like(rho)
    dF = np.zeros((3, 5, 5) + q.shape[1:], dtype=q.dtype)
    for c in range(3):
        dF[c, 0, 1 + c] = one
        for i in range(3):
            dF[c, 1 + i] = q[1 + i] * du[c]
            dF[c, 1 + i, 1 + i] = dF[c, 1 + i, 1 + i] + u[c]
            if i == c:
                dF[c, 1 + i] = dF[c, 1 + i] + dp
        dF[c, 4] = u[c] * dp + (q[4] + p) * du[c]
        dF[c, 4, 4] = dF[c, 4, 4] + u[c]
    return dF


def _wave_speed(q, nrm, gamma):
    """a = |u.n| + c and da/dq[w] (d|x|/dx = sign(x), sign(0) = 0)."""
    rho = q[0]
    un = (q[1] * nrm[0] + q[2] * nrm[1] + q[3] * nrm[2]) / rho
    p = pressure(q, gamma)
    c = np.sqrt(gamma * p / rho)
    dun = np.zeros_like(q)
    dun[0] = -un / rho
    for i in range(3):
        dun[1 + i] = nrm[i] / rho
    dc = gamma / (2.0 * c) * (_dpressure(q, gamma) / rho)
    dc[0] = dc[0] - gamma / (2.0 * c) * p / (rho * rho)
    return np.abs(un) + c, np.sign(un) * dun + dc


def lax_friedrichs_jacobians(qL, qR, nrm, gamma):
    """(df/dqL, df/dqR), each [v, w, ...] = d f*[v] / d q[w] of lax_friedrichs; the maximum
    takes the left wave speed on ties."""
    dFL = euler_flux_jacobian(qL, gamma)
    dFR = euler_flux_jacobian(qR, gamma)
    aL, daL = _wave_speed(qL, nrm, gamma)
    aR, daR = _wave_speed(qR, nrm, gamma)
    left = aL >= aR
    lam = np.where(left, aL, aR)
    dlamL = np.where(left, daL, 0.0)
    dlamR = np.where(left, 0.0, daR)
    jump = qR - qL
    eye = np.eye(5).reshape((5, 5) + (1,) * (qL.ndim - 1))
    JL = 0.5 * normal_flux(dFL, nrm) + 0.5 * lam * eye - 0.5 * jump[:, None] * dlamL[None, :]
    JR = 0.5 * normal_flux(dFR, nrm) - 0.5 * lam * eye - 0.5 * jump[:, None] * dlamR[None, :]
    return JL, JR


def lifting_jacobian(q, gamma, Rgas):
    """dW[s, w, ...] = d (u, v, w, T)[s] / d q[w]."""
    rho = q[0]
    p = pressure(q, gamma)
    d = np.zeros((4,) + q.shape, dtype=q.dtype)
    d[0:3] = _dvelocity(q)
    d[3] = _dpressure(q, gamma) / (rho * Rgas)
    d[3, 0] = d[3, 0] - p / (rho * rho * Rgas)
    return d


def viscous_flux_jacobians(q, grad, gamma, mu, Pr, Rgas):
    """(dFv/dq [c, v, w, ...], dFv/dgrad [c, v, s, d, ...]) of viscous_flux."""
    u = q[1:4] / q[0]
    du = _dvelocity(q)
    kappa = mu * gamma * Rgas / ((gamma - 1.0) * Pr)
    shp = q.shape[1:]
    dtype = np.result_type(q, grad)
    # tau[i, c] and its derivative with respect to grad[s, d]
    div = grad[0, 0] + grad[1, 1] + grad[2, 2]
    tau = np.empty((3, 3) + shp, dtype=dtype)
    dtau = np.zeros((3, 3, 4, 3) + shp, dtype=dtype)
    for i in range(3):
        for c in range(3):
            tau[i, c] = mu * (grad[i, c] + grad[c, i])
            dtau[i, c, i, c] += mu
            dtau[i, c, c, i] += mu
            if i == c:
                tau[i, c] = tau[i, c] - mu * (2.0 / 3.0) * div
                for s in range(3):
                    dtau[i, c, s, s] -= mu * (2.0 / 3.0)
    dq = np.zeros((3, 5, 5) + shp, dtype=dtype)
    dg = np.zeros((3, 5, 4, 3) + shp, dtype=dtype)
    for c in range(3):
        for i in range(3):
            dg[c, 1 + i] = dtau[i, c]
            dq[c, 4] = dq[c, 4] + tau[i, c] * du[i]
            dg[c, 4] = dg[c, 4] + u[i] * dtau[i, c]
        dg[c, 4, 3, c] = dg[c, 4, 3, c] + kappa
    return dq, dg


# ---------------------------------------------------------------------------------------------
# Entropy-conservative two-point flux for the entropy-stable split form (Sec. 2, the paper's
# stabilisation, citing Chandrashekar 2013).  Entropy S = -rho s / (gamma - 1) with
# s = ln(p rho^-gamma); beta = rho / (2 p).
# ---------------------------------------------------------------------------------------------
def log_mean(a, b):
    """Logarithmic mean (a - b) / (ln a - ln b), = a when a = b.  The logarithm of the ratio is
    taken as log1p((a - b) / b), accurate also when a and b are close."""
    a, b = np.broadcast_arrays(a, b)
    d = a - b
    same = d == 0
    den = np.log1p(np.where(same, 1.0, d / b))
    return np.where(same, a, d / np.where(same, 1.0, den))


def entropy(q, gamma):
    """Mathematical entropy S(q) = -rho s / (gamma - 1)."""
    p = pressure(q, gamma)
    s = np.log(p) - gamma * np.log(q[0])
    return -q[0] * s / (gamma - 1.0)


def entropy_variables(q, gamma):
    """v = dS/dq: ((gamma - s)/(gamma - 1) - rho |u|^2 / (2p), rho u / p, -rho / p)."""
    rho = q[0]
    u = q[1:4] / rho
    p = pressure(q, gamma)
    s = np.log(p) - gamma * np.log(rho)
    out = np.empty_like(q, dtype=np.result_type(q, p))
    out[0] = (gamma - s) / (gamma - 1.0) - 0.5 * rho * (u[0] ** 2 + u[1] ** 2 + u[2] ** 2) / p
    out[1:4] = rho * u / p
    out[4] = -rho / p
    return out


def entropy_potential(q, nrm):
    """Entropy flux potential psi.n = rho u.n of S (the flux potential of the pair (S, F_S))."""
    return q[1] * nrm[0] + q[2] * nrm[1] + q[3] * nrm[2]


def chandrashekar_flux(qL, qR, nrm, gamma):
    """Two-point flux F#(qL, qR).n (Chandrashekar 2013): with logarithmic means rho_ln, beta_ln
    and arithmetic means (.)_avg,
        F_rho = rho_ln u_avg.n
        F_m   = rho_avg / (2 beta_avg) n + u_avg F_rho
        F_E   = (1 / (2 (gamma - 1) beta_ln) - |u|^2_avg / 2) F_rho + u_avg . F_m,
    where |u|^2_avg is the mean of the two squared speeds.  Symmetric, consistent with the Euler
    flux, and entropy conservative: (v_R - v_L).F# = psi_R - psi_L."""
    rL, rR = qL[0], qR[0]
    uL, uR = qL[1:4] / rL, qR[1:4] / rR
    pL, pR = pressure(qL, gamma), pressure(qR, gamma)
    bL, bR = 0.5 * rL / pL, 0.5 * rR / pR
    r_ln = log_mean(rL, rR)
    b_ln = log_mean(bL, bR)
    u_avg = 0.5 * (uL + uR)
    p_hat = 0.5 * (rL + rR) / (bL + bR)
    u2_avg = 0.5 * ((uL ** 2).sum(axis=0) + (uR ** 2).sum(axis=0))
    un = u_avg[0] * nrm[0] + u_avg[1] * nrm[1] + u_avg[2] * nrm[2]
    out = np.empty(np.broadcast_shapes(qL.shape, qR.shape), dtype=np.result_type(qL, qR))
    out[0] = r_ln * un
    for i in range(3):
        out[1 + i] = p_hat * nrm[i] + u_avg[i] * out[0]
    out[4] = ((0.5 / ((gamma - 1.0) * b_ln) - 0.5 * u2_avg) * out[0]
              + u_avg[0] * out[1] + u_avg[1] * out[2] + u_avg[2] * out[3])
    return out
