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
