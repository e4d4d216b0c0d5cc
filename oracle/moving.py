"""Moving meshes: the modal time stepping of Alg. 1 with a Jacobian that changes in time.

Test infrastructure of the oracle.  The paper projects onto the modes with M = V^T W J V and
notes that this cannot be precomputed when the Jacobian changes in time (Alg. 1).  Here every
element corner follows a prescribed motion

    x(t) = x0 + d sin(omega t),   xdot(t) = d omega cos(omega t)

(d [n_elems][8][3] per corner; images of a periodic vertex move alike when d is a periodic
function of x0), and each element moves with the trilinear interpolation of its corners.  The
weak form of Eq. (1) on the moving element (arbitrary Lagrangian-Eulerian form) is

    d/dt (M u~) = r(u~, t):   the flux relative to the moving grid, F - q xdot, in the volume
                              term and the LF flux through the moving faces,

written as M du~/dt = r - (dM/dt) u~ with dM/dt u~ = V^T W (dJ/dt q), so the state stays the
modal coefficients (hexahedra: nodal values) and LSERK4 advances it as on a fixed mesh, every
stage with the geometry, M and dJ/dt at its own time t + c_s dt.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .dg import DGOracle, LSERK_A, LSERK_B, LSERK_C


class MovingDG:
    """DG residual and LSERK4 steps on a mesh whose corners move as x0 + d sin(omega t)."""

    def __init__(self, mesh, N, disp, omega, **kw):
        self.mesh0 = mesh
        self.N = int(N)
        self.disp = np.asarray(disp, dtype=np.float64)
        if self.disp.shape != mesh.corner_xyz.shape:
            raise ValueError("disp must have the shape of corner_xyz")
        self.omega = float(omega)
        self.kw = kw

    def mesh_at(self, t):
        xyz = self.mesh0.corner_xyz + self.disp * np.sin(self.omega * t)
        return dataclasses.replace(self.mesh0, corner_xyz=xyz)

    def at(self, t) -> DGOracle:
        """The oracle of the mesh at time t, with the grid velocity of that instant."""
        return DGOracle(self.mesh_at(t), self.N,
                        corner_velocity=self.disp * (self.omega * np.cos(self.omega * t)), **self.kw)

    def residual(self, U, t):
        return self.at(t).residual(U)

    def rk_steps(self, U, t0, dt, n_steps, K=None):
        """n_steps of LSERK4 from time t0; stage s of step i takes the mesh at t0 + (i + c_s) dt."""
        U = np.array(U, dtype=float)
        K = np.zeros_like(U) if K is None else np.array(K, dtype=float)
        for i in range(n_steps):
            for s in range(5):
                K = LSERK_A[s] * K + self.residual(U, t0 + (i + LSERK_C[s]) * dt)
                U = U + dt * LSERK_B[s] * K
        return U, K
