"""PyTorch autograd front end of the residual and its adjoint.

* residual(dg, U): dU/dt with backward (dR/dU)^T g by the library's adjoint kernels;
* nodal(dg, U): nodal values q = V u~ with backward V^T qbar;
* rk_solve(dg, U0, dt, n_steps, checkpoint_every): U after n LSERK4 steps; backward runs the
  reverse stage recursion with the step-start state checkpointed every `checkpoint_every`
  steps and each segment's stage states recomputed forward once;
* kinetic_energy(dg, U): sum over nodes of w J |rho u|^2 / (2 rho), differentiable.

All device work is done by libpolydg; this module only orders the calls and keeps the
checkpoints (device copies).
"""
from __future__ import annotations

import torch


class _Residual(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, dg):
        U = U.detach().contiguous()
        ctx.save_for_backward(U)
        ctx.dg = dg
        return dg.residual(U)

    @staticmethod
    def backward(ctx, g):
        (U,) = ctx.saved_tensors
        return ctx.dg.vjp(U, g.contiguous()), None


class _Nodal(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, dg):
        ctx.dg = dg
        return dg.nodal(U.detach().contiguous())

    @staticmethod
    def backward(ctx, qbar):
        return ctx.dg.nodal_adjoint(qbar), None


def rk_gradient(dg, U0, dt, n_steps, grad_final, checkpoint_every=5):
    """dJ/dU0 from dJ/dU_n through n_steps LSERK4 steps started at U0 (K = 0 at every step).

    The forward pass keeps the state at the start of every `checkpoint_every`-th step; the
    reverse pass recomputes one segment at a time from its checkpoint, keeping the input state
    of each of its stages (5 * checkpoint_every device states), and runs the reverse stages."""
    ce = max(1, int(checkpoint_every))
    K = dg.zeros_state()
    ckpts = {}
    U = U0.detach().clone()
    for step in range(n_steps):
        if step % ce == 0:
            ckpts[step] = U.clone()
        dg.rk_steps(U, K, dt, 1)
    Ubar = grad_final.detach().clone().contiguous()
    Kbar = dg.zeros_state()
    for seg in sorted(ckpts, reverse=True):
        seg_end = min(seg + ce, n_steps)
        U = ckpts[seg].clone()
        stages = []
        for _ in range(seg, seg_end):
            for s in range(5):
                stages.append(U.clone())
                dg.rk_stage(U, K, dt, s)
        for i in reversed(range(len(stages))):
            dg.rk_stage_adjoint(stages[i], Ubar, Kbar, dt, i % 5)
        del stages
    return Ubar


class _RKSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, dg, dt, n_steps, checkpoint_every):
        U0 = U0.detach().contiguous()
        ctx.save_for_backward(U0)
        ctx.args = (dg, dt, n_steps, checkpoint_every)
        U = U0.clone()
        dg.rk_steps(U, dg.zeros_state(), dt, n_steps)
        return U

    @staticmethod
    def backward(ctx, g):
        (U0,) = ctx.saved_tensors
        dg, dt, n_steps, ce = ctx.args
        return rk_gradient(dg, U0, dt, n_steps, g, ce), None, None, None, None


def residual(dg, U):
    return _Residual.apply(U, dg)


def nodal(dg, U):
    return _Nodal.apply(U, dg)


def rk_solve(dg, U0, dt, n_steps, checkpoint_every=5):
    return _RKSolve.apply(U0, dg, float(dt), int(n_steps), int(checkpoint_every))


def kinetic_energy(dg, U, wJ=None):
    q = nodal(dg, U)
    wJ = dg.node_weights() if wJ is None else wJ
    ke = 0.5 * (q[:, 1] ** 2 + q[:, 2] ** 2 + q[:, 3] ** 2) / q[:, 0]
    return (ke * wJ).sum()
