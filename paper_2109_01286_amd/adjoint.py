"""Gradients through many Runge-Kutta steps: a torch.autograd.Function
whose backward runs the library's hand-written adjoint step
(``hfd_rk_step_adjoint``) in reverse, with checkpointing.

Forward: ``nsteps`` steps of fixed size ``dt`` from U0, keeping the state
every ``ckpt_every`` steps (float64, device).  Backward: segments in reverse;
each segment is recomputed from its checkpoint, keeping every step's input
and its two Runge-Kutta stages for the segment only, then its steps are
reversed from those.  Memory: nsteps/ckpt_every + 3 ckpt_every states; work:
one extra forward pass.
"""
from __future__ import annotations

import torch


class RKSteps(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, solver, nsteps, dt, ckpt_every):
        U = U0.detach().clone()
        ckpts = []
        for k in range(nsteps):
            if k % ckpt_every == 0:
                ckpts.append(U.clone())
            solver.rk_step(U, dt)
        ctx.solver = solver
        ctx.nsteps = nsteps
        ctx.dt = dt
        ctx.ckpt_every = ckpt_every
        ctx.ckpts = ckpts
        return U

    @staticmethod
    def backward(ctx, gU):
        S, dt, ce, n = ctx.solver, ctx.dt, ctx.ckpt_every, ctx.nsteps
        lam = gU.detach().contiguous().clone()
        nxt = torch.empty_like(lam)
        # (input, stage 1, stage 2) of every step of a segment, one buffer
        # for all segments
        buf = torch.empty((min(ce, n), 3) + tuple(lam.shape), dtype=lam.dtype,
                          device=lam.device)
        for seg in reversed(range(len(ctx.ckpts))):
            k0 = seg * ce
            k1 = min(n, k0 + ce)
            U = ctx.ckpts[seg].clone()
            for i in range(k1 - k0):
                buf[i, 0].copy_(U)
                S.rk_step_stages(U, dt, buf[i, 1], buf[i, 2])
            for i in reversed(range(k1 - k0)):
                S.rk_step_adjoint_stages(buf[i, 0], buf[i, 1], buf[i, 2], dt, lam, out=nxt)
                lam, nxt = nxt, lam
        ctx.ckpts = None
        return lam, None, None, None, None


def rk_steps(U0, solver, nsteps, dt, ckpt_every=20):
    """U after ``nsteps`` RK3 steps of size ``dt`` from U0 (internal order,
    float64 device tensor), differentiable with respect to U0."""
    return RKSteps.apply(U0, solver, nsteps, dt, ckpt_every)


def pressure_disk_objective(U, xy, center, radius, area, gamma=1.4):
    """J = sum_v A_v [|x_v - c| < r] p_v^2 over owned vertices (torch; U in
    internal order, ``xy``/``area`` per internal vertex, device tensors)."""
    rho, m, n, E = U[0], U[1], U[2], U[3]
    p = (gamma - 1.0) * (E - 0.5 * (m * m + n * n) / rho)
    d = xy - torch.as_tensor(center, dtype=xy.dtype, device=xy.device)
    mask = (d * d).sum(dim=1) < radius * radius
    return torch.sum(torch.where(mask, area * p * p, torch.zeros_like(p)))
