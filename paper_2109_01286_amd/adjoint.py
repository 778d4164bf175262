"""Gradients through many Runge-Kutta steps: a torch.autograd.Function
whose backward runs the library's hand-written adjoint step in reverse, with
checkpointing.  The steps and their adjoints run in the solver's precision:
float64, or the mixed form (float32 arithmetic, float64 states and
lambdas).

Two checkpointing schedules:

* uniform (``ckpt_every``): the forward keeps the state every ``ckpt_every``
  steps; the backward replays each segment from its checkpoint, keeping every
  step's input and two Runge-Kutta stages for that segment only, then
  reverses its steps.  Memory: nsteps/ckpt_every + 3 ckpt_every states;
  work: one extra forward pass.
* binomial (``snapshots`` = s state slots, the initial state included): the
  reversal schedule with the fewest forward steps for that memory (Griewank
  and Walther's revolve).  With t the smallest integer such that
  C(s + t, t) >= n, reversing n steps costs t n - C(s + t, t - 1) forward
  steps; the schedule splits the steps at the point that minimises
  m + cost(n - m, s - 1) + cost(m, s), recursively.  The forward pass stores
  the snapshots of the schedule's first descent, which it computes anyway.
  Memory: s states plus one step's two stages.
"""
from __future__ import annotations

import math

import torch


# ---- binomial schedule ------------------------------------------------------------
def revolve_cost(n, s):
    """Forward steps needed to reverse ``n`` steps with ``s`` state slots
    (the slot of the start state included), not counting the steps taken
    with the adjoint of each step."""
    if n <= 1:
        return 0
    if s < 1:
        raise ValueError("at least one snapshot slot (the start state) is needed")
    t = 0
    while math.comb(s + t, t) < n:
        t += 1
    return t * n - math.comb(s + t, t - 1)


def revolve_split(n, s):
    """Where the optimal schedule stores its next snapshot, 1 <= m < n (s >= 2)."""
    best_m, best_c = 1, None
    for m in range(1, n):
        c = m + revolve_cost(n - m, s - 1) + revolve_cost(m, s)
        if best_c is None or c < best_c:
            best_m, best_c = m, c
    return best_m


def revolve_spine(n, s):
    """Snapshot positions of the schedule's first descent (starting at 0)."""
    pos = [0]
    k, slots = 0, s
    while n - k > 1 and slots >= 2:
        k += revolve_split(n - k, slots)
        slots -= 1
        pos.append(k)
    return pos


class _Work:
    """Buffers and counters shared by one backward pass."""

    def __init__(self, S, dt, lam):
        self.S, self.dt = S, dt
        self.lam = lam
        self.nxt = torch.empty_like(lam)
        self.U1 = torch.empty_like(lam)
        self.U2 = torch.empty_like(lam)
        self.forward_steps = 0
        self.live = 0          # snapshots held (spine and recursion)
        self.peak = 0

    def advance(self, U, k):
        for _ in range(k):
            self.S.rk_step_stages(U, self.dt, self.U1, self.U2)
        self.forward_steps += k

    def reverse_step(self, Un):
        """lam <- adjoint of the step starting at Un."""
        U = Un.clone()
        self.S.rk_step_stages(U, self.dt, self.U1, self.U2)
        self.forward_steps += 1
        self.S.rk_step_adjoint_stages(Un, self.U1, self.U2, self.dt, self.lam, out=self.nxt)
        self.lam, self.nxt = self.nxt, self.lam


def _reverse(W, U0, n, s):
    """Reverse the ``n`` steps that start at state U0 (kept), with ``s``
    slots including U0's."""
    if n == 1:
        W.reverse_step(U0)
        return
    if s == 1:
        for i in reversed(range(n)):
            U = U0.clone()
            W.advance(U, i)
            W.reverse_step(U)
        return
    m = revolve_split(n, s)
    Um = U0.clone()
    W.advance(Um, m)
    W.live += 1
    W.peak = max(W.peak, W.live)
    _reverse(W, Um, n - m, s - 1)
    del Um
    W.live -= 1
    _reverse(W, U0, m, s)


class RKStepsRevolve(torch.autograd.Function):
    # forward steps taken by the last backward pass and the most snapshots it
    # held at once (for measurement and tests)
    last_stats = None

    @staticmethod
    def forward(ctx, U0, solver, nsteps, dt, snapshots):
        spine = revolve_spine(nsteps, snapshots)
        U = U0.detach().clone()
        U1, U2 = torch.empty_like(U), torch.empty_like(U)
        snaps = []
        for k in range(nsteps):
            if len(snaps) < len(spine) and k == spine[len(snaps)]:
                snaps.append(U.clone())
            solver.rk_step_stages(U, dt, U1, U2)
        ctx.solver, ctx.nsteps, ctx.dt, ctx.s = solver, nsteps, dt, snapshots
        ctx.spine, ctx.snaps = spine, snaps
        return U

    @staticmethod
    def backward(ctx, gU):
        W = _Work(ctx.solver, ctx.dt, gU.detach().contiguous().clone())
        spine, n = ctx.spine, ctx.nsteps
        for j in reversed(range(len(spine))):
            end = spine[j + 1] if j + 1 < len(spine) else n
            W.live = j + 1     # spine snapshots 0..j are still held
            W.peak = max(W.peak, W.live)
            _reverse(W, ctx.snaps[j], end - spine[j], ctx.s - j)
            ctx.snaps[j] = None
        RKStepsRevolve.last_stats = {"forward_steps": W.forward_steps, "peak_snapshots": W.peak}
        ctx.snaps = None
        return W.lam, None, None, None, None


# ---- uniform schedule ------------------------------------------------------------------
class RKSteps(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, solver, nsteps, dt, ckpt_every):
        U = U0.detach().clone()
        U1, U2 = torch.empty_like(U), torch.empty_like(U)
        ckpts = []
        for k in range(nsteps):
            if k % ckpt_every == 0:
                ckpts.append(U.clone())
            solver.rk_step_stages(U, dt, U1, U2)
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


def rk_steps(U0, solver, nsteps, dt, ckpt_every=20, snapshots=None):
    """U after ``nsteps`` float64 RK3 steps of size ``dt`` from U0 (internal
    order, float64 device tensor), differentiable with respect to U0.
    ``snapshots``: use the binomial schedule with that many state slots;
    otherwise checkpoints every ``ckpt_every`` steps."""
    if snapshots is not None:
        return RKStepsRevolve.apply(U0, solver, nsteps, dt, int(snapshots))
    return RKSteps.apply(U0, solver, nsteps, dt, ckpt_every)


def pressure_disk_objective(U, xy, center, radius, area, gamma=1.4):
    """J = sum_v A_v [|x_v - c| < r] p_v^2 over owned vertices (torch; U in
    internal order, ``xy``/``area`` per internal vertex, device tensors)."""
    rho, m, n, E = U[0], U[1], U[2], U[3]
    p = (gamma - 1.0) * (E - 0.5 * (m * m + n * n) / rho)
    d = xy - torch.as_tensor(center, dtype=xy.dtype, device=xy.device)
    mask = (d * d).sum(dim=1) < radius * radius
    return torch.sum(torch.where(mask, area * p * p, torch.zeros_like(p)))
