"""The binomial checkpointing schedule (CPU, with a stand-in solver whose
step is a nonlinear map with a known adjoint):

* the closed-form cost equals the optimum of the recursion over split points
  (brute force on small sizes);
* the gradient equals torch autograd through the same steps;
* the backward takes cost(n, s) - (forward steps of the first descent, done
  by the forward pass) + n forward steps (one per adjoint step) and never
  holds more than s snapshots.
"""
import functools

import pytest
import torch

from paper_2109_01286_amd.adjoint import (RKStepsRevolve, revolve_cost, revolve_spine,
                                          rk_steps)


@functools.lru_cache(maxsize=None)
def brute(n, s):
    if n <= 1:
        return 0
    if s == 1:
        return n * (n - 1) // 2
    return min(m + brute(n - m, s - 1) + brute(m, s) for m in range(1, n))


def test_closed_form_cost_is_the_optimum():
    for s in range(1, 6):
        for n in range(1, 40):
            assert revolve_cost(n, s) == brute(n, s), (n, s)


class Stub:
    """U <- U + dt c tanh(U) (elementwise), with its adjoint."""

    def __init__(self, c):
        self.c = c
        self.steps = 0

    def f(self, U, dt):
        return U + dt * self.c * torch.tanh(U)

    def rk_step_stages(self, U, dt, U1, U2):
        U1.copy_(U)
        U2.copy_(U)
        U.copy_(self.f(U, dt))
        self.steps += 1
        return U

    def rk_step_adjoint_stages(self, Un, U1, U2, dt, lam, out):
        assert torch.equal(U1, Un) and torch.equal(U2, Un)
        out.copy_(lam + dt * self.c * (1.0 - torch.tanh(Un) ** 2) * lam)
        return out


@pytest.mark.parametrize("n,s", [(1, 1), (2, 1), (7, 1), (7, 2), (20, 3), (45, 3), (45, 5),
                                 (64, 8)])
def test_gradient_step_count_and_memory(n, s):
    gen = torch.Generator().manual_seed(n * 10 + s)
    c = torch.randn(16, dtype=torch.float64, generator=gen)
    U0 = torch.randn(16, dtype=torch.float64, generator=gen)
    lam = torch.randn(16, dtype=torch.float64, generator=gen)
    dt = 0.1
    S = Stub(c)
    X = U0.clone().requires_grad_(True)
    Y = X
    for _ in range(n):
        Y = S.f(Y, dt)
    (ref,) = torch.autograd.grad(Y, X, lam)
    S.steps = 0
    U = U0.clone().requires_grad_(True)
    out = rk_steps(U, S, n, dt, snapshots=s)
    assert S.steps == n
    (g,) = torch.autograd.grad(out, U, lam)
    assert torch.allclose(g, ref, rtol=1e-13, atol=0.0)
    st = RKStepsRevolve.last_stats
    expect = revolve_cost(n, s) - revolve_spine(n, s)[-1] + n
    assert st["forward_steps"] == expect == S.steps - n
    assert st["peak_snapshots"] <= s
