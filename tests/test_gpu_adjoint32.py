"""The float32 adjoint of the mixed form (float32 arithmetic on the mixed
form's own stage states, float64 accumulation of lambda across the
Runge-Kutta stages) against the float64 adjoint, which the float64 tests
pin to autograd through the oracle and to central differences.  Central
differences of the float32 forward are not used: its rounding (1e-7
relative) over any usable step swamps them."""
import numpy as np
import pytest
import torch

from paper_2109_01286_amd import inputs

from ._helpers import lib_solver

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

CASES = {
    "vortex21": ("vortex21", None, {"w3_cap": 2.0}, "smooth"),
    "vortex21-paper": ("vortex21", None, {"w3_cap": 2.0}, "paper"),
    "shockvortex": ("shockvortex2049", 17, {"w3_cap": 2.0}, "paper"),
    "tgv": ("tgv513", 17, {"mu": 0.01}, "smooth"),
    "couette": ("couette", 31, {"mu": 0.1, "prandtl": 100.0, "gas_R": 20.0 / 7.0}, "smooth"),
}


def rel(a, b):
    return float(torch.linalg.norm(a - b) / torch.linalg.norm(b))


def solver(key, flux="rusanov"):
    name, scale, kw, sw = CASES[key]
    m, U, _ = inputs.workload(name, scale)
    S = lib_solver(m, 0, switch=sw, flux=flux, **kw)
    wref = U[0:4, m.ghost_src == -1].mean(axis=1)
    return m, U, S, wref


# HLLC is checked on the diagonal vortex flow only.  Its flux is not
# differentiable where the contact speed S_M is 0 (continuous there, its
# derivative jumps between the two star regions).  In the shock-vortex state
# S_M is exactly 0 on every edge normal to the uniform flow outside the
# vortex; float32 rounding of the interface states puts those edges on either
# side, so the two precisions differentiate different one-sided branches
# there.
@pytest.mark.parametrize("key,flux", [(k, "rusanov") for k in CASES] +
                         [("shockvortex", "roe"), ("vortex21-paper", "roe"),
                          ("vortex21-paper", "hllc")])
def test_fp32_adjoint_residual_close_to_fp64(key, flux):
    """J^T lam at the same state in both precisions, the switch pinned to
    the float64 decisions so that both differentiate the same branches."""
    m, U, S, wref = solver(key, flux)
    Ud = torch.as_tensor(S.to_internal(U), device=DEV)
    rng = np.random.default_rng(11)
    lam = torch.as_tensor(S.to_internal(rng.standard_normal(U.shape)), device=DEV)
    _, mask, _ = S.edge_states(Ud)
    S.force_switch_mask(mask)
    ref = S.adjoint_residual(Ud, lam)
    S.set_precision("fp32", wref)
    got = S.adjoint_residual(Ud, lam)
    S.force_switch_mask(None)
    owned = torch.as_tensor(S.to_internal((m.ghost_src == -1).astype(np.float64)[None])[0],
                            device=DEV) > 0
    err = max(rel(got[4 * k:4 * k + 4][:, owned], ref[4 * k:4 * k + 4][:, owned]) for k in range(3))
    print(f"[adjoint32] {key}/{flux}: adjoint residual rel err per block (max) {err:.2e}")
    assert torch.all(got[:, ~owned] == 0.0)
    assert err < 1e-4


def test_fp32_saved_stages_equal_recompute():
    """In the mixed form rk_step_stages returns rk_step's state and stages,
    and the adjoint step from them equals the one that recomputes them."""
    m, U, S, wref = solver("shockvortex")
    S.set_precision("fp32", wref)
    Ud = torch.as_tensor(S.to_internal(U), device=DEV)
    dt = S.stable_dt(Ud, 0.3).item()
    rng = np.random.default_rng(12)
    lam = torch.as_tensor(S.to_internal(rng.standard_normal(U.shape)), device=DEV)
    X, Y = Ud.clone(), Ud.clone()
    U1, U2 = torch.empty_like(Ud), torch.empty_like(Ud)
    S.rk_step(X, dt)
    S.rk_step_stages(Y, dt, U1, U2)
    assert torch.equal(X, Y)
    a = S.rk_step_adjoint(Ud, dt, lam)
    b = S.rk_step_adjoint_stages(Ud, U1, U2, dt, lam)
    assert torch.equal(a, b)


@pytest.mark.parametrize("snapshots", [None, 3])
def test_fp32_gradient_through_steps_close_to_fp64(snapshots):
    """dJ/dU0 of the pressure-disk objective after 12 steps (checkpoints every
    5 steps, or the binomial schedule with 3 slots), float32 against float64:
    within 1e-3 relative (the two forward trajectories differ by float32
    rounding, ~1e-6)."""
    from paper_2109_01286_amd.adjoint import pressure_disk_objective, rk_steps
    m, U, S, wref = solver("vortex21")
    Ud0 = torch.as_tensor(S.to_internal(U), device=DEV)
    dt = 0.5 * S.stable_dt(Ud0, 0.3).item()
    xy = torch.as_tensor(m.xy[S.old_of_new], device=DEV)
    area = torch.as_tensor(inputs.vertex_areas(m)[S.old_of_new], device=DEV)
    grads, Js = {}, {}
    for prec in ("fp64", "fp32"):
        S.set_precision(prec, wref)
        U0d = Ud0.clone().requires_grad_(True)
        kw = dict(snapshots=snapshots) if snapshots else dict(ckpt_every=5)
        J = pressure_disk_objective(rk_steps(U0d, S, 12, dt, **kw), xy, (7.0, 7.0), 1.5, area)
        (g,) = torch.autograd.grad(J, U0d)
        grads[prec], Js[prec] = g, J.item()
    err = rel(grads["fp32"], grads["fp64"])
    print(f"[adjoint32] 12-step gradient fp32 vs fp64: rel err {err:.2e}, "
          f"J rel diff {abs(Js['fp32'] - Js['fp64']) / abs(Js['fp64']):.2e}")
    assert abs(Js["fp32"] - Js["fp64"]) <= 1e-5 * abs(Js["fp64"])
    assert err < 1e-3
