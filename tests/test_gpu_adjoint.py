"""GPU adjoint (hand-written, float64) against (i) torch autograd through
the CPU oracle and (ii) central finite differences of the GPU residual."""
import numpy as np
import pytest
import torch

from paper_2109_01286_amd import inputs

from ._helpers import lib_solver, oracle_scheme, oracle_weights_for_lib

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

CASES = {
    "vortex21": ("vortex21", None, {}, "paper"),
    "vortex21-weno": ("vortex21", None, {"w3_cap": 2.0}, "weno"),
    "shockvortex": ("shockvortex2049", 17, {"w3_cap": 2.0}, "paper"),
    "tgv": ("tgv513", 17, {"mu": 0.01}, "smooth"),
    "couette": ("couette", 31, {"mu": 0.1, "prandtl": 100.0, "gas_R": 20.0 / 7.0}, "smooth"),
    # smallest meshes: 36 owned vertices (a partial vertex block), fewer edges
    # than one block of the edge reverse; periodic, and with ghost regions
    "tiny": ("vortex21", 7, {"w3_cap": 2.0}, "paper"),
    "tiny_ghost": ("riemann201", 6, {"w3_cap": 2.0}, "weno"),
}


def setup_case(key, force=True, switch=None):
    """Oracle and library on one mesh, the oracle's weights imported.  With
    ``force`` the library's switch is pinned to the oracle's decisions at U
    (valid for one residual evaluation; a Runge-Kutta step re-decides at
    every stage on both sides)."""
    name, scale, kw, sw = CASES[key]
    sw = switch or sw
    m, U, _ = inputs.workload(name, scale)
    sc = oracle_scheme(m, **kw)
    S = lib_solver(m, 0, switch=sw, **kw)
    ow = oracle_weights_for_lib(S, sc)
    S.import_weights(ow["w5"], ow["w3"], ow["dv"], ow["de"], ow["dvis"])
    if force:
        _, _, mask, _ = sc.edge_states(torch.as_tensor(U), sw)
        S.force_switch_mask(torch.as_tensor(mask.numpy()[ow["pos"]], device=DEV))
    return m, U, sc, S, sw


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("key", list(CASES))
def test_adjoint_residual_matches_autograd(key):
    m, U, sc, S, sw = setup_case(key)
    rng = np.random.default_rng(3)
    lam = rng.standard_normal(U.shape)
    lam[:, m.ghost_src != -1] = 0.0
    Ut = torch.tensor(U, requires_grad=True)
    R = sc.residual(Ut, sw)
    (ref,) = torch.autograd.grad(R, Ut, torch.as_tensor(lam))
    ref = ref.numpy()
    # the oracle's derivative w.r.t. ghost rows: copies were moved onto
    # their sources by the ghost fill; Dirichlet data are not differentiated
    owned = m.ghost_src == -1
    Ud = torch.as_tensor(S.to_internal(U), device=DEV)
    ld = torch.as_tensor(S.to_internal(lam), device=DEV)
    got = S.to_input(S.adjoint_residual(Ud, ld).cpu().numpy())
    assert np.all(got[:, ~owned] == 0.0)
    err = rel(got[:, owned], ref[:, owned])
    print(f"[adjoint] {key}: rel err vs autograd {err:.2e}")
    assert err < 1e-10
    if "mu" in CASES[key][2]:
        # the viscous rows carry a visible part of the adjoint: the inviscid
        # adjoint on the same weights is far from the reference
        kw = {k: v for k, v in CASES[key][2].items() if k not in ("mu", "prandtl", "gas_R")}
        S0 = lib_solver(m, 0, switch=sw, **kw)
        ow = oracle_weights_for_lib(S0, sc)
        S0.import_weights(ow["w5"], ow["w3"], ow["dv"], ow["de"])
        inv = S0.to_input(S0.adjoint_residual(torch.as_tensor(S0.to_internal(U), device=DEV),
                                              torch.as_tensor(S0.to_internal(lam), device=DEV)).cpu().numpy())
        share = rel(inv[:, owned], ref[:, owned])
        print(f"[adjoint] {key}: inviscid adjoint differs by {share:.2e}")
        assert share > 1e-3


@pytest.mark.parametrize("key", ["vortex21", "tgv"])
def test_adjoint_dot_product_with_finite_differences(key):
    """<lam, (R(U + e d) - R(U - e d)) / 2e> = <J^T lam, d> on the GPU, 32
    seeded directions, on the smooth branch, inviscid and viscous (central differences through the
    WENO weights alpha = d/(1e-6 + beta)^2 are not accurate at any step size;
    those branches are checked against autograd above).  The step is 1e-8
    of each component's scale: the FD error falls linearly with the step down
    to rounding (kinks of |u.n| and of the maximum in the Rusanov flux are
    crossed with a probability proportional to it), ~1e-7 here."""
    m, U, sc, S, sw = setup_case(key, force=False, switch="smooth")
    rng = np.random.default_rng(4)
    owned = m.ghost_src == -1
    Ud = torch.as_tensor(S.to_internal(U), device=DEV)
    lam = torch.as_tensor(S.to_internal(rng.standard_normal(U.shape)), device=DEV)
    JTl = S.adjoint_residual(Ud, lam)
    fds, ads = [], []
    for k in range(32):
        d = torch.as_tensor(S.to_internal(rng.standard_normal(U.shape) * np.abs(U).max(axis=1, keepdims=True)),
                            device=DEV)
        eps = 1e-8
        Rp = S.residual(Ud + eps * d)
        Rm = S.residual(Ud - eps * d)
        fds.append(float(torch.sum(lam * (Rp - Rm)) / (2 * eps)))
        ads.append(float(torch.sum(JTl * d)))
    fds, ads = np.array(fds), np.array(ads)
    # relative to the typical directional derivative (a single random
    # direction can make <J^T lam, d> small by cancellation)
    errs = np.abs(fds - ads) / np.sqrt(np.mean(ads ** 2))
    print(f"[adjoint] {key} FD directional errors: max {errs.max():.2e}, median {np.median(errs):.2e}")
    assert errs.max() < 1e-6


@pytest.mark.parametrize("key", ["vortex21-weno", "shockvortex", "tgv", "couette", "tiny_ghost"])
def test_rk_step_adjoint_matches_autograd(key):
    m, U, sc, S, sw = setup_case(key, force=False)
    dt = sc.stable_dt(U, 0.3)
    rng = np.random.default_rng(5)
    lam = rng.standard_normal(U.shape)
    Ut = torch.tensor(U, requires_grad=True)
    U1 = sc.rk3_step(Ut, dt, sw)
    (ref,) = torch.autograd.grad(U1, Ut, torch.as_tensor(lam))
    ref = ref.numpy()
    Ud = torch.as_tensor(S.to_internal(U), device=DEV)
    ld = torch.as_tensor(S.to_internal(lam), device=DEV)
    got = S.to_input(S.rk_step_adjoint(Ud, dt, ld).cpu().numpy())
    # both sides took the same branches at every stage
    U1g = Ud.clone()
    S.rk_step(U1g, dt)
    assert np.abs(S.to_input(U1g.cpu().numpy()) - U1.detach().numpy()).max() < 1e-10
    owned = m.ghost_src == -1
    dirich = m.ghost_src == -2
    err = rel(got[:, owned], ref[:, owned])
    print(f"[adjoint] {key} rk step: rel err vs autograd {err:.2e}")
    assert err < 1e-10
    # Dirichlet data pass through; the oracle's gradient there also holds the
    # residual's dependence on them, which the library leaves out
    assert np.array_equal(got[:, dirich], lam[:, dirich])
    assert np.all(got[:, m.ghost_src >= 0] == 0.0)


def test_adjoint_from_saved_stages_equals_recompute():
    """rk_step_stages returns the state of rk_step and its two stages; the
    adjoint step from those stages is the adjoint step that recomputes them,
    bit for bit (same kernels, same inputs)."""
    m, U, sc, S, sw = setup_case("shockvortex", force=False)
    dt = sc.stable_dt(U, 0.3)
    rng = np.random.default_rng(7)
    Ud = torch.as_tensor(S.to_internal(U), device=DEV)
    lam = torch.as_tensor(S.to_internal(rng.standard_normal(U.shape)), device=DEV)
    X, Y = Ud.clone(), Ud.clone()
    U1, U2 = torch.empty_like(Ud), torch.empty_like(Ud)
    S.rk_step(X, dt)
    S.rk_step_stages(Y, dt, U1, U2)
    assert torch.equal(X, Y)
    a = S.rk_step_adjoint(Ud, dt, lam)
    b = S.rk_step_adjoint_stages(Ud, U1, U2, dt, lam)
    assert torch.equal(a, b)


def test_binomial_checkpointing_equals_uniform():
    """The binomial schedule (3 snapshot slots) and the uniform one run the
    same float64 steps and adjoint steps: the gradients agree bit for bit."""
    from paper_2109_01286_amd.adjoint import RKStepsRevolve, revolve_cost, revolve_spine, rk_steps
    m, U, sc, S, sw = setup_case("vortex21", force=False, switch="smooth")
    dt = 0.5 * sc.stable_dt(U, 0.3)
    rng = np.random.default_rng(8)
    lam = torch.as_tensor(S.to_internal(rng.standard_normal(U.shape)), device=DEV)
    grads = []
    for kw in (dict(ckpt_every=5), dict(snapshots=3)):
        U0 = torch.as_tensor(S.to_internal(U), device=DEV).requires_grad_(True)
        out = rk_steps(U0, S, 12, dt, **kw)
        (g,) = torch.autograd.grad(out, U0, lam)
        grads.append(g)
    assert torch.equal(grads[0], grads[1])
    st = RKStepsRevolve.last_stats
    assert st["forward_steps"] == revolve_cost(12, 3) - revolve_spine(12, 3)[-1] + 12
    assert st["peak_snapshots"] <= 3


def test_gradient_through_steps_with_checkpoints():
    """rk_steps (checkpointed, hand-written adjoint) against autograd through
    the oracle's steps and against central differences of the GPU forward,
    smooth branch, 12 steps, checkpoints every 5 steps (partial segment)."""
    from paper_2109_01286_amd.adjoint import pressure_disk_objective, rk_steps
    m, U, sc, S, sw = setup_case("vortex21", force=False, switch="smooth")
    dt = 0.5 * sc.stable_dt(U, 0.3)
    nsteps = 12
    xy = torch.as_tensor(m.xy[S.old_of_new], device=DEV)
    area = torch.as_tensor(inputs.vertex_areas(m)[S.old_of_new], device=DEV)

    def J_gpu(U0d):
        return pressure_disk_objective(rk_steps(U0d, S, nsteps, dt, 5), xy, (7.0, 7.0), 1.5, area)

    U0d = torch.as_tensor(S.to_internal(U), device=DEV).requires_grad_(True)
    J = J_gpu(U0d)
    (g,) = torch.autograd.grad(J, U0d)
    g = S.to_input(g.cpu().numpy())
    # oracle: autograd through its own steps
    Ut = torch.tensor(U, requires_grad=True)
    X = Ut
    for _ in range(nsteps):
        X = sc.rk3_step(X, dt, sw)
    xo = torch.as_tensor(m.xy)
    ao = torch.as_tensor(inputs.vertex_areas(m))
    Jo = pressure_disk_objective(X, xo, (7.0, 7.0), 1.5, ao)
    (go,) = torch.autograd.grad(Jo, Ut)
    go = go.numpy()
    assert abs(J.item() - Jo.item()) <= 1e-12 * abs(Jo.item())
    err = rel(g, go)
    print(f"[adjoint] {nsteps}-step gradient vs oracle autograd: rel err {err:.2e}")
    assert err < 1e-10
    # central differences of the GPU forward in 8 seeded directions
    rng = np.random.default_rng(6)
    errs = []
    with torch.no_grad():
        for k in range(8):
            d = rng.standard_normal(U.shape) * np.abs(U).max(axis=1, keepdims=True)
            dd = torch.as_tensor(S.to_internal(d), device=DEV)
            eps = 1e-7
            Jp = J_gpu(U0d.detach() + eps * dd).item()
            Jm = J_gpu(U0d.detach() - eps * dd).item()
            fd = (Jp - Jm) / (2 * eps)
            ad = float(np.sum(g * d))
            errs.append(abs(fd - ad) / abs(ad))
    print(f"[adjoint] {nsteps}-step gradient FD errors: max {max(errs):.2e}")
    assert max(errs) < 1e-6


def test_imported_viscous_rows_reach_the_adjoint():
    """Importing only the viscous rows after the adjoint's first call refreshes
    its transposed copy: the result equals that of a fresh context which
    imported the same rows before its first call (bit for bit)."""
    m, U, _ = inputs.workload("tgv513", 9)
    rng = np.random.default_rng(21)
    lam = rng.standard_normal(U.shape)
    A = lib_solver(m, 0, switch="smooth", mu=0.01)
    B = lib_solver(m, 0, switch="smooth", mu=0.01)
    dvis = 2.0 * A.export_weights()["dvis"]
    Ud = torch.as_tensor(A.to_internal(U), device=DEV)
    ld = torch.as_tensor(A.to_internal(lam), device=DEV)
    first = A.adjoint_residual(Ud, ld)
    A.import_weights(dvis=dvis)
    again = A.adjoint_residual(Ud, ld)
    B.import_weights(dvis=dvis)
    ref = B.adjoint_residual(Ud, ld)
    assert not torch.equal(first, again)
    assert torch.equal(again, ref)
