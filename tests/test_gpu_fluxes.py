"""GPU parity of the Riemann-flux variants (Roe with entropy fix, HLLC)
against the oracle: edge fluxes and the residual in float64 (1e-12, or the
rounding scale of cancelling fluxes) with the oracle's weights imported, the
mixed form to 1e-5 with the switch forced to the oracle's decisions, the
runtime flux switch, and the adjoint of both fluxes against autograd through
the oracle."""
import numpy as np
import pytest
import torch

from paper_2109_01286_amd import hfd, inputs

from ._helpers import (block_rel_err, cancellation_scale, lib_solver, oracle_scheme,
                       oracle_weights_for_lib, residual_within, same_nans)

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

CASES = {
    "vortex21": ("vortex21", None, {}, "paper"),
    "riemann": ("riemann201", 25, {"w3_cap": 2.0}, "weno"),
    "shockvortex": ("shockvortex2049", 25, {"w3_cap": 2.0}, "paper"),
}
FLUXES = ["roe", "hllc"]

_pairs = {}


def pair(key, flux):
    if (key, flux) not in _pairs:
        name, scale, kw, sw = CASES[key]
        print(f"[flux parity] building {key} / {flux}", flush=True)
        m, U, _ = inputs.workload(name, scale)
        sc = oracle_scheme(m, flux=flux, **kw)
        S = lib_solver(m, 0, switch=sw, flux=flux, **kw)
        ow = oracle_weights_for_lib(S, sc)
        S.import_weights(ow["w5"], ow["w3"], ow["dv"], ow["de"])
        _pairs[(key, flux)] = (m, U, sw, sc, S, ow)
    return _pairs[(key, flux)]


@pytest.mark.parametrize("key", list(CASES))
@pytest.mark.parametrize("flux", FLUXES)
def test_edge_flux_fp64(key, flux):
    m, U, sw, sc, S, ow = pair(key, flux)
    wl, wr, mask, h = sc.edge_states(torch.as_tensor(U), sw)
    _, gmask, gh = S.edge_states(torch.as_tensor(S.to_internal(U), device=DEV))
    pos = ow["pos"]
    assert np.array_equal(gmask.cpu().numpy(), mask.numpy()[pos])
    a, b = gh.cpu().numpy(), h.numpy()[pos].T
    f = same_nans(a, b)
    err = np.linalg.norm((a - b)[f]) / np.linalg.norm(b[f])
    print(f"[flux parity] {key}/{flux}: edge flux rel err {err:.2e}")
    assert err <= 1e-12


@pytest.mark.parametrize("key", list(CASES))
@pytest.mark.parametrize("flux", FLUXES)
def test_residual_fp64(key, flux):
    m, U, sw, sc, S, ow = pair(key, flux)
    owned = m.ghost_src == -1
    ref = sc.residual(U, sw)
    got = S.to_input(S.residual(torch.as_tensor(S.to_internal(U), device=DEV)).cpu().numpy())
    q = residual_within(got, ref, cancellation_scale(sc, U, sw), owned)
    print(f"[flux parity] {key}/{flux}: residual rel err {block_rel_err(got, ref, owned):.2e}")
    assert q <= 1.0


@pytest.mark.parametrize("key", list(CASES))
@pytest.mark.parametrize("flux", FLUXES)
def test_residual_mixed(key, flux):
    m, U, sw, sc, S, ow = pair(key, flux)
    owned = m.ghost_src == -1
    _, _, mask, _ = sc.edge_states(torch.as_tensor(U), sw)
    ref = sc.residual(U, sw)
    S.set_precision("fp32", U[0:4, owned].mean(axis=1))
    try:
        S.force_switch_mask(torch.as_tensor(mask.numpy()[ow["pos"]], device=DEV))
        got = S.to_input(S.residual(torch.as_tensor(S.to_internal(U), device=DEV)).cpu().numpy())
        err = block_rel_err(got, ref, owned)
        print(f"[flux parity] {key}/{flux}: mixed residual rel err {err:.2e}")
        assert err <= 1e-5
    finally:
        S.force_switch_mask(None)
        S.set_precision("fp64")


def test_runtime_flux_switch_equals_created_flux():
    m, U, sw, sc, S, ow = pair("shockvortex", "hllc")
    T = lib_solver(m, 0, switch=sw, w3_cap=2.0)
    T.import_weights(ow["w5"], ow["w3"], ow["dv"], ow["de"])
    Ud = torch.as_tensor(S.to_internal(U), device=DEV)
    T.set_flux("hllc")
    assert torch.equal(T.residual(Ud), S.residual(Ud))
    T.set_flux("rusanov")
    assert not torch.equal(T.residual(Ud), S.residual(Ud))
    with pytest.raises(hfd.HfdError) as e:
        T.set_flux(7)
    assert e.value.status == 1


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("key", ["vortex21", "shockvortex"])
@pytest.mark.parametrize("flux", FLUXES)
def test_adjoint_residual_matches_autograd(key, flux):
    """The adjoint differentiates the Roe and HLLC fluxes by dual numbers
    through the branches they take: against autograd through the oracle,
    switch pinned to the oracle's decisions."""
    m, U, sw, sc, S, ow = pair(key, flux)
    _, _, mask, _ = sc.edge_states(torch.as_tensor(U), sw)
    S.force_switch_mask(torch.as_tensor(mask.numpy()[ow["pos"]], device=DEV))
    try:
        rng = np.random.default_rng(13)
        lam = rng.standard_normal(U.shape)
        lam[:, m.ghost_src != -1] = 0.0
        Ut = torch.tensor(U, requires_grad=True)
        (ref,) = torch.autograd.grad(sc.residual(Ut, sw), Ut, torch.as_tensor(lam))
        ref = ref.numpy()
        owned = m.ghost_src == -1
        got = S.to_input(S.adjoint_residual(torch.as_tensor(S.to_internal(U), device=DEV),
                                            torch.as_tensor(S.to_internal(lam), device=DEV))
                         .cpu().numpy())
        err = rel(got[:, owned], ref[:, owned])
        print(f"[flux adjoint] {key}/{flux}: rel err vs autograd {err:.2e}")
        assert np.all(got[:, ~owned] == 0.0)
        assert err < 1e-10
    finally:
        S.force_switch_mask(None)


@pytest.mark.parametrize("flux", FLUXES)
def test_rk_step_adjoint_matches_autograd(flux):
    m, U, sw, sc, S, ow = pair("shockvortex", flux)
    dt = sc.stable_dt(U, 0.3)
    rng = np.random.default_rng(14)
    lam = rng.standard_normal(U.shape)
    Ut = torch.tensor(U, requires_grad=True)
    U1 = sc.rk3_step(Ut, dt, sw)
    (ref,) = torch.autograd.grad(U1, Ut, torch.as_tensor(lam))
    ref = ref.numpy()
    Ud = torch.as_tensor(S.to_internal(U), device=DEV)
    got = S.to_input(S.rk_step_adjoint(Ud, dt, torch.as_tensor(S.to_internal(lam), device=DEV))
                     .cpu().numpy())
    # both sides took the same branches at every stage
    U1g = Ud.clone()
    S.rk_step(U1g, dt)
    assert np.abs(S.to_input(U1g.cpu().numpy()) - U1.detach().numpy()).max() < 1e-10
    owned = m.ghost_src == -1
    err = rel(got[:, owned], ref[:, owned])
    print(f"[flux adjoint] shockvortex/{flux} rk step: rel err vs autograd {err:.2e}")
    assert err < 1e-10
