"""The passes that stage data in LDS (the vertex pass each block's distinct
state rows and edge fluxes, the edge passes each 128-edge block's distinct
stencil rows, the edge reverse each 128-edge block's distinct lambda rows)
give the same bits as the passes that gather every slot and node from HBM
(only where the data is read from differs, not the arithmetic): the
residual, the adjoint residual and Runge-Kutta steps, float64 and mixed,
Euler and viscous, the three switch modes of the workloads, small instances
of every workload and the full-size shock-vortex mesh."""
import pytest
import torch

from paper_2109_01286_amd import inputs

from ._helpers import lib_solver

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

CASES = [("vortex21", None), ("riemann201", 61), ("tgv513", 65), ("couette", 41),
         ("sod_circle", 41), ("shockvortex2049", 65), ("vortex21", 7), ("riemann201", 6)]


def options(name, prm):
    kw = dict(switch=prm["switch"], mu=prm.get("mu", 0.0), gamma=prm["gamma"])
    if prm.get("mu", 0.0) > 0:
        kw.update(prandtl=prm["prandtl"], gas_R=prm["gas_R"])
    if prm["switch"] == "paper":
        kw["w3_cap"] = 2.0   # bounded 3-node weights, as every Euler run here
    return kw


def staged_and_gathered(name, scale, prec):
    m, U, prm = inputs.workload(name, scale)
    kw = options(name, prm)
    A = lib_solver(m, 0, **kw)
    B = lib_solver(m, 0, stage_off=1, **kw)
    if prec == "fp32":
        wref = U[0:4, m.ghost_src == -1].mean(axis=1)
        A.set_precision("fp32", wref)
        B.set_precision("fp32", wref)
    assert A.info["stage_idx_bytes"] in (1, 2)
    assert B.info["stage_idx_bytes"] == 0
    return A, B, torch.as_tensor(A.to_internal(U), device=DEV)


def same_bits(a, b):
    return torch.equal(a.view(torch.int64), b.view(torch.int64))


def mostly_finite(x):
    # (the quadrant and shock cases carry a few non-finite entries where the
    # method breaks down, in the oracle as well; they must match bit for bit)
    return torch.isfinite(x).double().mean().item() > 0.9


def check(A, B, Ud, steps=2, stable=True):
    ra, rb = A.residual(Ud), B.residual(Ud)
    assert mostly_finite(ra)
    assert same_bits(ra, rb)
    gen = torch.Generator(device="cpu").manual_seed(5)
    lam = torch.randn(Ud.shape, generator=gen, dtype=torch.float64).to(DEV)
    ga, gb = A.adjoint_residual(Ud, lam), B.adjoint_residual(Ud, lam)
    assert same_bits(ga, gb)
    dt = A.stable_dt(Ud, 0.3)
    Ua, Ub = Ud.clone(), Ud.clone()
    for _ in range(steps):
        A.rk_step(Ua, dt)
        B.rk_step(Ub, dt)
    if stable:
        assert mostly_finite(Ua)
    assert same_bits(Ua, Ub)


@pytest.mark.parametrize("name,scale", CASES)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_stage_matches_gather_bitwise(name, scale, prec):
    print(f"[stage] {name} scale={scale} {prec}", flush=True)
    A, B, Ud = staged_and_gathered(name, scale, prec)
    # the quadrant and circular-Sod states break down within a few steps
    # under the readings (identically on both paths)
    check(A, B, Ud, stable=name not in ("riemann201", "sod_circle"))


def test_stage_matches_gather_full_size():
    print("[stage] shockvortex2049 full size fp32", flush=True)
    A, B, Ud = staged_and_gathered("shockvortex2049", None, "fp32")
    print(f"[stage] local ids of {A.info['stage_idx_bytes']} byte(s), lists up to "
          f"{A.info['stage_max_rows']} rows and {A.info['stage_max_edges']} edges", flush=True)
    check(A, B, Ud, steps=1)
