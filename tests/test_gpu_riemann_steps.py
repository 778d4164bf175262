"""The 2D Riemann case (four quadrant states, 201 x 201, transmissive ghost
regions) marched ten Runge-Kutta steps with WENO everywhere, the HLLC flux
and capped 3-node weights at CFL 0.03, in float64 and in the float32 mixed
form (the float32 run takes the float64 run's time steps): both stay finite
with positive density and pressure, and the float32 state and its residual
agree with the float64 ones per block (w, w_x, w_y)."""
import pytest
import torch

from paper_2109_01286_amd import hfd, inputs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _positive(S, U):
    rho, mx, my, E = U[0:4, :S.n_owned]
    p = 0.4 * (E - 0.5 * (mx * mx + my * my) / rho)
    return bool(torch.isfinite(U[:, :S.n_owned]).all() and (rho > 0).all() and (p > 0).all())


def test_riemann_ten_steps_float32_against_float64():
    m, U0, prm = inputs.workload("riemann201", None)
    S = hfd.Solver(m.xy, m.tri, m.ghost_src, m.period, device=0, switch="weno",
                   w3_cap=2.0, flux="hllc")
    print(f"[riemann201] {m.nv} vertices, weno, hllc, cfl 0.03, 10 steps", flush=True)
    U64 = torch.as_tensor(S.to_internal(U0), device=DEV)
    dts = []
    for _ in range(10):
        dts.append(S.stable_dt(U64, 0.03).item())
        S.rk_step(U64, dts[-1])
        assert _positive(S, U64)
    R64 = S.residual(U64)
    S.set_precision("fp32", U0[0:4, m.ghost_src == -1].mean(axis=1))
    U32 = torch.as_tensor(S.to_internal(U0), device=DEV)
    for dt in dts:
        S.rk_step(U32, dt)
        assert _positive(S, U32)
    R32 = S.residual(U64)
    own = slice(0, S.n_owned)
    for k in range(3):
        b = slice(4 * k, 4 * k + 4)
        ds = float(torch.linalg.norm(U32[b, own] - U64[b, own]) / torch.linalg.norm(U64[b, own]))
        dr = float(torch.linalg.norm(R32[b, own] - R64[b, own]) / torch.linalg.norm(R64[b, own]))
        print(f"[riemann201] block {k}: state {ds:.2e}, residual {dr:.2e}", flush=True)
        # 1e-5: the float32 tolerance of the residual (measured: state
        # 8e-9 / 2.1e-6 / 2.1e-6, residual 2.0e-6 / 2.8e-6 / 2.7e-6)
        assert ds < 1e-5 and dr < 1e-5, (k, ds, dr)
