"""Errors against closed-form solutions on the GPU, float32 (mixed form)
against float64: the vortex of Section 3.1 advected exactly, and the decaying
Taylor-Green vortex (small lattice: under the readings the viscous path of
the recipe's 513 x 513 lattice grows a mode from its second step on).  The
float32 error may be at most twice the float64 one."""
import numpy as np
import pytest
import torch

from paper_2109_01286_amd import hfd, inputs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

CASES = {
    # workload, lattice, options, steps
    "vortex21": ("vortex21", None, dict(switch="paper", w3_cap=2.0), 20),
    "tgv129": ("tgv513", 129, dict(switch="smooth", mu=0.01, prandtl=0.72, gas_R=1.0), 20),
}


def exact(key, m, t):
    if key == "vortex21":
        return inputs.isentropic_vortex(m, center=(5.0, 5.0), beta=5.0, t=t)
    return inputs.taylor_green(m, t=t, nu=0.01)


@pytest.mark.parametrize("key", list(CASES))
def test_float32_error_within_twice_float64(key):
    name, scale, kw, steps = CASES[key]
    m, U0, _ = inputs.workload(name, scale)
    S = hfd.Solver(m.xy, m.tri, m.ghost_src, m.period, device=0, **kw)
    owned = m.ghost_src == -1
    wref = U0[0:4, owned].mean(axis=1)
    err = {}
    for prec in ("fp64", "fp32"):
        S.set_precision(prec, wref)
        U = torch.as_tensor(S.to_internal(U0), device=DEV)
        dt = torch.empty(1, dtype=torch.float64, device=DEV)
        t = 0.0
        for _ in range(steps):
            S.stable_dt(U, 0.3, out=dt)
            t += dt.item()
            S.rk_step(U, dt)
        S.check()
        Uh = S.to_input(U.cpu().numpy())
        Ue = exact(key, m, t)
        err[prec] = [float(np.sqrt(np.mean((Uh[q, owned] - Ue[q, owned]) ** 2))) for q in range(4)]
    print(f"[accuracy] {key}: rho L2 fp64 {err['fp64'][0]:.4e} fp32 {err['fp32'][0]:.4e}")
    for q in range(4):
        assert np.isfinite(err["fp64"][q])
        assert err["fp32"][q] <= 2.0 * err["fp64"][q]
