"""The edge kernels and the edge reverse are compiled once per switch mode of
eq. 2d_hweno_intp: the paper's switch on omega_1, Hermite everywhere, WENO
everywhere, and a forced mask.  Where two instantiations take the same
decisions they evaluate the same formulas: a solver forced to the paper
switch's own mask, to the all-Hermite mask or to the all-WENO mask gives the
residual, the interface states and the adjoint residual of the paper,
smooth-only and WENO-only solvers to rounding (the compiler schedules each
instantiation on its own, so the operations need not be fused alike).  (The
WENO-only edge reverse writes rows of 24 instead of 72 values; the vertex
reverse reads them at that width.)"""
import numpy as np
import pytest
import torch

from paper_2109_01286_amd import hfd, inputs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

CASES = {"shockvortex": ("shockvortex2049", 25), "vortex21": ("vortex21", None),
         "riemann": ("riemann201", 25)}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("key", list(CASES))
def test_forced_masks_reproduce_each_switch_mode(key, prec):
    name, scale = CASES[key]
    print(f"[switch modes] {key} {prec}", flush=True)
    m, U, _ = inputs.workload(name, scale)
    wref = U[0:4, m.ghost_src == -1].mean(axis=1)
    rng = np.random.default_rng(3)
    lam0 = rng.standard_normal(U.shape)
    out = {}
    for sw in ("paper", "smooth", "weno", "forced"):
        S = hfd.Solver(m.xy, m.tri, m.ghost_src, m.period, device=0,
                       switch="paper" if sw == "forced" else sw, w3_cap=2.0)
        if prec == "fp32":
            S.set_precision("fp32", wref)
        Ud = torch.as_tensor(S.to_internal(U), device=DEV)
        lam = torch.as_tensor(S.to_internal(lam0), device=DEV)
        if sw == "forced":
            wlr, mask, _ = S.edge_states(Ud)
            masks = {"paper": mask, "smooth": torch.zeros_like(mask),
                     "weno": torch.full_like(mask, 0xFF)}
            for mode, mk in masks.items():
                S.force_switch_mask(mk)
                out[("forced", mode)] = (S.residual(Ud), S.edge_states(Ud)[0],
                                         S.adjoint_residual(Ud, lam))
            S.force_switch_mask(None)
        else:
            out[sw] = (S.residual(Ud), S.edge_states(Ud)[0], S.adjoint_residual(Ud, lam))
        S.close()
    # Rounding: the forward results agree to a few units of the precision;
    # the adjoint's derivatives of the WENO weights divide by (eps + beta)^3
    # and amplify it about 2000 times (measured 2e-13 in float64, 1.5e-4 in
    # float32 with WENO everywhere).  A wrong instantiation or a wrong row
    # width would differ at O(1).
    u = 1.1e-16 if prec == "fp64" else 6e-8
    for mode in ("paper", "smooth", "weno"):
        for a, b, what, tol in zip(out[mode], out[("forced", mode)],
                                   ("residual", "interface states", "adjoint residual"),
                                   (1e3 * u, 1e3 * u, 3e4 * u)):
            nan_a, nan_b = ~torch.isfinite(a), ~torch.isfinite(b)
            assert torch.equal(nan_a, nan_b), f"{key} {prec} {mode}: {what}: non-finite entries differ"
            a, b = a[~nan_a], b[~nan_b]
            rel = float((a - b).abs().max() / b.abs().max().clamp_min(1e-300))
            print(f"[switch modes] {key} {prec} {mode} {what}: max rel diff {rel:.1e}", flush=True)
            assert rel <= tol, f"{key} {prec} {mode}: {what} differs from the forced mask's"
