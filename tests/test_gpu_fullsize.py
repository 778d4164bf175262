"""Parity at the full workload sizes, in the configuration bench.py times:
the library computes the whole mesh (GPU weights, float64 and mixed), the
oracle computes its own weights and residual at a sample of owned vertices.
The switch is forced to the oracle's decisions on the sampled vertices'
edges; what remains is the difference of two float64 SVD/QR precomputes
(conditioning-scaled, ~1e-8 relative at most) and float32 rounding."""
import time

import numpy as np
import pytest
import torch

from oracle import scheme as osch
from paper_2109_01286_amd import inputs

from ._helpers import cancellation_scale, edge_map, lib_solver, residual_within, same_nans

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

FULL = {
    "riemann201": dict(switch="weno", w3_cap=2.0),
    "tgv513": dict(switch="smooth", mu=0.01),
    "vortex257": dict(switch="paper"),
    "shockvortex2049": dict(switch="paper", w3_cap=2.0),
    "couette": dict(switch="smooth", mu=0.1, prandtl=100.0, gas_R=20.0 / 7.0),
    "sod_circle": dict(switch="paper", w3_cap=2.0),
}


def sample_owned(m, k, seed):
    rng = np.random.default_rng(seed)
    owned = np.nonzero(m.ghost_src == -1)[0]
    return np.sort(rng.choice(owned, size=k, replace=False))


@pytest.mark.parametrize("name", list(FULL))
def test_full_size_residual_at_sampled_vertices(name):
    kw = FULL[name]
    t0 = time.time()
    m, U, prm = inputs.workload(name)
    print(f"[full] {name}: {m.nv} vertices", flush=True)
    S = lib_solver(m, 0, **kw)
    sample = sample_owned(m, 64, seed=11)
    opts = osch.Options(mu=kw.get("mu", 0.0), w3_cap=kw.get("w3_cap", 0.0),
                        prandtl=kw.get("prandtl", 0.72), gas_R=kw.get("gas_R", 1.0))
    sc = osch.Scheme(m.xy, m.tri, m.ghost_src, m.period, opts, verts=sample)
    print(f"[full] {name}: setups {time.time() - t0:.1f} s", flush=True)
    # force the library's switch to the oracle's decisions on the sample's edges
    Ut = torch.as_tensor(U)
    _, _, omask, _ = sc.edge_states(Ut, kw["switch"])
    Ud = torch.as_tensor(S.to_internal(U), device=DEV)
    _, gmask, _ = S.edge_states(Ud)
    emap = edge_map(S, sc.topo)
    lib_of_oracle = -np.ones(sc.topo.edges.shape[0], dtype=np.int64)
    lib_of_oracle[emap] = np.arange(emap.size)
    mask = gmask.cpu().numpy().copy()
    oe = sc.ew.edges
    mask[lib_of_oracle[oe]] = omask.numpy()
    flips = int(np.count_nonzero(gmask.cpu().numpy()[lib_of_oracle[oe]] != omask.numpy()))
    S.force_switch_mask(torch.as_tensor(mask, device=DEV))
    ref = sc.residual(U, kw["switch"])
    scale = cancellation_scale(sc, U, kw["switch"])
    own = np.zeros(m.nv, dtype=bool)
    own[sample] = True
    got = S.to_input(S.residual(Ud).cpu().numpy())
    q64 = residual_within(got, ref, scale, own, rel=1e-8, abs_rel=1e-12)
    wref = U[0:4, m.ghost_src == -1].mean(axis=1)
    S.set_precision("fp32", wref)
    got32 = S.to_input(S.residual(Ud).cpu().numpy())
    # float32: 1e-5 relative, plus float32 rounding of the cancelling sums
    q32 = residual_within(got32, ref, scale, own, rel=1e-5, abs_rel=1e-6)
    print(f"[full] {name}: switch flips {flips}, fp64 tolerance use {q64:.3f}, "
          f"fp32 tolerance use {q32:.3f}", flush=True)
    assert q64 <= 1.0 and q32 <= 1.0


def test_full_size_rk_step_and_dt():
    """One step of the benchmark workload: dt equals the oracle's, the
    sampled vertices' increments agree (float64)."""
    kw = FULL["shockvortex2049"]
    m, U, prm = inputs.workload("shockvortex2049")
    S = lib_solver(m, 0, **kw)
    sample = sample_owned(m, 32, seed=12)
    opts = osch.Options(w3_cap=2.0)
    sc = osch.Scheme(m.xy, m.tri, m.ghost_src, m.period, opts, verts=sample)
    Ud = torch.as_tensor(S.to_internal(U), device=DEV)
    dt = S.stable_dt(Ud, 0.3)
    odt = sc.stable_dt(U, 0.3)
    assert abs(dt.item() - odt) <= 1e-14 * odt
    R = S.to_input(S.residual(Ud).cpu().numpy())
    S.rk_step(Ud, dt)
    S.check()
    got = S.to_input(Ud.cpu().numpy())
    # first-stage consistency: the step's increment is dt times a mix of the
    # three stage residuals; its first-order part is dt * R(U)
    inc = (got - U)[:, sample]
    assert np.all(np.isfinite(inc))
    assert np.linalg.norm(inc - odt * R[:, sample]) <= 0.1 * np.linalg.norm(odt * R[:, sample]) + 1e-12
