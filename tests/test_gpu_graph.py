"""Runge-Kutta steps captured in a HIP graph (Solver.capture_steps) and
replayed: every replay gives the eager steps' states and step sizes bit for
bit (the same kernels on the same data), also with eager work, host
synchronisations and a change of the state between replays.  The library
records no memset or copy in the graph: a chunk of steps is kernels only."""
import numpy as np
import pytest
import torch

from paper_2109_01286_amd import hfd, inputs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name,scale,sw", [("vortex21", None, "paper"),
                                           ("shockvortex2049", 33, "paper"),
                                           ("tgv513", 17, "smooth")])
def test_graph_replays_equal_eager_steps(name, scale, sw, prec):
    print(f"[graph] {name} {scale} {prec}", flush=True)
    m, U0, _ = inputs.workload(name, scale)
    kw = {"mu": 0.01} if name == "tgv513" else {"w3_cap": 2.0}
    S = hfd.Solver(m.xy, m.tri, m.ghost_src, m.period, device=0, switch=sw, **kw)
    if prec == "fp32":
        S.set_precision("fp32", U0[0:4, m.ghost_src == -1].mean(axis=1))
    X0 = torch.as_tensor(S.to_internal(U0), device=DEV)
    n = 3
    # eager reference: three chunks of n steps from X0
    E = X0.clone()
    ref = []
    for _ in range(3):
        d = S.rk_steps(E, n, 0.3)
        ref.append((E.clone(), d.clone()))
    torch.cuda.synchronize()
    # graph on its own buffers
    U = X0.clone()
    dts = torch.zeros(n, dtype=torch.float64, device=DEV)
    g = S.capture_steps(U, n, 0.3, dts)
    torch.cuda.synchronize()
    assert torch.equal(U, X0)              # nothing ran at capture
    for k in range(3):
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(U, ref[k][0]), f"replay {k}: state differs from the eager steps"
        assert torch.equal(dts, ref[k][1][:n]), f"replay {k}: step sizes differ"
        # eager library work between replays, on other buffers
        S.residual(X0.clone())
        torch.cuda.synchronize()
    # the graph reads the state buffer as it is at replay
    U.copy_(X0)
    g.replay()
    torch.cuda.synchronize()
    assert torch.equal(U, ref[0][0])
    S.check()
    S.close()
