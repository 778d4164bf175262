"""The entry point that allocates nothing, hfd_stable_dt_noalloc, against
hfd_stable_dt through the C ABI: two calls in a row on one GPU, the second
on a smaller mesh, each bit for bit equal to the allocating entry point (a
minimum is exact, so no tolerance applies)."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2109_01286_amd import hfd, inputs


def _solver_and_state(name):
    m, U, prm = inputs.workload(name)
    S = hfd.Solver(m.xy, m.tri, m.ghost_src, m.period, device=0)
    return S, torch.as_tensor(S.to_internal(U), device="cuda:0")


@pytest.mark.gpu
def test_noalloc_time_step_equals_stable_dt_on_two_calls():
    cases = [("vortex257", 0.3), ("vortex21", 0.7)]   # second call: smaller mesh
    solvers = [(_solver_and_state(n), cfl) for n, cfl in cases]
    for (S, U), cfl in solvers:
        print(f"[noalloc] n_owned {S.n_owned}, cfl {cfl}", flush=True)
        ref = S.stable_dt(U, cfl)
        got = torch.full((1,), float("nan"), dtype=torch.float64, device=U.device)
        S.stable_dt_noalloc(U, cfl, got)
        torch.cuda.synchronize()
        assert np.isfinite(ref.item()) and ref.item() > 0.0
        assert got.item() == ref.item(), (got.item(), ref.item())
    # the first mesh again after the smaller one (the scratch keeps the last
    # call's partial minima; every call writes all the partials it reads)
    (S, U), cfl = solvers[0]
    got = torch.empty(1, dtype=torch.float64, device=U.device)
    S.stable_dt_noalloc(U, cfl, got)
    assert got.item() == S.stable_dt(U, cfl).item()


@pytest.mark.gpu
def test_noalloc_time_step_arguments():
    S, U = _solver_and_state("vortex21")
    L = hfd.lib()
    out = torch.empty(1, dtype=torch.float64, device=U.device)
    st = L.hfd_stable_dt_noalloc(S._h, ctypes.c_void_p(U.data_ptr()), -1.0,
                                 ctypes.c_void_p(out.data_ptr()), None)
    assert st == 1 and b"cfl" in L.hfd_last_error(S._h)
    st = L.hfd_stable_dt_noalloc(S._h, None, 0.3, ctypes.c_void_p(out.data_ptr()), None)
    assert st == 1
