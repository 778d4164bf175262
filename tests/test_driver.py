"""Checkpoint/resume and per-step metrics of the time-marching driver."""
import json

import numpy as np
import pytest
import torch

from paper_2109_01286_amd import driver, hfd, inputs

from ._helpers import lib_solver


def test_checkpoint_file_round_trip_and_mesh_check(tmp_path):
    """The checkpoint holds the state in the caller's order with step and
    time; it refuses a solver of another mesh (host-only contexts: no GPU)."""
    m, U, _ = inputs.workload("vortex21")
    S = lib_solver(m, -1)
    path = str(tmp_path / "ck.npz")

    class Dev:                      # a stand-in for a device tensor
        def __init__(self, a):
            self.a = a

        def detach(self):
            return self

        def cpu(self):
            return self

        def numpy(self):
            return self.a
    driver.save(path, S, Dev(S.to_internal(U)), 7, 0.125)
    with np.load(path, allow_pickle=False) as d:
        assert np.array_equal(d["U"], U) and int(d["step"]) == 7 and float(d["t"]) == 0.125
    m2, _, _ = inputs.workload("vortex21", 11)
    with pytest.raises(ValueError):
        driver.load(path, lib_solver(m2, -1), device="cpu")


@pytest.mark.gpu
def test_resume_is_bitwise_and_metrics_are_logged(tmp_path):
    m, U, _ = inputs.workload("vortex21")
    S = lib_solver(m, 0, switch="paper", w3_cap=2.0)
    Ud = torch.as_tensor(S.to_internal(U), device="cuda:0")
    log = str(tmp_path / "run.jsonl")
    ck = str(tmp_path / "ck.npz")
    A = Ud.clone()
    exact = lambda t: inputs.isentropic_vortex(m, center=(5.0, 5.0), beta=5.0, t=t)
    step, t = driver.march(S, A, 10, cfl=0.3, log=log, ckpt=ck, ckpt_every=5, exact=exact)
    assert step == 10
    recs = [json.loads(ln) for ln in open(log)]
    assert [r["step"] for r in recs] == list(range(1, 11))
    r = recs[-1]
    assert len(r["residual_l2"]) == 3 and 0.0 <= r["weno_fraction"] <= 1.0
    assert r["min_rho"] > 0 and r["min_p"] > 0 and r["rho_l2_error"] < 0.05
    # the checkpoint was last written at step 10; resume from a step-5 one
    B = Ud.clone()
    driver.march(S, B, 5, cfl=0.3, ckpt=ck, ckpt_every=5)
    Bl, s5, t5 = driver.load(ck, S)
    assert s5 == 5
    driver.march(S, Bl, 5, cfl=0.3, step0=s5, t0=t5)
    assert torch.equal(Bl, A)
