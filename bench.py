#!/usr/bin/env python
"""Throughput of the Hermite finite-difference hot path on one MI355X.

One step = one full three-stage TVD Runge-Kutta step of the whole mesh:
time step (min over vertices), then per stage the edge pass (Hermite/WENO
reconstruction + Rusanov flux of every edge) and the vertex pass
(least-squares divergence + Runge-Kutta update of every owned vertex).
Inputs are synthetic (seeded jittered lattice, closed-form initial state)
and resident in HBM before the timed region.

Default workload: Mach 1.1 normal shock + isentropic vortex on [0,2]x[0,1],
2049 x 1025 jittered lattice with 5 ghost layers (2.1 M owned vertices,
6.4 M active edges).  The metric is vertex-RK-stage updates per second
(owned vertices x 3 stages x steps / wall time); the float32 mixed form is
the reported value, float64 is measured beside it.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload_options(name, prm):
    kw = dict(switch=prm["switch"], mu=prm.get("mu", 0.0))
    if prm.get("mu", 0.0) > 0:
        kw.update(prandtl=prm["prandtl"], gas_R=prm["gas_R"])
    if prm["switch"] in ("paper", "weno"):
        # bounded 3-node weights: without them the 3-node branch fails the
        # runs within a few steps
        kw["w3_cap"] = 2.0
    return kw


def time_precision(S, U0d, prec, wref, steps, warmup, cfl, chunk):
    """Time `steps` steps in chunks of `chunk` steps, each chunk starting
    again from the initial state (the captured shock of this method grows
    until the solution fails after a few dozen steps, so every timed step
    is one of the first `chunk` steps of the same evolution).  Only the
    steps are inside the timed regions, each bracketed by device
    synchronisations."""
    import torch
    S.set_precision(prec, wref)
    U = U0d.clone()
    dts = torch.empty(max(chunk, warmup, 1), dtype=torch.float64, device=U.device)
    S.rk_steps(U, warmup, cfl, dts)
    torch.cuda.synchronize()
    S.check()
    S.kernel_times()
    wall = 0.0
    done = 0
    while done < steps:
        n = min(chunk, steps - done)
        U.copy_(U0d)
        torch.cuda.synchronize()
        S.set_timing(True)
        t0 = time.perf_counter()
        # n x (device-side time step, Runge-Kutta step) in one library call
        S.rk_steps(U, n, cfl, dts)
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
        S.set_timing(False)
        S.check()
        done += n
    e_ms, n_e, v_ms, n_v = S.kernel_times()
    info = S.refresh_info()
    # the edge passes read a side's 3-node rows only where that side takes
    # the 3-node branch: count those sides at the initial state
    bytes_edge = info["bytes_edge_launch"]
    w3_sides = None
    if info["bytes_edge_w3_side"] > 0:
        _, mask, _ = S.edge_states(U0d, want_mask=True, want_flux=False)
        mask = mask.to(torch.int32)
        w3_sides = int(((mask & 0xF) != 0).sum().item() + ((mask >> 4) != 0).sum().item())
        bytes_edge += w3_sides * info["bytes_edge_w3_side"]
    return dict(U=U, wall=wall, edge_ms=e_ms / max(n_e, 1), vertex_ms=v_ms / max(n_v, 1),
                n_edge=n_e, n_vertex=n_v, bytes_edge=bytes_edge, w3_sides=w3_sides,
                bytes_vertex=info["bytes_vertex_launch"],
                bytes_vertex_staged=info["bytes_vertex_staged"])


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    if it was taken for this workload and the current kernel source."""
    from paper_2109_01286_amd import profile_summary
    path = os.path.join(ROOT, "profiles", f"{workload}_kernel_stats_traffic.json")
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    if d.get("workload") != workload or d.get("kernel_sources_sha256") != profile_summary.source_digest():
        return None
    for name, v in d["per_launch"].items():
        if name.startswith(kernel):
            return v["bytes"]
    return None


def roofline(r):
    kern = {}
    for k in ("edge", "vertex"):
        ms = r[f"{k}_ms"]
        gbs = r[f"bytes_{k}"] / (ms * 1e-3) / 1e9
        kern[k] = dict(avg_ms=ms, alg_bytes=r[f"bytes_{k}"], achieved_gbs=gbs,
                       frac=gbs / HBM_PEAK_GBS, launches=r[f"n_{k}"])
    if r.get("bytes_vertex_staged"):
        # the float32 vertex pass stages its blocks in LDS and reads 1-byte
        # local ids plus lists instead of 4-byte slot ids: its own bytes
        # beside the method's
        kern["vertex"]["staged_bytes"] = r["bytes_vertex_staged"]
        kern["vertex"]["staged_gbs"] = r["bytes_vertex_staged"] / (r["vertex_ms"] * 1e-3) / 1e9
    dom = max(kern, key=lambda k: kern[k]["avg_ms"])
    return dom, kern


def cpu_baseline(m, U0, prm, kw, budget_s):
    """The oracle, as it is, on a bounded sample of the same workload."""
    import numpy as np
    import torch

    from oracle import scheme as osch
    owned = np.nonzero(m.ghost_src == -1)[0]
    # a compact patch of owned vertices around the vortex / shock region
    c = m.xy[owned].mean(axis=0) if m.period[0] else np.array([0.4, 0.5])
    d = np.max(np.abs(m.xy[owned] - c), axis=1)
    sample = owned[np.argsort(d, kind="stable")[:1024]]
    sample.sort()
    opts = osch.Options(gamma=1.4, mu=kw.get("mu", 0.0), w3_cap=kw.get("w3_cap", 0.0))
    t0 = time.perf_counter()
    sc = osch.Scheme(m.xy, m.tri, m.ghost_src, m.period, opts, verts=sample)
    setup = time.perf_counter() - t0
    Ut = torch.as_tensor(U0)

    def timed(budget):
        n = 0
        t0 = time.perf_counter()
        while True:
            sc.residual(Ut, kw["switch"])
            n += 1
            el = time.perf_counter() - t0
            if el > budget:
                return n, el

    n, el = timed(budget_s)
    cores = torch.get_num_threads()
    # the same on one thread, on a third of the budget
    torch.set_num_threads(1)
    try:
        n1, el1 = timed(budget_s / 3)
    finally:
        torch.set_num_threads(cores)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return dict(value=sample.size * n / el, unit="vertex-stage/s", cores=cores,
                kind="oracle",
                sample=f"{sample.size} owned vertices (a compact patch), {n} residual "
                       f"evaluations in {el:.1f} s; oracle setup {setup:.1f} s not timed",
                value_1_thread=sample.size * n1 / el1,
                host={"cpu": model, "logical_cpus": os.cpu_count(),
                      "affinity": len(os.sched_getaffinity(0))})


def accuracy_runs():
    """Errors against closed-form solutions, float32 (mixed) and float64, on
    the cases that stay finite under the readings (the shock-vortex has no
    closed form; its float32-float64 difference is reported with the
    throughput):
      - the vortex on the 21 x 21 lattice, 20 steps at CFL 0.3, paper switch
        with the 3-node cap 2 (without it the run fails), against the exactly
        advected vortex;
      - the Taylor-Green vortex on the 129 x 129 lattice, 20 steps at CFL 0.3,
        smooth switch, against the incompressible decay exp(-2 nu t) (the
        513 x 513 lattice of the same recipe is unstable after two steps).
    L2 (root mean square over owned vertices) and max errors of rho and of
    the momentum rho u."""
    import numpy as np
    import torch

    from paper_2109_01286_amd import hfd, inputs
    cases = {"vortex21": ("vortex21", None, {"switch": "paper", "w3_cap": 2.0}),
             "tgv129": ("tgv513", 129, None)}
    out = {}
    for key, (name, scale, over) in cases.items():
        m, U0, prm = inputs.workload(name, scale)
        kw = workload_options(name, prm)
        if over:
            kw.update(over)
        S = hfd.Solver(m.xy, m.tri, m.ghost_src, m.period, device=0, **kw)
        wref = U0[0:4, m.ghost_src == -1].mean(axis=1)
        owned = m.ghost_src == -1
        res = {}
        for prec in ("fp64", "fp32"):
            S.set_precision(prec, wref)
            U = torch.as_tensor(S.to_internal(U0), device="cuda:0")
            dt = torch.empty(1, dtype=torch.float64, device="cuda:0")
            t = 0.0
            for _ in range(prm["steps"] if key == "vortex21" else 20):
                S.stable_dt(U, 0.3, out=dt)
                t += dt.item()
                S.rk_step(U, dt)
            S.check()
            Uh = S.to_input(U.cpu().numpy())
            if key == "vortex21":
                Ue = inputs.isentropic_vortex(m, center=(5.0, 5.0), beta=5.0, t=t)
            else:
                Ue = inputs.taylor_green(m, t=t, nu=prm["mu"])
            e = {}
            for q, nm in ((0, "rho"), (1, "rho_u")):
                d = Uh[q, owned] - Ue[q, owned]
                e[nm] = {"l2": float(np.sqrt(np.mean(d * d))), "max": float(np.abs(d).max())}
            res[prec] = dict(t=t, **e)
        res["fp32_over_fp64_l2_rho"] = res["fp32"]["rho"]["l2"] / res["fp64"]["rho"]["l2"]
        out[key] = res
        del S
    return out


# the five configurations: workload, lattice size (None = full), options
CONFIGS = {
    "vortex21": ("vortex21", None, dict(switch="paper")),
    "riemann201": ("riemann201", None, dict(switch="paper", w3_cap=2.0)),
    "tgv513": ("tgv513", None, dict(switch="smooth", mu=0.01, prandtl=0.72, gas_R=1.0)),
    "vortex257": ("vortex257", None, dict(switch="weno", w3_cap=2.0)),
    "shockvortex2049": ("shockvortex2049", None, dict(switch="paper", w3_cap=2.0)),
}


def fp32_residual_errors():
    """Per configuration, the residual of the float32 mixed form at the
    initial state against the float64 form's on the same GPU weights, at
    every owned vertex, with the branch of eq. 2d_hweno_intp forced to the
    float64 decisions (the decisions that differ are counted): per block
    (w, w_x, w_y) the relative L2 error and the largest element error over
    the block's largest value.  The float64 form itself agrees with the
    oracle to 1e-12 on imported weights and to the precompute's
    conditioning (<= 1e-8) at these sizes (GPU tests).  Two floors that
    float32 data alone impose, as the float64 residual's relative change:
    ``state_rounding`` rounds the whole state to float32, ``pert_rounding``
    only the perturbation about the reference state (what the mixed form
    holds in float32)."""
    import torch

    from paper_2109_01286_amd import hfd, inputs

    def blocks(a, b, own):
        # finite entries of both (the method can produce non-positive
        # pressure at an edge midpoint, e.g. the Riemann case's first
        # residual; those entries are counted, not compared)
        l2, el, bad = [], [], 0
        for k in range(3):
            x, y = a[4 * k:4 * k + 4, own], b[4 * k:4 * k + 4, own]
            f = torch.isfinite(x) & torch.isfinite(y)
            bad += int((~f).sum().item())
            x, y = x[f], y[f]
            l2.append(float(torch.linalg.norm(x - y) / torch.linalg.norm(y)))
            el.append(float((x - y).abs().max() / y.abs().max()))
        return l2, el, bad

    out = {}
    for key, (name, scale, kw) in CONFIGS.items():
        m, U0, prm = inputs.workload(name, scale)
        S = hfd.Solver(m.xy, m.tri, m.ghost_src, m.period, device=0, **kw)
        Ud = torch.as_tensor(S.to_internal(U0), device="cuda:0")
        own = slice(0, S.n_owned)
        wref = U0[0:4, m.ghost_src == -1].mean(axis=1)
        R64 = S.residual(Ud)
        _, mask64, _ = S.edge_states(Ud, want_mask=True, want_flux=False)
        sr, _, _ = blocks(S.residual(Ud.float().double()), R64, own)
        Up = Ud.float().double()
        wr = torch.as_tensor(wref, device=Ud.device)[:, None]
        Up[0:4] = wr + (Ud[0:4] - wr).float().double()
        pr, _, _ = blocks(S.residual(Up), R64, own)
        S.set_precision("fp32", wref)
        _, mask32, _ = S.edge_states(Ud, want_mask=True, want_flux=False)
        flips = int((mask32 != mask64).sum().item())
        S.force_switch_mask(mask64)
        R32 = S.residual(Ud)
        S.force_switch_mask(None)
        try:
            S.check()
            numeric = "ok"
        except hfd.HfdError:
            numeric = "non-finite or non-positive state met (property of the case)"
        l2, el, bad = blocks(R32, R64, own)
        out[key] = {"switch": kw["switch"], "owned": int(S.n_owned),
                    "fp32_rel_l2": max(l2), "fp32_rel_l2_blocks": l2,
                    "fp32_max_elem_rel_blocks": el,
                    "state_rounding_rel_l2_blocks": sr, "pert_rounding_rel_l2_blocks": pr,
                    "switch_flips": flips, "nonfinite_entries": bad, "check": numeric}
        del S
    return out


def riemann_after_steps(steps=10, cfl=0.03):
    """The 2D Riemann case (201 x 201) after ``steps`` Runge-Kutta steps in
    float64 and in the float32 mixed form, with WENO everywhere, the HLLC
    flux and capped 3-node weights at CFL 0.03: the smallest step at which
    this case stays finite for ten steps (at CFL 0.1 it fails in step 4, at
    0.3 in step 2; with the paper switch in step 1).  The float32 run takes
    the float64 run's time steps.  Reports per block (w, w_x, w_y) the
    relative L2 difference of the two states, and the float32 residual's
    relative L2 error at the float64 state after the steps."""
    import torch

    from paper_2109_01286_amd import hfd, inputs

    m, U0, prm = inputs.workload("riemann201", None)
    S = hfd.Solver(m.xy, m.tri, m.ghost_src, m.period, device=0, switch="weno",
                   w3_cap=2.0, flux="hllc")
    own = slice(0, S.n_owned)
    U64 = torch.as_tensor(S.to_internal(U0), device="cuda:0")
    dts = []
    for _ in range(steps):
        dts.append(S.stable_dt(U64, cfl).item())
        S.rk_step(U64, dts[-1])
    S.check()
    R64 = S.residual(U64)
    S.set_precision("fp32", U0[0:4, m.ghost_src == -1].mean(axis=1))
    U32 = torch.as_tensor(S.to_internal(U0), device="cuda:0")
    for dt in dts:
        S.rk_step(U32, dt)
    S.check()
    R32 = S.residual(U64)

    def rel(a, b):
        return [float(torch.linalg.norm(a[4 * k:4 * k + 4, own] - b[4 * k:4 * k + 4, own])
                      / torch.linalg.norm(b[4 * k:4 * k + 4, own])) for k in range(3)]

    return {"workload": "riemann201", "steps": steps, "cfl": cfl, "switch": "weno",
            "flux": "hllc", "w3_cap": 2.0, "t": float(sum(dts)),
            "state_fp32_vs_fp64_rel_l2_blocks": rel(U32, U64),
            "residual_fp32_vs_fp64_rel_l2_blocks": rel(R32, R64)}


def adjoint_fd(S, Ud, dt, steps, xy, area, g, ndir=32, seed=4242):
    """Central differences of the objective in ``ndir`` seeded directions
    delta ~ N(0, 1), step eps = 1e-6 ||U0||_inf / ||delta||_inf and eps / 4,
    against the adjoint's <g, delta>; errors relative to the rms directional
    derivative, for eps, eps / 4 and the Richardson combination
    (16 D(eps / 4) - D(eps)) / 15 (the WENO weights make the O(eps^2) term
    of the central difference visible at the configured step)."""
    import numpy as np
    import torch

    from paper_2109_01286_amd.adjoint import pressure_disk_objective
    gen = torch.Generator(device="cuda:0").manual_seed(seed)
    fd, ad = [], []
    u_inf = Ud.abs().max()
    for _ in range(ndir):
        d = torch.randn(Ud.shape, dtype=torch.float64, device="cuda:0", generator=gen)
        row = []
        for f in (1.0, 0.25):
            eps = float(1e-6 * u_inf / d.abs().max()) * f
            Js = []
            for sgn in (1.0, -1.0):
                X = Ud + sgn * eps * d
                for _ in range(steps):
                    S.rk_step(X, dt)
                Js.append(pressure_disk_objective(X, xy, (7.0, 7.0), 1.0, area))
            row.append(float((Js[0] - Js[1]) / (2.0 * eps)))
        fd.append(row)
        ad.append(float(torch.sum(g * d)))
    fd, ad = np.array(fd), np.array(ad)
    rms = float(np.sqrt(np.mean(ad ** 2)))
    rich = (16.0 * fd[:, 1] - fd[:, 0]) / 15.0
    e = lambda x: {"max": float(np.max(np.abs(x - ad)) / rms),
                   "median": float(np.median(np.abs(x - ad)) / rms)}
    return {"directions": ndir, "seed": seed, "eps": e(fd[:, 0]), "eps_quarter": e(fd[:, 1]),
            "richardson": e(rich), "switch_flips": 0,
            "note": "WENO-only switch: no branch of eq. 2d_hweno_intp to flip"}


def adjoint_ratio(steps=200, ckpt=20):
    """Adjoint/forward time of the isentropic vortex on the 257 x 257 periodic
    jittered lattice: gradient of J = sum A_v [|x - (7,7)| < 1] p^2 after
    `steps` RK3 steps of fixed size (from the initial state, CFL 0.3) with
    respect to the initial state, checkpoints every `ckpt` steps.  WENO-only
    switch with the 3-node cap: the paper's switch does not stay finite for
    200 steps at this resolution."""
    import numpy as np
    import torch

    from paper_2109_01286_amd import hfd, inputs
    from paper_2109_01286_amd.adjoint import pressure_disk_objective, rk_steps
    m, U, prm = inputs.workload("vortex257")
    S = hfd.Solver(m.xy, m.tri, m.ghost_src, m.period, device=0, switch="weno", w3_cap=2.0)
    Ud = torch.as_tensor(S.to_internal(U), device="cuda:0")
    dt = S.stable_dt(Ud, 0.3).item()
    xy = torch.as_tensor(m.xy[S.old_of_new], device="cuda:0")
    area = torch.as_tensor(inputs.vertex_areas(m)[S.old_of_new], device="cuda:0")
    # forward alone (warm once)
    X = Ud.clone()
    S.rk_step(X, dt)
    torch.cuda.synchronize()
    X = Ud.clone()
    t0 = time.perf_counter()
    for _ in range(steps):
        S.rk_step(X, dt)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    # one-time set-up, as for any later gradient on this mesh, not part of the
    # ratio: the adjoint's transposed maps, coefficient copies and work
    # buffers, and the first use of the objective's torch kernels (a one-step
    # gradient)
    t0 = time.perf_counter()
    U0 = Ud.clone().requires_grad_(True)
    Jw = pressure_disk_objective(rk_steps(U0, S, 1, dt, 1), xy, (7.0, 7.0), 1.0, area)
    torch.autograd.grad(Jw, U0)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    # forward with checkpoints + objective, then the backward pass
    U0 = Ud.clone().requires_grad_(True)
    t0 = time.perf_counter()
    Uf = rk_steps(U0, S, steps, dt, ckpt)
    J = pressure_disk_objective(Uf, xy, (7.0, 7.0), 1.0, area)
    torch.cuda.synchronize()
    t_fwd_ck = time.perf_counter() - t0
    t0 = time.perf_counter()
    (g,) = torch.autograd.grad(J, U0)
    torch.cuda.synchronize()
    t_bwd = time.perf_counter() - t0
    S.check()
    fd = adjoint_fd(S, Ud, dt, steps, xy, area, g)
    # the binomial schedule with 10 snapshot slots (memory: 10 states and one
    # step's stages, against 10 + 3 x 20 for the uniform schedule)
    from paper_2109_01286_amd.adjoint import RKStepsRevolve
    U0 = Ud.clone().requires_grad_(True)
    Jr = pressure_disk_objective(rk_steps(U0, S, steps, dt, snapshots=10), xy, (7.0, 7.0), 1.0,
                                 area)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    (gr,) = torch.autograd.grad(Jr, U0)
    torch.cuda.synchronize()
    t_rev = time.perf_counter() - t0
    revolve = {"snapshots": 10, "backward_ms": t_rev * 1e3,
               "adjoint_over_forward": t_rev / t_fwd,
               "backward_forward_steps": RKStepsRevolve.last_stats["forward_steps"],
               "grad_equal_to_uniform": bool(torch.equal(gr, g))}
    # the mixed form: float32 steps and adjoint steps (float64 states and
    # lambdas), the same schedule; its gradient against the float64 one
    S.set_precision("fp32", U[0:4, m.ghost_src == -1].mean(axis=1))
    X = Ud.clone()
    S.rk_step(X, dt)
    U0 = Ud.clone().requires_grad_(True)
    Jw = pressure_disk_objective(rk_steps(U0, S, 1, dt, 1), xy, (7.0, 7.0), 1.0, area)
    torch.autograd.grad(Jw, U0)
    torch.cuda.synchronize()
    X = Ud.clone()
    t0 = time.perf_counter()
    for _ in range(steps):
        S.rk_step(X, dt)
    torch.cuda.synchronize()
    t_fwd32 = time.perf_counter() - t0
    U0 = Ud.clone().requires_grad_(True)
    J32 = pressure_disk_objective(rk_steps(U0, S, steps, dt, ckpt), xy, (7.0, 7.0), 1.0, area)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    (g32,) = torch.autograd.grad(J32, U0)
    torch.cuda.synchronize()
    t_bwd32 = time.perf_counter() - t0
    S.check()
    fp32 = {"forward_ms": t_fwd32 * 1e3, "backward_ms": t_bwd32 * 1e3,
            "adjoint_over_forward": t_bwd32 / t_fwd32,
            "J_rel_diff_vs_fp64": abs(J32.item() - J.item()) / abs(J.item()),
            "grad_rel_l2_diff_vs_fp64": float(torch.linalg.norm(g32 - g) / torch.linalg.norm(g))}
    return {"workload": "vortex257", "steps": steps, "ckpt_every": ckpt, "dtype": "f64",
            "binomial": revolve, "fp32": fp32,
            "switch": "weno", "forward_ms": t_fwd * 1e3,
            "forward_with_checkpoints_ms": t_fwd_ck * 1e3, "backward_ms": t_bwd * 1e3,
            "adjoint_setup_ms": t_setup * 1e3,
            "adjoint_over_forward": t_bwd / t_fwd, "J": J.item(),
            "grad_finite": bool(torch.isfinite(g).all().item()), "fd_check": fd}


def graph_line(steps=200, chunk=20):
    """Forward steps on the vortex 257 x 257 lattice (65 536 vertices: each
    launch takes a few tens of microseconds, so launch overheads show),
    issued from the host `chunk` steps per library call, against the same
    chunk captured once in a HIP graph (Solver.capture_steps) and replayed.
    WENO everywhere with the 3-node cap, device-side CFL 0.3 time steps; both
    runs start from the initial state and must end in the same state."""
    import torch

    from paper_2109_01286_amd import hfd, inputs
    m, U, prm = inputs.workload("vortex257")
    S = hfd.Solver(m.xy, m.tri, m.ghost_src, m.period, device=0, switch="weno", w3_cap=2.0)
    out = {"workload": "vortex257", "steps": steps, "steps_per_call": chunk}
    for prec in ("fp64", "fp32"):
        if prec == "fp32":
            S.set_precision("fp32", U[0:4, m.ghost_src == -1].mean(axis=1))
        X0 = torch.as_tensor(S.to_internal(U), device="cuda:0")
        dts = torch.empty(chunk, dtype=torch.float64, device="cuda:0")
        X = X0.clone()
        S.rk_steps(X, chunk, 0.3, dts)
        X.copy_(X0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps // chunk):
            S.rk_steps(X, chunk, 0.3, dts)
        torch.cuda.synchronize()
        t_eager = time.perf_counter() - t0
        Y = X0.clone()
        g = S.capture_steps(Y, chunk, 0.3, dts)
        g.replay()
        Y.copy_(X0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps // chunk):
            g.replay()
        torch.cuda.synchronize()
        t_graph = time.perf_counter() - t0
        S.check()
        out[prec] = {"eager_ms_per_step": t_eager / steps * 1e3,
                     "graph_ms_per_step": t_graph / steps * 1e3,
                     "same_final_state": bool(torch.equal(X, Y))}
    return out


def viscous_line(steps=12, warmup=1):
    """Throughput of the viscous path on the Taylor-Green recipe at 513 x 513
    (262 k vertices, about the one-GPU share of the shock-vortex mesh split
    eight ways; its working set exceeds the MALL), float32 and float64, with
    the vertex pass against the HBM roofline.  Every timed step restarts
    from the initial state: under the readings the lattice is unstable from
    the second step on."""
    import torch

    from paper_2109_01286_amd import hfd, inputs
    m, U0, prm = inputs.workload("tgv513")
    kw = workload_options("tgv513", prm)
    S = hfd.Solver(m.xy, m.tri, m.ghost_src, m.period, device=0, **kw)
    U0d = torch.as_tensor(S.to_internal(U0), device="cuda:0")
    wref = U0[0:4, m.ghost_src == -1].mean(axis=1)
    out = {"workload": "tgv513", "owned": int(m.n_owned()), "steps": steps,
           "steps_per_restart": 1}
    gen = torch.Generator(device="cuda:0").manual_seed(12)
    lam = torch.randn(U0d.shape, dtype=torch.float64, device="cuda:0", generator=gen)
    for prec in ("fp32", "fp64"):
        r = time_precision(S, U0d, prec, wref, steps, warmup, 0.3, 1)
        _, kern = roofline(r)
        out[prec] = {"value": m.n_owned() * 3 * steps / r["wall"],
                     "unit": "vertex-stage/s", "ms_per_step": r["wall"] / steps * 1e3,
                     "kernels": kern}
        # adjoint step (two stages recomputed, three adjoint residuals, the
        # viscous rows included) against the forward step, both from the
        # initial state
        dt = S.stable_dt(U0d, 0.3).item()
        X = U0d.clone()
        L = torch.empty_like(U0d)
        S.rk_step(X, dt)
        S.rk_step_adjoint(U0d, dt, lam, L)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            X.copy_(U0d)
            S.rk_step(X, dt)
        torch.cuda.synchronize()
        t_f = time.perf_counter() - t0
        t0 = time.perf_counter()
        for _ in range(steps):
            S.rk_step_adjoint(U0d, dt, lam, L)
        torch.cuda.synchronize()
        t_b = time.perf_counter() - t0
        S.check()
        out[prec]["adjoint_step_ms"] = t_b / steps * 1e3
        out[prec]["adjoint_step_over_step"] = t_b / t_f
        out[prec]["adjoint_finite"] = bool(torch.isfinite(L).all().item())
    del S
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--chunk", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="shockvortex2049")
    ap.add_argument("--scale", type=int, default=None)
    ap.add_argument("--cfl", type=float, default=0.3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--only", choices=["fp32", "fp64"], default=None)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-viscous", action="store_true")
    ap.add_argument("--no-flux-variants", action="store_true")
    ap.add_argument("--no-config-errors", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="run one device-to-device copy of this size first (a "
                         "known-size kernel for calibrating HBM byte counters)")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the mesh would be partitioned with a halo exchange per stage).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2109_01286_amd import hfd, inputs

    t0 = time.perf_counter()
    m, U0, prm = inputs.workload(a.workload, a.scale)
    kw = workload_options(a.workload, prm)
    log(f"[bench] {a.workload}: {m.nv} vertices ({m.n_owned()} owned), inputs "
        f"{time.perf_counter() - t0:.1f} s")
    torch.cuda.init()
    torch.cuda.synchronize()
    mem0 = (torch.cuda.mem_get_info(0), torch.cuda.memory_reserved(0))
    t0 = time.perf_counter()
    S = hfd.Solver(m.xy, m.tri, m.ghost_src, m.period, device=0, **kw)
    info = S.info
    torch.cuda.synchronize()
    mem1 = (torch.cuda.mem_get_info(0), torch.cuda.memory_reserved(0))
    log(f"[bench] setup {time.perf_counter() - t0:.1f} s (host {info['setup_ms'][0]:.0f} ms, "
        f"upload {info['setup_ms'][1]:.0f} ms, GPU precompute {info['setup_ms'][2]:.0f} ms); "
        f"{info['n_edges']} active edges, ranks {info['rank_hist'][10:15]}")
    U0d = torch.as_tensor(S.to_internal(U0), device="cuda:0")
    if a.copy_probe_mb:
        n = a.copy_probe_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy probe: {a.copy_probe_mb} MiB device-to-device")
        del src, dst
    wref = U0[0:4, m.ghost_src == -1].mean(axis=1)

    res = {}
    for prec in ("fp64", "fp32"):
        if a.only and prec != a.only:
            continue
        r = time_precision(S, U0d, prec, wref, a.steps, a.warmup, a.cfl, a.chunk)
        r["rate"] = m.n_owned() * 3 * a.steps / r["wall"]
        dom, kern = roofline(r)
        r["dom"], r["kern"] = dom, kern
        res[prec] = r
        log(f"[bench] {prec}: {r['wall'] / a.steps * 1e3:.3f} ms/step, "
            f"{r['rate'] / 1e9:.3f} G vertex-stage/s; edge {kern['edge']['avg_ms']:.3f} ms "
            f"({kern['edge']['achieved_gbs']:.0f} GB/s), vertex {kern['vertex']['avg_ms']:.3f} ms "
            f"({kern['vertex']['achieved_gbs']:.0f} GB/s)")
    # Riemann-flux variants: the same steps with Roe's and the HLLC flux
    # (edge-pass arithmetic only; the bytes are those of the Rusanov run)
    variants = {}
    if not a.no_flux_variants:
        for prec in res:
            variants[prec] = {"rusanov": {"edge_ms": res[prec]["edge_ms"],
                                          "ms_per_step": res[prec]["wall"] / a.steps * 1e3}}
            for fx in ("roe", "hllc"):
                S.set_flux(fx)
                try:
                    r = time_precision(S, U0d, prec, wref, a.chunk, 2, a.cfl, a.chunk)
                    variants[prec][fx] = {"edge_ms": r["edge_ms"],
                                          "ms_per_step": r["wall"] / a.chunk * 1e3}
                except hfd.HfdError as e:
                    variants[prec][fx] = {"error": str(e)}
                finally:
                    S.set_flux("rusanov")
            log(f"[bench] {prec} edge pass by flux: " + ", ".join(
                f"{k} {v.get('edge_ms', float('nan')):.3f} ms" for k, v in variants[prec].items()))
    torch.cuda.synchronize()
    mem2 = (torch.cuda.mem_get_info(0), torch.cuda.memory_reserved(0))

    def lib_bytes(a0, a1):
        # device memory taken between two points, less what torch's caching
        # allocator reserved meanwhile: the library's own allocations
        return (a0[0][0] - a1[0][0]) - (a1[1] - a0[1])

    total = mem0[0][1]
    fwd = lib_bytes(mem0, mem2)
    device_memory = {
        "total_gb": total / 1e9,
        "library_after_setup_gb": lib_bytes(mem0, mem1) / 1e9,
        "library_forward_gb": fwd / 1e9,
        "bytes_per_owned_vertex": fwd / m.n_owned(),
        "owned_vertices_fitting": int(0.95 * total / (fwd / m.n_owned())),
        "note": "forward path with both precisions resident (float64 coefficients "
                "and their float32 copies); the adjoint's buffers come on first use",
    }
    log(f"[bench] device memory: {fwd / 1e9:.2f} GB for the forward path "
        f"({fwd / m.n_owned():.0f} B per owned vertex; "
        f"{device_memory['owned_vertices_fitting'] / 1e6:.0f} M owned vertices would fit "
        f"in 95 % of {total / 1e9:.0f} GB)")
    main_prec = "fp32" if "fp32" in res else "fp64"
    r = res[main_prec]
    dom, kern = r["dom"], r["kern"]
    diff = None
    if "fp32" in res and "fp64" in res:
        a64 = res["fp64"]["U"][0, :S.n_owned]
        a32 = res["fp32"]["U"][0, :S.n_owned]
        diff = float(torch.linalg.norm(a32 - a64) / torch.linalg.norm(a64))
    out = {
        "metric": "vertex-RK-stage updates/s",
        "value": r["rate"],
        "unit": "vertex-stage/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": r["wall"] / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (f64 RK state)" if main_prec == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": a.workload, "vertices": int(m.nv), "owned": int(m.n_owned()),
                   "edges": int(info["n_edges"]), "switch": kw["switch"],
                   "w3_cap": kw.get("w3_cap", 0.0), "cfl": a.cfl,
                   "steps_per_restart": a.chunk},
        "roofline": {"bound": "hbm", "kernel": dom,
                     "achieved": kern[dom]["achieved_gbs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": kern[dom]["frac"],
                     "traffic": (measured_traffic(a.workload, "k_vertex<float" if dom == "vertex"
                                                  else "k_edge2<float")
                                 if main_prec == "fp32" else None)},
        "kernels": kern,
        "device_memory": device_memory,
    }
    if main_prec == "fp32":
        # counter traffic of the float32 passes, when taken for this source
        for k, name in (("edge", "k_edge2<float"), ("vertex", "k_vertex<float")):
            kern[k]["traffic"] = measured_traffic(a.workload, name)
    if variants:
        out["flux_variants"] = variants
    if "fp64" in res and main_prec == "fp32":
        k64 = res["fp64"]["kern"]
        # counter traffic of the float64 passes, when taken for this source
        for k, name in (("edge", "k_edge2<double"), ("vertex", "k_vertex<double")):
            k64[k]["traffic"] = measured_traffic(a.workload, name)
        out["fp64"] = {"value": res["fp64"]["rate"],
                       "ms_per_step": res["fp64"]["wall"] / a.steps * 1e3,
                       "kernels": k64}
        out["fp32_vs_fp64_rho_rel_l2"] = diff
    # The secondary measurements below report a failure in their own entry
    # instead of losing the line.
    def section(key, run, describe):
        try:
            out[key] = run()
            log(describe(out[key]))
        except Exception as e:  # noqa: BLE001 - recorded, not hidden
            out[key] = {"error": f"{type(e).__name__}: {e}"}
            log(f"[bench] {key} failed: {out[key]['error']}")

    if not a.no_accuracy:
        section("accuracy", accuracy_runs, lambda r: "[bench] accuracy: " + ", ".join(
            f"{k} rho L2 fp64 {v['fp64']['rho']['l2']:.3e} fp32 {v['fp32']['rho']['l2']:.3e}"
            for k, v in r.items()))
    if not a.no_config_errors:
        section("riemann_steps", riemann_after_steps, lambda r: (
            f"[bench] riemann201 after {r['steps']} steps (WENO, HLLC, CFL {r['cfl']}): "
            "fp32 vs fp64 state " + "/".join(f"{x:.1e}" for x in r["state_fp32_vs_fp64_rel_l2_blocks"])
            + ", residual " + "/".join(f"{x:.1e}" for x in r["residual_fp32_vs_fp64_rel_l2_blocks"])))
    if not a.no_config_errors:
        section("fp32_error", fp32_residual_errors, lambda r: "[bench] fp32 residual error: " +
                "; ".join(f"{k} " + "/".join(f"{x:.1e}" for x in v['fp32_rel_l2_blocks']) +
                          " (perturbation rounding " +
                          "/".join(f"{x:.1e}" for x in v['pert_rounding_rel_l2_blocks']) + ")"
                          for k, v in r.items()))
    if not a.no_graph:
        section("graph", graph_line, lambda r: "[bench] HIP graph (vortex257, 20 steps per "
                "call): " + ", ".join(f"{p} {r[p]['eager_ms_per_step']:.3f} ms/step eager, "
                                      f"{r[p]['graph_ms_per_step']:.3f} replayed"
                                      for p in ("fp64", "fp32")))
    if not a.no_viscous:
        section("viscous", viscous_line, lambda v: "[bench] viscous (tgv513): " + ", ".join(
            f"{p} {v[p]['value'] / 1e9:.3f} G vertex-stage/s, vertex "
            f"{v[p]['kernels']['vertex']['avg_ms']:.3f} ms "
            f"({v[p]['kernels']['vertex']['frac'] * 100:.0f} % of HBM), adjoint step "
            f"{v[p]['adjoint_step_over_step']:.2f} x step" for p in ("fp32", "fp64")))
    if not a.no_adjoint:
        del S
        torch.cuda.empty_cache()
        section("adjoint", adjoint_ratio, lambda r: (
            f"[bench] adjoint/forward (vortex257, 200 steps): f64 "
            f"{r['adjoint_over_forward']:.2f}, f32 {r['fp32']['adjoint_over_forward']:.2f} "
            f"(f32 gradient vs f64: {r['fp32']['grad_rel_l2_diff_vs_fp64']:.1e} rel L2); FD "
            f"agreement {r['fd_check']['eps']['max']:.1e} at eps, "
            f"{r['fd_check']['richardson']['max']:.1e} extrapolated"))
    if not a.no_cpu:
        log("[bench] timing the CPU oracle on a sample ...")
        section("cpu_baseline", lambda: cpu_baseline(m, U0, prm, kw, a.cpu_budget),
                lambda r: f"[bench] oracle: {r['value']:.3g} vertex-stage/s on {r['cores']} threads")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
