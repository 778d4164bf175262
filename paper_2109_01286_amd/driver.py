"""Time marching with per-step metrics and checkpoint/resume, on top of the
binding (every step runs in the library's kernels; this module only
sequences calls, reduces a few diagnostics with torch and writes files).

* ``metrics(solver, U)``: residual L2 norms per block (w, w_x, w_y), the
  fraction of (edge side, characteristic component) pairs that take the
  3-node WENO branch of eq. 2d_hweno_intp, the edge sides whose Hermite row
  dropped singular values beyond the structural one, min rho and min p over
  owned vertices.
* ``save`` / ``load``: the state in the caller's vertex order with the step
  count and time, as a numpy ``.npz`` (no pickled objects), tagged with the
  mesh size so that a checkpoint is not loaded onto another mesh.  With the
  same step sizes the resumed run is bit for bit the uninterrupted one.
* ``march``: ``nsteps`` steps of size dt (fixed, or CFL-limited and
  recomputed on the device each step), one JSON line of metrics every
  ``log_every`` steps, a checkpoint every ``ckpt_every`` steps.
"""
from __future__ import annotations

import json
import os

import numpy as np


def metrics(solver, U, gamma=None):
    """Diagnostics of the state U (internal order, device [12, nv])."""
    import torch
    g = float(solver.opts.gamma if gamma is None else gamma)
    no = solver.n_owned
    R = solver.residual(U)
    res = [float(torch.linalg.norm(R[4 * k:4 * k + 4, :no])) for k in range(3)]
    _, mask, _ = solver.edge_states(U, want_mask=True, want_flux=False)
    m = mask.to(torch.int32)
    bits = torch.stack([(m >> b) & 1 for b in range(8)])
    rho = U[0, :no]
    p = (g - 1.0) * (U[3, :no] - 0.5 * (U[1, :no] ** 2 + U[2, :no] ** 2) / rho)
    hist = solver.info["rank_hist"]
    return {"residual_l2": res, "weno_fraction": float(bits.float().mean()),
            "weno_fraction_by_component": [float(bits[[q, 4 + q]].float().mean())
                                           for q in range(4)],
            "edge_sides_truncated": int(sum(hist[:14])),
            "min_rho": float(rho.min()), "min_p": float(p.min())}


def save(path, solver, U, step, t):
    """Write U (internal order, device) in the caller's order with the step
    count and time."""
    Ui = solver.to_input(U.detach().cpu().numpy())
    tmp = path + ".tmp.npz"
    np.savez(tmp, U=Ui, step=np.int64(step), t=np.float64(t), nv=np.int64(solver.nv),
             n_owned=np.int64(solver.n_owned))
    os.replace(tmp, path)


def load(path, solver, device=None):
    """(U internal order on the solver's device, step, t) from ``save``."""
    import torch
    with np.load(path, allow_pickle=False) as d:
        if int(d["nv"]) != solver.nv or int(d["n_owned"]) != solver.n_owned:
            raise ValueError(f"checkpoint for {int(d['nv'])} vertices, solver has {solver.nv}")
        U = torch.as_tensor(solver.to_internal(d["U"]),
                            device=device or f"cuda:{solver.device}")
        return U.contiguous(), int(d["step"]), float(d["t"])


def march(solver, U, nsteps, dt=None, cfl=0.3, step0=0, t0=0.0, log=None, log_every=1,
          ckpt=None, ckpt_every=0, exact=None):
    """Advance U in place by ``nsteps`` RK3 steps.  ``dt``: fixed step size,
    or None for the CFL-limited step recomputed on the device each step.
    ``log``: a path (JSON lines appended) or a file object; ``exact(t)``, if
    given, returns the exact state (caller's order) and the line gets the L2
    and max errors of rho.  ``ckpt``: checkpoint path written every
    ``ckpt_every`` steps.  Returns (step, t)."""
    import torch
    fh = open(log, "a") if isinstance(log, str) else log
    dtd = torch.empty(1, dtype=torch.float64, device=U.device)
    step, t = step0, t0
    try:
        for _ in range(nsteps):
            if dt is None:
                solver.stable_dt(U, cfl, out=dtd)
                h = dtd.item()
                solver.rk_step(U, dtd)
            else:
                h = float(dt)
                solver.rk_step(U, h)
            step += 1
            t += h
            solver.check()
            if fh is not None and log_every and step % log_every == 0:
                rec = {"step": step, "t": t, "dt": h, **metrics(solver, U)}
                if exact is not None:
                    own = solver.old_of_new[:solver.n_owned]   # owned, caller's ids
                    e = solver.to_input(U.cpu().numpy())[0, own] - exact(t)[0, own]
                    rec["rho_l2_error"] = float(np.sqrt(np.mean(e * e)))
                    rec["rho_max_error"] = float(np.abs(e).max())
                fh.write(json.dumps(rec) + "\n")
                fh.flush()
            if ckpt and ckpt_every and step % ckpt_every == 0:
                save(ckpt, solver, U, step, t)
    finally:
        if isinstance(log, str) and fh is not None:
            fh.close()
    return step, t
