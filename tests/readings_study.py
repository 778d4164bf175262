"""Readings of the paper compared on the oracle (CPU, test infrastructure).

Where the paper is open or inconsistent the oracle takes one reading (see the
headers of oracle/weights.py and oracle/scheme.py); the alternatives are
options of the same oracle.  This module measures, for each reading, the two
properties that decide whether the method can run the paper's cases:

* linear stability: the largest real part of the spectrum of the residual
  linearised about a state (the Jacobian by reverse-mode autograd through
  the oracle, eigenvalues by LAPACK), times the lattice spacing h;
* accuracy: the L2 truncation error of the value block of the residual at
  the exact isentropic vortex (Section 3.1), whose time derivative is
  -(w_x + w_y), under refinement.

``python -m tests.readings_study [euler|viscous|orders ...]`` prints the
full-size table (21 x 21 Euler and 33 x 33 viscous spectra, 21/41/81 orders);
tests/test_readings.py gates smaller instances of the same measurements.
"""
from __future__ import annotations

import json
import math
import sys

import numpy as np
import torch

from oracle import scheme as osch
from paper_2109_01286_amd import inputs

# reading name -> oracle options (the first is the default reading)
READINGS = {
    "default": {},
    # Section 2.2 literally: physical frame, plain pseudo-inverse, dropping
    # rule on all 15 entries, no fold; plain 3 x 6 minimum norm (Q5, Q8)
    "physical": dict(hermite="physical"),
    # dropping rule on all 15 entries of the edge-frame row (Q6)
    "drop_all": dict(drop="all"),
    # the branches as Algorithm 1 prints them (Q1)
    "algorithm": dict(branch="algorithm"),
    # degree 4 for the inviscid divergence fit (Q10)
    "deg_inv4": dict(deg_inv=4),
}
VISCOUS_READINGS = {
    "default": {},
    # degree 5 for the viscous vertex-only fit (Q10)
    "deg_vis5": dict(deg_vis=5),
}


def _max_growth(sc, U0, switch):
    V = U0.shape[1]
    f = lambda x: sc.residual(x.reshape(12, V), switch).reshape(-1)
    J = torch.func.jacrev(f, chunk_size=512)(torch.as_tensor(U0).reshape(-1)).numpy()
    ev, vec = np.linalg.eig(J)
    k = int(np.argmax(ev.real))
    v = vec[:, k].reshape(12, V)
    blocks = np.array([np.linalg.norm(v[4 * b:4 * b + 4]) for b in range(3)])
    return float(ev.real[k]), float(abs(ev.imag[k])), blocks / blocks.max()


def euler_spectrum(kw, n=21, jitter=0.2, seed=1, switch="paper"):
    """Vortex lattice of the first configuration (n x n periodic on [0, 10]^2)
    linearised about its free stream (rho, u, v, p) = (1, 1, 1, 1): at a
    uniform state omega = d, so the paper switch takes one branch everywhere
    (the 5-node value for eq. 2d_hweno_intp, the 3-node values for
    Algorithm 1's order).  Returns max Re(lambda) h and the eigenvector's
    norms over (w, w_x, w_y)."""
    m = inputs.jittered_grid(n, n, 10.0, 10.0, (True, True), 0, seed=seed, jitter=jitter)
    sc = osch.Scheme(m.xy, m.tri, m.ghost_src, m.period, osch.Options(**kw))
    U0 = np.zeros((12, m.nv))
    U0[0:4] = np.array([1.0, 1.0, 1.0, 1.0 / 0.4 + 1.0])[:, None]
    re, im, blocks = _max_growth(sc, U0, switch)
    h = 10.0 / (n - 1)
    return dict(re_h=re * h, im_h=im * h, blocks=blocks.tolist(), h=h)


def viscous_spectrum(kw, n=33, jitter=0.2, seed=3, mu=0.01):
    """Taylor-Green recipe of the third configuration (n x n periodic on
    [0, 2 pi]^2, Mach 0.1, Pr 0.72) linearised about its initial state with
    the smooth path, with viscosity mu and with mu = 0 on the same mesh: the
    viscous part's own growth is the difference."""
    m, U, prm = inputs.workload("tgv513", scale=n)
    out = {}
    for key, mu_ in (("visc", mu), ("inviscid", 0.0)):
        o = osch.Options(mu=mu_, prandtl=prm["prandtl"], gas_R=prm["gas_R"], **kw)
        sc = osch.Scheme(m.xy, m.tri, m.ghost_src, m.period, o)
        re, im, blocks = _max_growth(sc, U, "smooth")
        out[key] = dict(re=re, im=im, blocks=blocks.tolist())
    out["h"] = 2.0 * math.pi / (n - 1)
    return out


def truncation_errors(kw, ns=(21, 41, 81), jitter=0.2, seed=1, switches=("smooth", "paper")):
    """L2 error of the value block against -(w_x + w_y) at the exact
    isentropic vortex (beta = 5, free stream (1, 1, 1, 1)) per lattice and
    switch, and the orders between successive lattices."""
    errs = {s: [] for s in switches}
    for n in ns:
        m = inputs.jittered_grid(n, n, 10.0, 10.0, (True, True), 0, seed=seed, jitter=jitter)
        U = inputs.isentropic_vortex(m, beta=5.0)
        sc = osch.Scheme(m.xy, m.tri, m.ghost_src, m.period, osch.Options(**kw))
        for s in switches:
            r = sc.residual(U, s)
            errs[s].append(float(np.sqrt(np.mean((r[0:4] + U[4:8] + U[8:12]) ** 2))))
    orders = {s: [math.log2(e[i] / e[i + 1]) for i in range(len(e) - 1)]
              for s, e in errs.items()}
    return dict(ns=list(ns), errors=errs, orders=orders)


def main(argv):
    torch.set_num_threads(max(1, torch.get_num_threads()))
    what = argv or ["euler", "viscous", "orders"]
    res = {}
    if "euler" in what:
        for name, kw in READINGS.items():
            res[f"euler/{name}"] = euler_spectrum(kw)
            print(name, "euler 21", json.dumps(res[f"euler/{name}"]), flush=True)
    if "viscous" in what:
        for name, kw in VISCOUS_READINGS.items():
            res[f"viscous/{name}"] = viscous_spectrum(kw)
            print(name, "viscous 33", json.dumps(res[f"viscous/{name}"]), flush=True)
    if "orders" in what:
        for name, kw in READINGS.items():
            for jit in (0.2, 0.0):
                r = truncation_errors(kw, jitter=jit)
                res[f"orders/{name}/{jit}"] = r
                print(name, "orders jitter", jit, json.dumps(r), flush=True)
    return res


if __name__ == "__main__":
    main(sys.argv[1:])
