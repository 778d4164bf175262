"""Reference solution of the circular Sod problem (Section 3.3) for tests:
the flow stays radially symmetric, so the 2D Euler equations reduce to
    d_t U + d_r F(U) = -(1/r) G(U),
    U = (rho, rho u, E), F = (rho u, rho u^2 + p, u (E + p)),
    G = (rho u, rho u^2, u (E + p)),
in the radius r (u the radial velocity).  The paper compares its profiles
with this "exact" solution; it is computed here by a fine second-order
finite-volume scheme (minmod-limited linear reconstruction of the
primitive variables, HLLC flux with Davis wave speeds, Heun time stepping,
mirror condition at r = 0, zero-gradient outer boundary).  This is test
infrastructure for the physical problem, not the paper's method.
"""
from __future__ import annotations

import numpy as np


def _prim(U, g):
    rho = U[0]
    u = U[1] / rho
    p = (g - 1.0) * (U[2] - 0.5 * rho * u * u)
    return rho, u, p


def _cons(rho, u, p, g):
    return np.stack([rho, rho * u, p / (g - 1.0) + 0.5 * rho * u * u])


def _minmod(a, b):
    return np.where(a * b > 0.0, np.sign(a) * np.minimum(np.abs(a), np.abs(b)), 0.0)


def _hllc(rl, ul, pl, rr, ur, pr, g):
    cl, cr = np.sqrt(g * pl / rl), np.sqrt(g * pr / rr)
    sl = np.minimum(ul - cl, ur - cr)
    sr = np.maximum(ul + cl, ur + cr)
    sm = (pr - pl + rl * ul * (sl - ul) - rr * ur * (sr - ur)) / (rl * (sl - ul) - rr * (sr - ur))
    El = pl / (g - 1.0) + 0.5 * rl * ul * ul
    Er = pr / (g - 1.0) + 0.5 * rr * ur * ur
    Fl = np.stack([rl * ul, rl * ul * ul + pl, ul * (El + pl)])
    Fr = np.stack([rr * ur, rr * ur * ur + pr, ur * (Er + pr)])

    def star(r, u, p, E, s):
        f = r * (s - u) / (s - sm)
        return np.stack([f, f * sm, f * (E / r + (sm - u) * (sm + p / (r * (s - u))))])

    Ul = np.stack([rl, rl * ul, El])
    Ur = np.stack([rr, rr * ur, Er])
    Fsl = Fl + sl * (star(rl, ul, pl, El, sl) - Ul)
    Fsr = Fr + sr * (star(rr, ur, pr, Er, sr) - Ur)
    return np.where(sl >= 0, Fl, np.where(sm >= 0, Fsl, np.where(sr > 0, Fsr, Fr)))


def _rhs(U, r, dr, g):
    rho, u, p = _prim(U, g)
    # ghost cells: mirror at r = 0 (u -> -u), zero gradient outside
    W = [np.concatenate([q[1::-1] * s, q, q[-1:] * np.ones(2)])
         for q, s in ((rho, 1.0), (u, -1.0), (p, 1.0))]
    sl = [_minmod(w[1:-1] - w[:-2], w[2:] - w[1:-1]) for w in W]
    # face j between cells j-1 and j (j = 0 .. N), extended arrays index j + 1
    L = [w[1:-2] + 0.5 * s[:-1] for w, s in zip(W, sl)]
    R = [w[2:-1] - 0.5 * s[1:] for w, s in zip(W, sl)]
    F = _hllc(L[0], L[1], L[2], R[0], R[1], R[2], g)
    E = U[2]
    G = np.stack([rho * u, rho * u * u, u * (E + p)])
    return -(F[:, 1:] - F[:, :-1]) / dr - G / r


def solve(t_end=0.2, R=1.5, n=6000, g=1.4, r0=0.5, inner=(1.0, 0.0, 1.0),
          outer=(0.125, 0.0, 0.1), cfl=0.4):
    """Cell centres r and (rho, u, p) at t_end."""
    dr = R / n
    r = (np.arange(n) + 0.5) * dr
    ins = r < r0
    U = _cons(np.where(ins, inner[0], outer[0]), np.where(ins, inner[1], outer[1]),
              np.where(ins, inner[2], outer[2]), g)
    t = 0.0
    while t < t_end - 1e-14:
        rho, u, p = _prim(U, g)
        dt = min(cfl * dr / np.max(np.abs(u) + np.sqrt(g * p / rho)), t_end - t)
        U1 = U + dt * _rhs(U, r, dr, g)
        U = 0.5 * (U + U1 + dt * _rhs(U1, r, dr, g))
        t += dt
    return (r, *_prim(U, g))
