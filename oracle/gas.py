"""Oracle gas dynamics (test infrastructure only), torch float64 on the CPU.

Plain formulas of the compressible Euler/Navier-Stokes equations in
conservative variables w = (rho, rho u, rho v, E), ideal gas.  Written with
torch so that autograd can differentiate the oracle's residual.

Readings (the paper names a "Riemann flux solver" without choosing one and
gives no viscous constitutive law):

* Riemann flux: Rusanov (local Lax-Friedrichs),
  h = (F(wL).n + F(wR).n)/2 - lam_max (wR - wL)/2,
  lam_max = max(|u_n| + c) over the two states.  The paper admits any
  Riemann solver; two variants are provided as options: Roe's flux with
  Harten's entropy fix on the acoustic waves, and the HLLC flux (Toro) with
  the Davis-Einfeldt wave-speed estimates.
* Characteristic projection (Algorithm 1): Roe average of the two end
  states of the edge, right eigenvectors of the flux Jacobian along the edge
  direction n as columns of R in the order (u_n - c, u_n, u_n + c, u_n),
  L = R^-1 (taken by a library matrix inverse here).
* Viscous flux: Newtonian, Stokes hypothesis (lambda = -2/3 mu), constant
  mu, Fourier heat flux with kappa = mu c_p / Pr, c_p = gamma R/(gamma-1),
  T = p/(rho R); gradients of u, v, T from (w, w_x, w_y) by the chain rule.
"""
from __future__ import annotations

import torch


def primitives(w, gamma):
    """w [..., 4] -> rho, u, v, p."""
    rho = w[..., 0]
    u = w[..., 1] / rho
    v = w[..., 2] / rho
    p = (gamma - 1.0) * (w[..., 3] - 0.5 * rho * (u * u + v * v))
    return rho, u, v, p


def flux_f(w, gamma):
    rho, u, v, p = primitives(w, gamma)
    return torch.stack([rho * u, rho * u * u + p, rho * u * v,
                        (w[..., 3] + p) * u], dim=-1)


def flux_g(w, gamma):
    rho, u, v, p = primitives(w, gamma)
    return torch.stack([rho * v, rho * u * v, rho * v * v + p,
                        (w[..., 3] + p) * v], dim=-1)


def normal_flux(w, n, gamma):
    """F(w) . n = f nx + g ny."""
    return flux_f(w, gamma) * n[..., 0:1] + flux_g(w, gamma) * n[..., 1:2]


def sound_speed(w, gamma):
    rho, u, v, p = primitives(w, gamma)
    return torch.sqrt(gamma * p / rho)


def roe_average(wa, wb, gamma):
    """Roe-averaged velocity, total enthalpy and sound speed of wa, wb."""
    ra, ua, va, pa = primitives(wa, gamma)
    rb, ub, vb, pb = primitives(wb, gamma)
    sa, sb = torch.sqrt(ra), torch.sqrt(rb)
    Ha = (wa[..., 3] + pa) / ra
    Hb = (wb[..., 3] + pb) / rb
    u = (sa * ua + sb * ub) / (sa + sb)
    v = (sa * va + sb * vb) / (sa + sb)
    H = (sa * Ha + sb * Hb) / (sa + sb)
    c = torch.sqrt((gamma - 1.0) * (H - 0.5 * (u * u + v * v)))
    return u, v, H, c


def roe_eigenvectors(wa, wb, n, gamma):
    """Right eigenvectors (columns) of the flux Jacobian along n at the Roe
    average of wa and wb; shape [..., 4, 4]."""
    u, v, H, c = roe_average(wa, wb, gamma)
    q2 = u * u + v * v
    nx, ny = n[..., 0], n[..., 1]
    un = u * nx + v * ny
    ut = -u * ny + v * nx
    one = torch.ones_like(u)
    zero = torch.zeros_like(u)
    cols = [
        torch.stack([one, u - c * nx, v - c * ny, H - un * c], dim=-1),
        torch.stack([one, u, v, 0.5 * q2], dim=-1),
        torch.stack([one, u + c * nx, v + c * ny, H + un * c], dim=-1),
        torch.stack([zero, -ny, nx, ut], dim=-1),
    ]
    return torch.stack(cols, dim=-1)


def rusanov(wl, wr, n, gamma):
    fl = normal_flux(wl, n, gamma)
    fr = normal_flux(wr, n, gamma)
    _, ul, vl, _ = primitives(wl, gamma)
    _, ur, vr, _ = primitives(wr, gamma)
    sl = torch.abs(ul * n[..., 0] + vl * n[..., 1]) + sound_speed(wl, gamma)
    sr = torch.abs(ur * n[..., 0] + vr * n[..., 1]) + sound_speed(wr, gamma)
    lam = torch.maximum(sl, sr)
    return 0.5 * (fl + fr) - 0.5 * lam[..., None] * (wr - wl)


def roe_flux(wl, wr, n, gamma, delta=0.1):
    """Roe's flux h = (F(wL).n + F(wR).n)/2 - R |Lambda| R^-1 (wR - wL)/2 at
    the Roe average, eigenvalues (u_n - c, u_n, u_n + c, u_n) in the column
    order of roe_eigenvectors.  Harten's entropy fix on the two acoustic
    waves: |lambda| < d is replaced by (lambda^2 + d^2) / (2 d), with
    d = delta (|u_n| + c) of the Roe state (delta = 0: no fix)."""
    u, v, H, c = roe_average(wl, wr, gamma)
    un = u * n[..., 0] + v * n[..., 1]
    lam = torch.stack([un - c, un, un + c, un], dim=-1)
    alam = torch.abs(lam)
    if delta > 0:
        d = (delta * (torch.abs(un) + c))[..., None]
        fixed = torch.where(alam < d, (lam * lam + d * d) / (2.0 * d), alam)
        acoustic = torch.tensor([True, False, True, False])
        alam = torch.where(acoustic, fixed, alam)
    R = roe_eigenvectors(wl, wr, n, gamma)
    alpha = torch.linalg.solve(R, (wr - wl)[..., None])[..., 0]
    diss = (R @ (alam * alpha)[..., None])[..., 0]
    return 0.5 * (normal_flux(wl, n, gamma) + normal_flux(wr, n, gamma)) - 0.5 * diss


def hllc_flux(wl, wr, n, gamma):
    """Toro's HLLC flux.  Wave speeds S_L = min(u_nL - c_L, u_n - c),
    S_R = max(u_nR + c_R, u_n + c) (Roe state on the right of each), contact
    speed S_M from the two momentum balances; star states
    U*_K = rho_K (S_K - u_nK)/(S_K - S_M) (1, u_K + (S_M - u_nK) n,
    E_K/rho_K + (S_M - u_nK)(S_M + p_K/(rho_K (S_K - u_nK)))), and
    F*_K = F_K + S_K (U*_K - U_K); the flux is F_L, F*_L, F*_R or F_R as
    0 lies left of S_L, between S_L and S_M, between S_M and S_R, or right
    of S_R."""
    nx, ny = n[..., 0], n[..., 1]
    rl, ul, vl, pl = primitives(wl, gamma)
    rr, ur, vr, pr = primitives(wr, gamma)
    unl, unr = ul * nx + vl * ny, ur * nx + vr * ny
    cl, cr = sound_speed(wl, gamma), sound_speed(wr, gamma)
    u, v, H, c = roe_average(wl, wr, gamma)
    un = u * nx + v * ny
    sl = torch.minimum(unl - cl, un - c)
    sr = torch.maximum(unr + cr, un + c)
    sm = (pr - pl + rl * unl * (sl - unl) - rr * unr * (sr - unr)) / (
        rl * (sl - unl) - rr * (sr - unr))

    def star(w, rho, uu, vv, p, unk, sk):
        f = rho * (sk - unk) / (sk - sm)
        return torch.stack([f, f * (uu + (sm - unk) * nx), f * (vv + (sm - unk) * ny),
                            f * (w[..., 3] / rho + (sm - unk) * (sm + p / (rho * (sk - unk))))],
                           dim=-1)

    fl, fr = normal_flux(wl, n, gamma), normal_flux(wr, n, gamma)
    fsl = fl + sl[..., None] * (star(wl, rl, ul, vl, pl, unl, sl) - wl)
    fsr = fr + sr[..., None] * (star(wr, rr, ur, vr, pr, unr, sr) - wr)
    return torch.where((sl >= 0)[..., None], fl,
                       torch.where((sm >= 0)[..., None], fsl,
                                   torch.where((sr >= 0)[..., None], fsr, fr)))


def riemann_flux(kind, wl, wr, n, gamma):
    if kind == "rusanov":
        return rusanov(wl, wr, n, gamma)
    if kind == "roe":
        return roe_flux(wl, wr, n, gamma)
    if kind == "hllc":
        return hllc_flux(wl, wr, n, gamma)
    raise ValueError(kind)


def viscous_flux(w, wx, wy, gamma, mu, prandtl, gas_R):
    """Viscous fluxes (f_vis, g_vis) [..., 4] at vertices from w and its
    gradient (Section 2.3, "Computing Viscous Flux")."""
    rho, u, v, p = primitives(w, gamma)

    def grads(d):
        r_ = d[..., 0]
        u_ = (d[..., 1] - u * r_) / rho
        v_ = (d[..., 2] - v * r_) / rho
        p_ = (gamma - 1.0) * (d[..., 3] - (u * d[..., 1] + v * d[..., 2])
                              + 0.5 * (u * u + v * v) * r_)
        T_ = (p_ - p / rho * r_) / (rho * gas_R)
        return u_, v_, T_

    ux, vx, Tx = grads(wx)
    uy, vy, Ty = grads(wy)
    kappa = mu * gamma * gas_R / ((gamma - 1.0) * prandtl)
    div = ux + vy
    txx = 2.0 * mu * ux - (2.0 / 3.0) * mu * div
    tyy = 2.0 * mu * vy - (2.0 / 3.0) * mu * div
    txy = mu * (uy + vx)
    zero = torch.zeros_like(rho)
    fv = torch.stack([zero, txx, txy, u * txx + v * txy + kappa * Tx], dim=-1)
    gv = torch.stack([zero, txy, tyy, u * txy + v * tyy + kappa * Ty], dim=-1)
    return fv, gv
