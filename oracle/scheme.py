"""Oracle residual and time stepping (test infrastructure only).

The unknowns of eq. HWENO are w, w_x and w_y at every vertex; each obeys a
conservation law whose divergence is evaluated by least squares at the
vertex.  The steps below follow Section 2.3 in the paper's order:

1. ghost vertices are filled (copy of their source vertex, or their own
   Dirichlet state);
2. per edge (Algorithm 1): Roe average of the two ends, L and R along the
   edge; characteristic values and gradients at the six stencil nodes; per
   side and characteristic component the uniform WENO5 weights of the five
   values, the switch of eq. 2d_hweno_intp, either the 5-node Hermite value
   or the omega-weighted 3-node values; back-projection with R; Rusanov
   flux along the edge;
3. per vertex: analytic f, g at the stencil vertices, the edge fluxes of
   the stencil edges, and the three stored row vectors give div f,
   div f_x, div f_y; viscous fluxes enter through the vertex-only rows;
4. three-stage TVD Runge-Kutta on all twelve unknowns (Section 2.3, last
   paragraph).

Readings:

* Switch (Q1/Q2 of the readings list): eq. 2d_hweno_intp is followed -- the
  5-node Hermite value when 0.01 < omega_1 < 0.79 (open interval), the
  WENO combination otherwise; Algorithm 1 states the branches the other way
  round, which contradicts the surrounding text.  Decided per side and per
  characteristic component.
* WENO weights: Jiang-Shu smoothness indicators on the five characteristic
  values taken as uniformly spaced, alpha_j = d_j/(eps + beta_j)^2 with
  eps = 1e-6 and the interpolation weights d = (1/16, 10/16, 5/16) (the
  unique weights that combine the three 3-point interpolants at x_{i+1/2}
  into the 5-point one).
* Derivatives are projected with the same L as the values.
* Time step: dt = CFL * min over owned vertices of h_min/(|u| + c), h_min
  the shortest incident edge.
* Residual of ghost vertices is zero; after a Runge-Kutta step the ghost
  rows are filled again (copies) or left at their Dirichlet state.

Modes: ``switch`` = "paper" (the rule above), "smooth" (always the 5-node
value), "weno" (always the WENO value), or an explicit per-edge mask
(uint8, bit 4*side + component set = WENO value).

Alternative readings (Options), for comparison with the defaults:
``branch="algorithm"`` takes the branches as Algorithm 1 prints them (the
omega-weighted 3-node values when 0.01 < omega_1 < 0.79, the 5-node value
otherwise); ``hermite``/``drop`` select the weight readings of
weights.edge_weights; ``deg_inv``/``deg_vis`` the degrees of the divergence
and viscous fits.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import gas, mesh as omesh, weights as ow

D_WENO = (1.0 / 16.0, 10.0 / 16.0, 5.0 / 16.0)


@dataclasses.dataclass
class Options:
    gamma: float = 1.4
    mu: float = 0.0
    prandtl: float = 0.72
    gas_R: float = 1.0
    weno_eps: float = 1e-6
    sw_lo: float = 0.01
    sw_hi: float = 0.79
    switch: object = "paper"
    w3_cap: float = 0.0     # 0: no dropping rule for the 3-node systems
    flux: str = "rusanov"   # Riemann flux: "rusanov", "roe" or "hllc"
    branch: str = "equation"  # "equation" (eq. 2d_hweno_intp) or "algorithm"
    hermite: str = "graded"   # weight reading: "graded" or "physical"
    drop: str = "value"       # entries the 5-node dropping rule tests
    deg_inv: int = 5          # degree of the inviscid divergence fit
    deg_vis: int = 4          # degree of the viscous vertex-only fit


def weno_omega(c, eps):
    """Nonlinear weights of uniform WENO5 interpolation; c [..., 5] in the
    side's stencil order (c_{-2} .. c_{2}); returns [..., 3]."""
    c0, c1, c2, c3, c4 = (c[..., k] for k in range(5))
    b1 = 13.0 / 12.0 * (c0 - 2 * c1 + c2) ** 2 + 0.25 * (c0 - 4 * c1 + 3 * c2) ** 2
    b2 = 13.0 / 12.0 * (c1 - 2 * c2 + c3) ** 2 + 0.25 * (c1 - c3) ** 2
    b3 = 13.0 / 12.0 * (c2 - 2 * c3 + c4) ** 2 + 0.25 * (3 * c2 - 4 * c3 + c4) ** 2
    a = torch.stack([D_WENO[0] / (eps + b1) ** 2, D_WENO[1] / (eps + b2) ** 2,
                     D_WENO[2] / (eps + b3) ** 2], dim=-1)
    return a / a.sum(dim=-1, keepdim=True)


def _t(x, dtype=torch.float64):
    return torch.as_tensor(np.asarray(x), dtype=dtype)


class Scheme:
    """Precomputed stencils and weights of one mesh, plus the residual.

    ``verts`` restricts the divergence (and the edges it needs) to a subset
    of owned vertices; the residual is then zero elsewhere.
    """

    def __init__(self, xy, tri, ghost_src, period, opts=None, verts=None,
                 topo=None):
        self.opts = opts or Options()
        self.xy = np.asarray(xy, dtype=np.float64)
        self.period = (float(period[0]), float(period[1]))
        self.ghost_src = np.asarray(ghost_src, dtype=np.int64)
        self.nv = self.xy.shape[0]
        self.topo = topo or omesh.build(self.xy, tri, ghost_src, self.period,
                                        verts)
        t = self.topo
        o = self.opts
        if o.branch not in ("equation", "algorithm"):
            raise ValueError(o.branch)
        self.ew = ow.edge_weights(t, self.xy, self.period, w3_cap=o.w3_cap,
                                  reading=o.hermite, drop=o.drop)
        viscous = o.mu > 0.0
        self.vr = ow.vertex_rows(t, self.xy, self.period, t.verts,
                                 viscous=viscous, deg=o.deg_inv,
                                 deg_vis=o.deg_vis)
        self._flatten()

    # -- layout -------------------------------------------------------------
    def _flatten(self):
        t, ew, vr = self.topo, self.ew, self.vr
        E = ew.edges.size
        self.edge_pos = -np.ones(t.edges.shape[0], dtype=np.int64)
        self.edge_pos[ew.edges] = np.arange(E)
        self.st = torch.as_tensor(t.stencil[ew.edges], dtype=torch.long)
        self.n = _t(ew.n)
        self.w5 = _t(ew.w5)
        self.w3 = _t(ew.w3)
        self.w5g = _t(ew.w5g)
        self.w3g = _t(ew.w3g)
        vs_own, vs_node, vs_c, vs_v = [], [], [], []
        es_own, es_edge, es_c = [], [], []
        for j, v in enumerate(vr.verts):
            S = t.vnodes[int(v)]
            M = t.vedges[int(v)]
            d = vr.d[j]
            N = len(S)
            vs_own += [j] * N
            vs_node += S
            vs_c.append(np.stack([d[0, 0:2 * N:2], d[0, 1:2 * N:2],
                                  d[1, 0:2 * N:2], d[1, 1:2 * N:2],
                                  d[2, 0:2 * N:2], d[2, 1:2 * N:2]], axis=1))
            if vr.dvis[j] is not None:
                vs_v.append(vr.dvis[j].T)
            es_own += [j] * len(M)
            es_edge += list(self.edge_pos[M])
            es_c.append(d[:, 2 * N:].T)
        self.verts = torch.as_tensor(vr.verts, dtype=torch.long)
        self.vs_own = torch.as_tensor(vs_own, dtype=torch.long)
        self.vs_node = torch.as_tensor(vs_node, dtype=torch.long)
        self.vs_c = _t(np.concatenate(vs_c))
        self.vs_v = _t(np.concatenate(vs_v)) if vs_v else None
        self.es_own = torch.as_tensor(es_own, dtype=torch.long)
        self.es_edge = torch.as_tensor(es_edge, dtype=torch.long)
        self.es_c = _t(np.concatenate(es_c))
        g = self.ghost_src
        self.gcopy = torch.as_tensor(np.nonzero(g >= 0)[0], dtype=torch.long)
        self.gsrc = torch.as_tensor(g[g >= 0], dtype=torch.long)

    # -- step 1 -------------------------------------------------------------
    def fill_ghosts(self, U):
        if self.gcopy.numel() == 0:
            return U
        W = U.clone()
        W[:, self.gcopy] = U[:, self.gsrc]
        return W

    # -- step 2 -------------------------------------------------------------
    def edge_states(self, U, switch=None, grad=False):
        """Left/right midpoint states, WENO mask and Riemann flux of every
        edge of the scheme.  Returns (wl [E,4], wr [E,4], mask [E] uint8,
        h [E,4]); with ``grad`` also the midpoint derivatives gl, gr
        [E, 2, 4] (d/dx, d/dy of each conservative component) of both sides:
        per characteristic component the derivative rows of the branch it
        takes -- the 5-node operator applied to (c, c_x, c_y), or the
        omega-weighted gradients of the three 3-node interpolants with the
        weights of the value -- then back-projected with R."""
        o = self.opts
        sw = o.switch if switch is None else switch
        W = self.fill_ghosts(U)
        Wn = W[:, self.st]                        # [12, E, 6]
        w = Wn[0:4].permute(1, 2, 0)              # [E, 6, 4]
        wx = Wn[4:8].permute(1, 2, 0)
        wy = Wn[8:12].permute(1, 2, 0)
        R = gas.roe_eigenvectors(w[:, 2], w[:, 3], self.n, o.gamma)
        L = torch.linalg.inv(R)
        c = torch.einsum("eqr,ejr->ejq", L, w)
        cx = torch.einsum("eqr,ejr->ejq", L, wx)
        cy = torch.einsum("eqr,ejr->ejq", L, wy)
        E = w.shape[0]
        mask = torch.zeros(E, dtype=torch.uint8)
        out, gout = [], []
        for s, nodes in enumerate(ow.SIDE_NODES):
            idx = list(nodes)
            cs, cxs, cys = c[:, idx], cx[:, idx], cy[:, idx]     # [E, 5, 4]
            w5 = self.w5[:, s]                                    # [E, 15]
            smooth = (torch.einsum("ej,ejq->eq", w5[:, 0::3], cs)
                      + torch.einsum("ej,ejq->eq", w5[:, 1::3], cxs)
                      + torch.einsum("ej,ejq->eq", w5[:, 2::3], cys))
            om = weno_omega(cs.permute(0, 2, 1), o.weno_eps)     # [E, 4, 3]
            subs = torch.stack([torch.einsum("et,etq->eq", self.w3[:, s, j],
                                             cs[:, j:j + 3]) for j in range(3)],
                               dim=-1)                            # [E, 4, 3]
            weno = (om * subs).sum(dim=-1)
            if isinstance(sw, str):
                if sw == "paper":
                    o1 = om[..., 0]
                    inside = (o1 > o.sw_lo) & (o1 < o.sw_hi)
                    use = inside if o.branch == "algorithm" else ~inside
                elif sw == "smooth":
                    use = torch.zeros_like(smooth, dtype=torch.bool)
                elif sw == "weno":
                    use = torch.ones_like(smooth, dtype=torch.bool)
                else:
                    raise ValueError(sw)
            else:
                m = torch.as_tensor(np.asarray(sw), dtype=torch.int64)
                use = torch.stack([((m >> (4 * s + q)) & 1) == 1
                                   for q in range(4)], dim=-1)
            for q in range(4):
                mask |= (use[:, q].to(torch.uint8) << (4 * s + q))
            C = torch.where(use, weno, smooth)
            out.append(torch.einsum("eqr,er->eq", R, C))
            if grad:
                gs = []
                for d in range(2):
                    g5 = self.w5g[:, s, d]                        # [E, 15]
                    gsm = (torch.einsum("ej,ejq->eq", g5[:, 0::3], cs)
                           + torch.einsum("ej,ejq->eq", g5[:, 1::3], cxs)
                           + torch.einsum("ej,ejq->eq", g5[:, 2::3], cys))
                    gsub = torch.stack([torch.einsum("et,etq->eq", self.w3g[:, s, j, d],
                                                     cs[:, j:j + 3]) for j in range(3)],
                                       dim=-1)
                    gw = (om * gsub).sum(dim=-1)
                    gs.append(torch.einsum("eqr,er->eq", R, torch.where(use, gw, gsm)))
                gout.append(torch.stack(gs, dim=1))               # [E, 2, 4]
        wl, wr = out
        h = gas.riemann_flux(o.flux, wl, wr, self.n, o.gamma)
        if grad:
            return wl, wr, mask, h, gout[0], gout[1]
        return wl, wr, mask, h

    # -- step 3 -------------------------------------------------------------
    def residual(self, U, switch=None):
        """dU/dt [12, V] of eq. HWENO (zero rows except the scheme's
        vertices)."""
        as_np = isinstance(U, np.ndarray)
        if as_np:
            U = torch.as_tensor(U, dtype=torch.float64)
        o = self.opts
        W = self.fill_ghosts(U)
        _, _, _, h = self.edge_states(U, switch)
        wn = W[0:4, self.vs_node].T                # [S, 4]
        f = gas.flux_f(wn, o.gamma)
        g = gas.flux_g(wn, o.gamma)
        c = self.vs_c
        nvt = self.verts.numel()
        acc = torch.zeros(nvt, 3, 4, dtype=torch.float64)
        for k in range(3):
            contrib = c[:, 2 * k:2 * k + 1] * f + c[:, 2 * k + 1:2 * k + 2] * g
            acc[:, k] = acc[:, k].index_add(0, self.vs_own, -contrib)
            ce = self.es_c[:, k:k + 1] * h[self.es_edge]
            acc[:, k] = acc[:, k].index_add(0, self.es_own, -ce)
        if o.mu > 0.0:
            wx = W[4:8, self.vs_node].T
            wy = W[8:12, self.vs_node].T
            fv, gv = gas.viscous_flux(wn, wx, wy, o.gamma, o.mu, o.prandtl,
                                      o.gas_R)
            r = self.vs_v                           # [S, 5]
            vis = [r[:, 0:1] * fv + r[:, 1:2] * gv,
                   r[:, 2:3] * fv + r[:, 3:4] * gv,
                   r[:, 3:4] * fv + r[:, 4:5] * gv]
            for k in range(3):
                acc[:, k] = acc[:, k].index_add(0, self.vs_own, vis[k])
        dU = torch.zeros(12, self.nv, dtype=torch.float64)
        dU = dU.index_copy(1, self.verts, acc.reshape(nvt, 12).T)
        return dU.numpy() if as_np else dU

    # -- step 4 -------------------------------------------------------------
    def finish_ghosts(self, Unew, Uold):
        """Ghost rows after a step: Dirichlet rows keep the old state, copy
        ghosts take their source."""
        g = torch.as_tensor(self.ghost_src)
        dirichlet = torch.nonzero(g == -2).flatten()
        if dirichlet.numel():
            Unew = Unew.clone()
            Unew[:, dirichlet] = Uold[:, dirichlet]
        return self.fill_ghosts(Unew)

    def rk3_step(self, U, dt, switch=None):
        as_np = isinstance(U, np.ndarray)
        if as_np:
            U = torch.as_tensor(U, dtype=torch.float64)
        U1 = U + dt * self.residual(U, switch)
        U2 = 0.75 * U + 0.25 * (U1 + dt * self.residual(U1, switch))
        U3 = (1.0 / 3.0) * U + (2.0 / 3.0) * (U2 + dt * self.residual(U2, switch))
        U3 = self.finish_ghosts(U3, U)
        return U3.numpy() if as_np else U3

    def stable_dt(self, U, cfl):
        U = torch.as_tensor(np.asarray(U), dtype=torch.float64)
        o = self.opts
        own = torch.as_tensor(np.nonzero(self.topo.owned)[0], dtype=torch.long)
        w = U[0:4, own].T
        rho, u, v, p = gas.primitives(w, o.gamma)
        c = torch.sqrt(o.gamma * p / rho)
        adj = self.topo.adj
        hmin = np.empty(own.numel())
        for j, v_ in enumerate(own.tolist()):
            r_ = omesh.rel(self.xy, self.period, v_, adj[v_])
            hmin[j] = np.min(np.hypot(r_[:, 0], r_[:, 1]))
        lam = torch.sqrt(u * u + v * v) + c
        return float(cfl * torch.min(_t(hmin) / lam))
