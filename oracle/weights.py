"""Oracle least-squares weights (test infrastructure only).

Section 2.2: the 15 data (c, c_x, c_y at five nodes) of one side of an edge
define a complete quartic through ``P k = r``; P is decomposed by SVD,
tiny singular values are ignored, the smallest one is dropped again and
again while any coefficient is not below one in magnitude, and with the
origin at the edge midpoint only the first row of the pseudo-inverse is
stored.  eq. 3nodes_intp: each 3-node substencil uses the 3 x 6 system of
the degree-2 basis, solved by SVD.  eq. flux_polynomials: the divergence of
a vertex comes from the least-squares fit of f and g to vertex values and
edge projections; only three row vectors d0, dx, dy of the pseudo-inverse
are stored.  Section 2.3, "Computing Viscous Flux": the viscous fluxes are
fitted to the same vertices only.

Readings (the paper leaves these open; see the test suite for what pins
each one):

* Frames.  Edge systems use x_hat = (x - x_mid)/h_e, h_e the length of the
  middle edge; vertex systems use x_hat = (x - x_v)/h_v, h_v the mean
  length of the edges at v.  Derivative data are scaled accordingly and
  the stored rows are converted back to physical units.
* "Non-zero" singular value: sigma > 1e-12 * sigma_1.  The 5-node Hermite
  matrix is singular for every stencil (the square of the conic through the
  five nodes has zero value and gradient at all of them), so its rank is
  capped at 14.
* Graded pseudo-inverse.  Among all least-squares solutions of the rank-r
  system, take the one whose highest-degree block is smallest:
  ``K = K_r - N pinv(N_top) K_r[top]`` with ``K_r`` the rank-r
  pseudo-inverse, ``N`` the discarded right singular vectors and ``top``
  the highest-degree rows (pinv threshold 1e-12 relative).  This is the
  small-h limit of the pseudo-inverse in physical units and does not
  depend on the mesh scale.  With full column rank it is the plain
  pseudo-inverse.
* Dropping rule: "any component of k" is read as any of the five value
  weights of the stored row; while one has magnitude >= 1 (and r > 1), r
  is lowered by one.
* Fold: the value weight of the side's anchor node (i for the left side,
  i+1 for the right side) absorbs 1 - sum(value weights), so constants are
  reproduced exactly; the same for the 3-node weights.
* 3-node systems: no dropping rule (the paper gives none for them).
* Divergence: polynomial degree 5 for the inviscid fit (vertices + edge
  midpoints), degree 4 for the viscous vertex-only fit; the centre vertex
  is part of the stencil; no weighting.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import basis
from .mesh import rel

RTOL = 1e-12


def svd_full(A):
    U, s, Vt = np.linalg.svd(A, full_matrices=True)
    return U, s, np.swapaxes(Vt, -1, -2)


def numerical_rank(s):
    """Count of singular values above 1e-12 of the largest (per item)."""
    s = np.asarray(s)
    return np.count_nonzero(s > RTOL * s[..., :1], axis=-1)


def graded_rows(U, s, V, r, top, rows):
    """Selected rows of the graded pseudo-inverse of rank ``r``.

    Batched over the leading axis; all items share ``r``.  Returns
    [batch, len(rows), m].
    """
    Vr = V[:, :, :r] / s[:, None, :r]
    Kr = np.einsum("bnr,bmr->bnm", Vr, U[:, :, :r])          # [b, n, m]
    out = Kr[:, rows, :]
    if V.shape[2] > r:
        N = V[:, :, r:]                                      # [b, n, n-r]
        Nt = N[:, top, :]                                    # [b, t, n-r]
        corr = np.linalg.pinv(Nt, rcond=RTOL) @ Kr[:, top, :]  # [b, n-r, m]
        out = out - N[:, rows, :] @ corr
    return out


def hermite_matrix(pts):
    """15 x 15 matrix P of the Hermite system (rows p, p_x, p_y per node,
    nodes in stencil order); ``pts`` [..., 5, 2]."""
    x, y = pts[..., 0], pts[..., 1]
    P = np.empty(pts.shape[:-2] + (15, 15))
    P[..., 0::3, :] = basis.p(x, y, 4)
    P[..., 1::3, :] = basis.px(x, y, 4)
    P[..., 2::3, :] = basis.py(x, y, 4)
    return P


def hermite_weights(pts, anchor=2, rank_cap=14):
    """Row of the graded Hermite pseudo-inverse with the dropping rule.

    ``pts`` [b, 5, 2] in the edge frame.  Returns (w [b, 15] in the edge
    frame: (value, d/dx, d/dy) per node, rank [b]).
    """
    pts = np.asarray(pts, dtype=np.float64)
    b = pts.shape[0]
    U, s, V = svd_full(hermite_matrix(pts))
    r = np.minimum(numerical_rank(s), rank_cap)
    top = basis.degree_block(4)
    w = np.empty((b, 15))
    todo = np.ones(b, dtype=bool)
    while np.any(todo):
        for rv in np.unique(r[todo]):
            idx = np.nonzero(todo & (r == rv))[0]
            wi = graded_rows(U[idx], s[idx], V[idx], int(rv), top, [0])[:, 0, :]
            w[idx] = wi
            drop = (np.max(np.abs(wi[:, 0::3]), axis=1) >= 1.0) & (rv > 1)
            r[idx[drop]] -= 1
            todo[idx[~drop]] = False
    w[:, 3 * anchor] += 1.0 - w[:, 0::3].sum(axis=1)
    return w, r


def three_node_weights(pts, anchor, cap=0.0):
    """Value weights of the graded 3 x 6 system (eq. 3nodes_intp) at the
    origin; ``pts`` [b, 3, 2], ``anchor`` local index of the side anchor.

    ``cap`` > 0 switches on a dropping rule for these systems (not in the
    paper, off by default): while a weight exceeds ``cap`` in magnitude the
    smallest kept singular value is dropped, as the 5-node rule does."""
    pts = np.asarray(pts, dtype=np.float64)
    A = basis.p(pts[..., 0], pts[..., 1], 2)                # [b, 3, 6]
    U, s, V = svd_full(A)
    r = numerical_rank(s)
    top = basis.degree_block(2)
    w = np.empty(pts.shape[:-1])
    todo = np.ones(w.shape[0], dtype=bool)
    while np.any(todo):
        for rv in np.unique(r[todo]):
            idx = np.nonzero(todo & (r == rv))[0]
            wi = graded_rows(U[idx], s[idx], V[idx], int(rv), top, [0])[:, 0, :]
            w[idx] = wi
            if cap > 0.0:
                drop = (np.max(np.abs(wi), axis=1) > cap) & (rv > 1)
            else:
                drop = np.zeros(idx.size, dtype=bool)
            r[idx[drop]] -= 1
            todo[idx[~drop]] = False
    w[:, anchor] += 1.0 - w.sum(axis=1)
    return w


def divergence_rows(node_pts, mid_pts, normals, h, deg=5):
    """d0, dx, dy of one vertex (three rows after eq. flux_polynomials).

    ``node_pts`` [N, 2] and ``mid_pts`` [M, 2] in the vertex frame,
    ``normals`` [M, 2] unit edge directions.  Columns: (f, g) per node
    interleaved, then one per edge.  Returns d [3, 2N+M] in physical units.
    """
    nb = basis.nterms(deg)
    N = node_pts.shape[0]
    M = mid_pts.shape[0]
    A = np.zeros((2 * N + M, 2 * nb))
    pn = basis.p(node_pts[:, 0], node_pts[:, 1], deg)
    A[0:2 * N:2, :nb] = pn
    A[1:2 * N:2, nb:] = pn
    pm = basis.p(mid_pts[:, 0], mid_pts[:, 1], deg)
    A[2 * N:, :nb] = pm * normals[:, 0:1]
    A[2 * N:, nb:] = pm * normals[:, 1:2]
    U, s, V = svd_full(A[None])
    r = int(numerical_rank(s)[0])
    top = basis.degree_block(deg)
    top = top + [nb + t for t in top]
    # a_2 + b_3 -> f_x + g_y ; a_4 + b_5 -> f_xx + g_xy ; a_5 + b_6 -> f_xy + g_yy
    rows = [1, nb + 2, 3, nb + 4, 4, nb + 5]
    K = graded_rows(U, s, V, r, top, rows)[0]
    d = np.stack([(K[0] + K[1]) / h, (K[2] + K[3]) / h ** 2,
                  (K[4] + K[5]) / h ** 2])
    return d, r


def viscous_rows(node_pts, h, deg=4):
    """Rows of the vertex-only fit (Section 2.3, viscous flux): returns
    [5, N] = (k_x/h, k_y/h, k_xx/h^2, k_xy/h^2, k_yy/h^2), so that
    div f_vis = r0.fv + r1.gv, its x-derivative r2.fv + r3.gv and its
    y-derivative r3.fv + r4.gv."""
    A = basis.p(node_pts[:, 0], node_pts[:, 1], deg)
    U, s, V = svd_full(A[None])
    r = int(numerical_rank(s)[0])
    K = graded_rows(U, s, V, r, basis.degree_block(deg), [1, 2, 3, 4, 5])[0]
    return np.stack([K[0] / h, K[1] / h, K[2] / h ** 2, K[3] / h ** 2,
                     K[4] / h ** 2]), r


@dataclasses.dataclass
class EdgeWeights:
    edges: np.ndarray     # [Ea] edge indices (into Topology.edges)
    n: np.ndarray         # [Ea, 2] unit direction i -> i+1
    h: np.ndarray         # [Ea] middle-edge length
    w5: np.ndarray        # [Ea, 2, 15] physical units: (value, d/dx, d/dy) per node
    w3: np.ndarray        # [Ea, 2, 3, 3] value weights per side and substencil
    rank: np.ndarray      # [Ea, 2]


# node order of each side within the six-node stencil (i-2 .. i+3)
SIDE_NODES = ((0, 1, 2, 3, 4), (5, 4, 3, 2, 1))


def edge_weights(topo, xy, period, edges=None, w3_cap=0.0):
    """Weights of the given (active) edges, both sides."""
    if edges is None:
        edges = np.nonzero(topo.active)[0]
    edges = np.asarray(edges)
    Ea = edges.size
    P = np.empty((Ea, 6, 2))
    n = np.empty((Ea, 2))
    h = np.empty(Ea)
    for j, e in enumerate(edges):
        st = topo.stencil[e]
        r_ = rel(xy, period, int(st[2]), st)
        hv = np.hypot(r_[3, 0], r_[3, 1])
        P[j] = (r_ - 0.5 * r_[3][None, :]) / hv
        n[j] = r_[3] / hv
        h[j] = hv
    w5 = np.empty((Ea, 2, 15))
    rank = np.empty((Ea, 2), dtype=np.int64)
    w3 = np.empty((Ea, 2, 3, 3))
    for s_, nodes in enumerate(SIDE_NODES):
        pts = P[:, list(nodes), :]
        w, r = hermite_weights(pts)
        w[:, 1::3] *= h[:, None]
        w[:, 2::3] *= h[:, None]
        w5[:, s_] = w
        rank[:, s_] = r
        for j in range(3):
            w3[:, s_, j] = three_node_weights(pts[:, j:j + 3, :], anchor=2 - j,
                                              cap=w3_cap)
    return EdgeWeights(edges=edges, n=n, h=h, w5=w5, w3=w3, rank=rank)


@dataclasses.dataclass
class VertexRows:
    verts: np.ndarray     # vertex ids
    d: list               # per vertex [3, 2N+M]
    dvis: list            # per vertex [5, N] or None
    h: np.ndarray


def vertex_rows(topo, xy, period, verts=None, viscous=False, deg=5, deg_vis=4):
    if verts is None:
        verts = np.nonzero(topo.owned)[0]
    d_all, dv_all, h_all = [], [], []
    edges = topo.edges
    for v in verts:
        v = int(v)
        S = topo.vnodes[v]
        M = topo.vedges[v]
        rn = rel(xy, period, v, topo.adj[v])
        hv = float(np.mean(np.hypot(rn[:, 0], rn[:, 1])))
        nodes = rel(xy, period, v, S) / hv
        a = edges[M, 0]
        ra = rel(xy, period, v, a)
        dab = np.stack([rel(xy, period, int(edges[m, 0]), [int(edges[m, 1])])[0]
                        for m in M])
        mids = (ra + 0.5 * dab) / hv
        nrm = dab / np.hypot(dab[:, 0], dab[:, 1])[:, None]
        d, _ = divergence_rows(nodes, mids, nrm, hv, deg)
        d_all.append(d)
        if viscous:
            dv, _ = viscous_rows(nodes, hv, deg_vis)
            dv_all.append(dv)
        else:
            dv_all.append(None)
        h_all.append(hv)
    return VertexRows(verts=np.asarray(verts), d=d_all, dvis=dv_all,
                      h=np.asarray(h_all))
