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

Alternative readings, kept as options so that they can be compared with the
ones above (``reading``/``drop`` of edge_weights, ``deg``/``deg_vis`` of
vertex_rows):

* ``reading="physical"``: Section 2.2 taken literally.  P is built in
  physical units with the origin at the edge midpoint; every numerically
  non-zero singular value (above sigma_1 * 15 * eps, the usual rank
  tolerance) is kept at first; while any of the 15 entries of the stored
  row P^+(1,:) has magnitude >= 1 the smallest kept one is dropped; the row
  of the plain pseudo-inverse is stored, with no graded correction and no
  fold.  The 3-node rows are the plain minimum-norm pseudo-inverse of the
  3 x 6 system in physical units (eq. 3nodes_intp), again with no fold.
* ``drop="all"``: the dropping rule tested on all 15 entries of the stored
  row (value and derivative weights in the edge frame), not only on the
  five value weights.
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


def hermite_weights(pts, anchor=2, rank_cap=14, drop="value", grad=False):
    """Row of the graded Hermite pseudo-inverse with the dropping rule.

    ``pts`` [b, 5, 2] in the edge frame.  ``drop``: "value" tests the five
    value weights, "all" every entry of the row.  Returns (w [b, 15] in the
    edge frame: (value, d/dx, d/dy) per node, rank [b]); with ``grad`` also
    g [b, 2, 15], rows 2 and 3 of the same operator (the x- and
    y-derivative of the fitted quartic at the midpoint, edge frame) at the
    final rank, their anchor value weight absorbing minus the sum of their
    value weights so that a constant has zero gradient.
    """
    tested = slice(0, 15, 3) if drop == "value" else slice(0, 15)
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
            big = (np.max(np.abs(wi[:, tested]), axis=1) >= 1.0) & (rv > 1)
            r[idx[big]] -= 1
            todo[idx[~big]] = False
    w[:, 3 * anchor] += 1.0 - w[:, 0::3].sum(axis=1)
    if not grad:
        return w, r
    g = np.empty((b, 2, 15))
    for rv in np.unique(r):
        idx = np.nonzero(r == rv)[0]
        g[idx] = graded_rows(U[idx], s[idx], V[idx], int(rv), top, [1, 2])
    g[:, :, 3 * anchor] -= g[:, :, 0::3].sum(axis=2)
    return w, r, g


def hermite_weights_physical(pts, grad=False):
    """First row of the plain pseudo-inverse of P in physical units with the
    dropping rule on all 15 entries (the literal reading of Section 2.2).

    ``pts`` [b, 5, 2] physical offsets from the edge midpoint.  Returns
    (w [b, 15] physical units: (value, d/dx, d/dy) per node, rank [b]); with
    ``grad`` also rows 2 and 3 at the final rank, g [b, 2, 15].
    """
    pts = np.asarray(pts, dtype=np.float64)
    U, s, V = svd_full(hermite_matrix(pts))
    r = np.count_nonzero(s > s[:, :1] * 15 * np.finfo(np.float64).eps, axis=1)
    w = np.empty((pts.shape[0], 15))
    g = np.empty((pts.shape[0], 2, 15))
    todo = np.ones(pts.shape[0], dtype=bool)
    while np.any(todo):
        for rv in np.unique(r[todo]):
            idx = np.nonzero(todo & (r == rv))[0]
            rv = int(rv)
            # rows 1..3 of V_r S_r^-1 U_r^T
            K = np.einsum("bjr,bmr->bjm", V[idx, 0:3, :rv] / s[idx, None, :rv],
                          U[idx, :, :rv])
            w[idx] = K[:, 0]
            g[idx] = K[:, 1:3]
            big = (np.max(np.abs(K[:, 0]), axis=1) >= 1.0) & (rv > 1)
            r[idx[big]] -= 1
            todo[idx[~big]] = False
    return (w, r, g) if grad else (w, r)


def three_node_weights_physical(pts, grad=False):
    """Value weights of the 3 x 6 system of eq. 3nodes_intp by the plain
    minimum-norm pseudo-inverse in physical units (no fold, no dropping);
    ``pts`` [b, 3, 2] physical offsets from the edge midpoint.  With
    ``grad`` also the x- and y-derivative rows at the midpoint [b, 2, 3]."""
    pts = np.asarray(pts, dtype=np.float64)
    A = basis.p(pts[..., 0], pts[..., 1], 2)                # [b, 3, 6]
    K = np.linalg.pinv(A)
    return (K[:, 0, :], K[:, 1:3, :]) if grad else K[:, 0, :]


def three_node_weights(pts, anchor, cap=0.0, grad=False):
    """Value weights of the graded 3 x 6 system (eq. 3nodes_intp) at the
    origin; ``pts`` [b, 3, 2], ``anchor`` local index of the side anchor.

    ``cap`` > 0 switches on a dropping rule for these systems (not in the
    paper, off by default): while a weight exceeds ``cap`` in magnitude the
    smallest kept singular value is dropped, as the 5-node rule does.  With
    ``grad`` also the x- and y-derivative rows of the same operator at the
    final rank [b, 2, 3] (the gradient of the fitted planar interpolant, or
    of the 1D quadratic along collinear nodes), the anchor absorbing minus
    their sums."""
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
                big = (np.max(np.abs(wi), axis=1) > cap) & (rv > 1)
            else:
                big = np.zeros(idx.size, dtype=bool)
            r[idx[big]] -= 1
            todo[idx[~big]] = False
    w[:, anchor] += 1.0 - w.sum(axis=1)
    if not grad:
        return w
    g = np.empty((w.shape[0], 2, 3))
    for rv in np.unique(r):
        idx = np.nonzero(r == rv)[0]
        g[idx] = graded_rows(U[idx], s[idx], V[idx], int(rv), top, [1, 2])
    g[:, :, anchor] -= g.sum(axis=2)
    return w, g


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
    # midpoint derivatives, physical units: d/dx and d/dy rows of the 5-node
    # operator [Ea, 2 sides, 2, 15] and of each 3-node one [Ea, 2, 3 subs, 2, 3]
    w5g: np.ndarray = None
    w3g: np.ndarray = None


# node order of each side within the six-node stencil (i-2 .. i+3)
SIDE_NODES = ((0, 1, 2, 3, 4), (5, 4, 3, 2, 1))


def edge_weights(topo, xy, period, edges=None, w3_cap=0.0, reading="graded",
                 drop="value"):
    """Weights of the given (active) edges, both sides.  ``reading``:
    "graded" (edge frame, graded pseudo-inverse, fold) or "physical" (the
    literal reading, see the module header); ``drop``: entries the 5-node
    dropping rule tests in the graded reading ("value" or "all")."""
    if reading not in ("graded", "physical") or drop not in ("value", "all"):
        raise ValueError((reading, drop))
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
    w5g = np.empty((Ea, 2, 2, 15))
    w3g = np.empty((Ea, 2, 3, 2, 3))
    for s_, nodes in enumerate(SIDE_NODES):
        pts = P[:, list(nodes), :]
        if reading == "physical":
            phys = pts * h[:, None, None]
            w, r, g = hermite_weights_physical(phys, grad=True)
            w5[:, s_], w5g[:, s_] = w, g
            rank[:, s_] = r
            for j in range(3):
                w3[:, s_, j], w3g[:, s_, j] = three_node_weights_physical(
                    phys[:, j:j + 3, :], grad=True)
            continue
        w, r, g = hermite_weights(pts, drop=drop, grad=True)
        # edge frame -> physical units: data (c, h c_x, h c_y), d/dx = d/dx_hat / h
        w[:, 1::3] *= h[:, None]
        w[:, 2::3] *= h[:, None]
        g[:, :, 0::3] /= h[:, None, None]
        w5[:, s_], w5g[:, s_] = w, g
        rank[:, s_] = r
        for j in range(3):
            w3[:, s_, j], g3 = three_node_weights(pts[:, j:j + 3, :], anchor=2 - j,
                                                  cap=w3_cap, grad=True)
            w3g[:, s_, j] = g3 / h[:, None, None]
    return EdgeWeights(edges=edges, n=n, h=h, w5=w5, w3=w3, rank=rank, w5g=w5g,
                       w3g=w3g)


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
