"""Shared test plumbing: building oracle and library views of one mesh and
mapping oracle arrays into the library's layout (no arithmetic of the
method here)."""
import numpy as np

from oracle import scheme as osch
from paper_2109_01286_amd import hfd


def lib_solver(m, device, **opts):
    return hfd.Solver(m.xy, m.tri, m.ghost_src, m.period, device=device, **opts)


def edge_map(S, topo):
    """Library edge j -> row of the oracle's sorted edge list."""
    ends, st = S.export_edges()
    key = topo.edges[:, 0] * S.nv + topo.edges[:, 1]
    idx = np.searchsorted(key, ends[:, 0].astype(np.int64) * S.nv + ends[:, 1])
    assert np.array_equal(key[idx], ends[:, 0].astype(np.int64) * S.nv + ends[:, 1])
    return idx


def oracle_weights_for_lib(S, sc):
    """Oracle weights arranged as the library's export/import layout."""
    emap = edge_map(S, sc.topo)
    pos = sc.edge_pos[emap]
    assert (pos >= 0).all()
    w5 = sc.ew.w5[pos]
    w3 = sc.ew.w3[pos]
    rank = sc.ew.rank[pos]
    vptr, vn, eptr, ve = S.export_vertex_stencils()
    vindex = {int(v): j for j, v in enumerate(sc.vr.verts)}
    dv = np.empty((vptr[-1], 6))
    de = np.empty((eptr[-1], 3))
    dvis = np.empty((vptr[-1], 5)) if sc.vr.dvis[0] is not None else None
    for k in range(S.n_owned):
        v = int(S.old_of_new[k])
        j = vindex[v]
        d = sc.vr.d[j]
        Sv = sc.topo.vnodes[v]
        Mv = sc.topo.vedges[v]
        N = len(Sv)
        # library slot -> oracle slot (same sets, possibly another order)
        npos = {u: i for i, u in enumerate(Sv)}
        epos = {e: i for i, e in enumerate(Mv)}
        ns = np.array([npos[int(u)] for u in vn[vptr[k]:vptr[k + 1]]])
        es = np.array([epos[int(emap[m])] for m in ve[eptr[k]:eptr[k + 1]]])
        assert ns.size == N and es.size == len(Mv)
        dv[vptr[k]:vptr[k + 1]] = np.stack([d[0, 2 * ns], d[0, 2 * ns + 1],
                                            d[1, 2 * ns], d[1, 2 * ns + 1],
                                            d[2, 2 * ns], d[2, 2 * ns + 1]], 1)
        de[eptr[k]:eptr[k + 1]] = d[:, 2 * N + es].T
        if dvis is not None:
            dvis[vptr[k]:vptr[k + 1]] = sc.vr.dvis[j][:, ns].T
    return dict(w5=w5, w3=w3, rank=rank, dv=dv, de=de, dvis=dvis, emap=emap, pos=pos)


def oracle_scheme(m, **kw):
    return osch.Scheme(m.xy, m.tri, m.ghost_src, m.period, osch.Options(**kw))


def same_nans(a, b):
    """Both sides must be non-finite at exactly the same places (the method
    can produce NaN, e.g. negative pressure; the GPU must agree where)."""
    fa, fb = ~np.isfinite(a), ~np.isfinite(b)
    assert np.array_equal(fa, fb), f"non-finite entries differ: {fa.sum()} vs {fb.sum()}"
    return ~fa


def block_rel_err(a, b, owned):
    """Max over the three blocks (w, w_x, w_y) of ||a - b|| / ||b|| over the
    owned vertices, finite entries only (non-finite ones must coincide)."""
    out = []
    for k in range(3):
        x = a[4 * k:4 * k + 4][:, owned]
        y = b[4 * k:4 * k + 4][:, owned]
        f = same_nans(x, y)
        out.append(np.linalg.norm((x - y)[f]) / max(np.linalg.norm(y[f]), 1e-300))
    return max(out)


def cancellation_scale(sc, U, switch):
    """Per-vertex sums of |coefficient| * |flux datum| of the oracle's
    divergence dot products, [12, V]: the scale against which float64
    rounding of the residual is measured when large fluxes cancel."""
    import torch

    from oracle import gas
    o = sc.opts
    Ut = torch.as_tensor(U)
    W = sc.fill_ghosts(Ut)
    _, _, _, h = sc.edge_states(Ut, switch)
    wn = W[0:4, sc.vs_node].T
    f = gas.flux_f(wn, o.gamma).abs()
    g = gas.flux_g(wn, o.gamma).abs()
    c = sc.vs_c.abs()
    nvt = sc.verts.numel()
    acc = torch.zeros(nvt, 3, 4, dtype=torch.float64)
    for k in range(3):
        acc[:, k] = acc[:, k].index_add(0, sc.vs_own, c[:, 2 * k:2 * k + 1] * f
                                        + c[:, 2 * k + 1:2 * k + 2] * g)
        acc[:, k] = acc[:, k].index_add(0, sc.es_own, sc.es_c[:, k:k + 1].abs()
                                        * h[sc.es_edge].abs())
    if o.mu > 0.0:
        fv, gv = gas.viscous_flux(wn, W[4:8, sc.vs_node].T, W[8:12, sc.vs_node].T,
                                  o.gamma, o.mu, o.prandtl, o.gas_R)
        r = sc.vs_v.abs()
        pairs = [(0, 1), (2, 3), (3, 4)]
        for k, (a, b) in enumerate(pairs):
            acc[:, k] = acc[:, k].index_add(0, sc.vs_own, r[:, a:a + 1] * fv.abs()
                                            + r[:, b:b + 1] * gv.abs())
    out = np.zeros((12, sc.nv))
    out[:, sc.verts.numpy()] = acc.reshape(nvt, 12).T.numpy()
    return out


def residual_within(got, ref, scale, owned, rel=1e-12, abs_rel=1e-14, elem=4.0):
    """Per block (w, w_x, w_y): ||got - ref|| <= rel ||ref|| + abs_rel ||scale||
    (L2 over the block), and element by element |got - ref| <= elem (rel
    max|ref| + abs_rel scale), so that an error at a few vertices is not
    diluted by the norm.  Returns the largest fraction of a bound used."""
    worst = 0.0
    for k in range(3):
        x = got[4 * k:4 * k + 4][:, owned]
        y = ref[4 * k:4 * k + 4][:, owned]
        s = scale[4 * k:4 * k + 4][:, owned]
        f = same_nans(x, y) & np.isfinite(s)
        tol = rel * np.linalg.norm(y[f]) + abs_rel * np.linalg.norm(s[f])
        q = np.linalg.norm((x - y)[f]) / tol
        assert np.isfinite(q)
        tol_e = elem * (rel * np.abs(y[f]).max() + abs_rel * s[f])
        q_e = np.max(np.abs((x - y)[f]) / tol_e)
        assert np.isfinite(q_e)
        worst = max(worst, q, q_e)
    return worst
