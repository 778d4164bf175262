"""Pins of the oracle's other alternative readings (each an option compared
with the default on the same functions):

* ``drop="all"``: the dropping rule of Section 2.2 tested on all 15 entries
  of the stored row;
* ``branch="algorithm"``: Algorithm 1's order of the two branches, the
  opposite of eq. 2d_hweno_intp's;
* ``deg_inv=4``: the divergence fit of eq. flux_polynomials at degree 4.
"""
import math

import numpy as np
import numpy.polynomial.polynomial as npp
import torch

from oracle import basis, mesh as omesh, scheme, weights as ow
from paper_2109_01286_amd import inputs

from .test_oracle_pins import _mesh_vertex, _random_stencils


def test_drop_all_leaves_every_entry_below_one_and_keeps_cubics():
    """After the rule on all 15 entries no entry of the stored row reaches
    one (unless the rank reached one), at least as many singular values are
    dropped as under the value-only rule, and the graded rows still
    reproduce every cubic at whatever rank the rule stopped."""
    rng = np.random.default_rng(37)
    S = _random_stencils(rng, 300, sd_ang=math.pi / 6)
    w, r = ow.hermite_weights(S, drop="all")
    wv, rv = ow.hermite_weights(S)
    pre = w.copy()
    pre[:, 6] -= 1.0 - w[:, 0::3].sum(axis=1)    # undo the fold at the anchor
    assert ((np.abs(np.delete(pre, 6, axis=1)).max(axis=1) < 1.0) | (r == 1)).all()
    assert (r <= rv).all() and (r < rv).any()
    for j in range(S.shape[0]):
        m = np.zeros((4, 4))
        for a, b in basis.exponents(3):
            m[a, b] = rng.standard_normal()
        x, y = S[j, :, 0], S[j, :, 1]
        data = np.stack([npp.polyval2d(x, y, m), npp.polyval2d(x, y, npp.polyder(m, axis=0)),
                         npp.polyval2d(x, y, npp.polyder(m, axis=1))], 1).ravel()
        assert abs(w[j] @ data - m[0, 0]) <= 1e-11 * (1.0 + np.abs(m).sum())


def test_algorithm_branch_order_takes_the_other_branch():
    """With the paper switch, Algorithm 1's order takes the 3-node branch
    exactly where eq. 2d_hweno_intp's order takes the 5-node one: the two
    masks are bitwise complements, edge by edge, on the same state."""
    m = inputs.jittered_grid(11, 11, 10.0, 10.0, (True, True), 0, seed=3, jitter=0.2)
    U = torch.as_tensor(inputs.isentropic_vortex(m, beta=5.0))
    masks = []
    for br in ("equation", "algorithm"):
        sc = scheme.Scheme(m.xy, m.tri, m.ghost_src, m.period,
                           scheme.Options(branch=br, w3_cap=2.0))
        masks.append(np.asarray(sc.edge_states(U, "paper")[2]).astype(np.int64))
    assert np.array_equal(masks[1], 255 - masks[0])
    assert 0 < np.count_nonzero(masks[0]) < masks[0].size


def test_degree4_divergence_rows_exact_for_quartic_fluxes():
    """At degree 4 the rows d0, dx, dy give the exact divergence and its
    derivatives for fluxes f, g of degree 4 (data from numpy.polynomial at
    the stencil's vertices and edge midpoints), and not for degree 5."""
    m, topo, verts = _mesh_vertex()
    rng = np.random.default_rng(41)
    vr = ow.vertex_rows(topo, m.xy, m.period, verts, deg=4)
    for deg, exact in ((4, True), (5, False)):
        worst = 0.0
        for j, v in enumerate(verts):
            S, M = topo.vnodes[int(v)], topo.vedges[int(v)]
            cf, cg = np.zeros((6, 6)), np.zeros((6, 6))
            for a, b in basis.exponents(deg):
                cf[a, b], cg[a, b] = rng.standard_normal(2)
            X = omesh.rel(m.xy, m.period, int(v), S)
            E = topo.edges[M]
            A = omesh.rel(m.xy, m.period, int(v), E[:, 0])
            D = np.array([omesh.rel(m.xy, m.period, int(a), [int(b)])[0] for a, b in E])
            mid = A + 0.5 * D
            nrm = D / np.hypot(D[:, 0], D[:, 1])[:, None]
            rhs = np.empty(2 * len(S) + len(M))
            rhs[0:2 * len(S):2] = npp.polyval2d(X[:, 0], X[:, 1], cf)
            rhs[1:2 * len(S):2] = npp.polyval2d(X[:, 0], X[:, 1], cg)
            rhs[2 * len(S):] = (npp.polyval2d(mid[:, 0], mid[:, 1], cf) * nrm[:, 0]
                                + npp.polyval2d(mid[:, 0], mid[:, 1], cg) * nrm[:, 1])
            d = vr.d[j]
            at0 = lambda c, kx, ky: npp.polyval2d(0.0, 0.0, npp.polyder(npp.polyder(c, m=kx, axis=0), m=ky, axis=1))
            want = np.array([at0(cf, 1, 0) + at0(cg, 0, 1),
                             at0(cf, 2, 0) + at0(cg, 1, 1),
                             at0(cf, 1, 1) + at0(cg, 0, 2)])
            scale = np.abs(d).sum(1) * np.abs(rhs).max()
            worst = max(worst, float((np.abs(d @ rhs - want) / scale).max()))
        if exact:
            assert worst <= 1e-10, worst
        else:
            assert worst > 1e-6, worst
