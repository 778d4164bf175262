"""Host setup of the library (C++) against the oracle: edges, six-node
stencils, vertex stencils, active set and renumbering must agree bit for
bit (integer results decided by float64 comparisons in the same order)."""
import numpy as np
import pytest

from oracle import mesh as omesh
from paper_2109_01286_amd import inputs

from ._helpers import edge_map, lib_solver

CASES = [("vortex21", None, {}), ("riemann201", 31, {}), ("shockvortex2049", 25, {}),
         ("tgv513", 33, {}), ("vortex257", 33, {"order": "none"}),
         ("riemann201", 31, {"order": "rcm"}), ("vortex21", None, {"order": "rcm"}),
         # the Delaunay mesh with the embedded circle of the circular Sod case
         ("sod_circle", 31, {})]


@pytest.mark.parametrize("name,scale,opts", CASES)
def test_stencils_bit_exact(name, scale, opts):
    m, _, _ = inputs.workload(name, scale)
    S = lib_solver(m, -1, **opts)
    topo = omesh.build(m.xy, m.tri, m.ghost_src, m.period)
    emap = edge_map(S, topo)
    assert set(emap.tolist()) == set(np.nonzero(topo.active)[0].tolist())
    ends, st = S.export_edges()
    assert np.array_equal(topo.stencil[emap], st.astype(np.int64))
    vptr, vn, eptr, ve = S.export_vertex_stencils()
    owned = np.nonzero(m.ghost_src == -1)[0]
    assert sorted(S.old_of_new[:S.n_owned].tolist()) == owned.tolist()
    for k in range(S.n_owned):
        v = int(S.old_of_new[k])
        # same sets; the library orders the slots by internal index
        assert sorted(vn[vptr[k]:vptr[k + 1]].tolist()) == topo.vnodes[v]
        assert sorted(emap[ve[eptr[k]:eptr[k + 1]]].tolist()) == topo.vedges[v]
        assert np.all(np.diff(ve[eptr[k]:eptr[k + 1]]) > 0)
        assert np.all(np.diff(S.new_of_old[vn[vptr[k]:vptr[k + 1]]]) > 0) or \
            (m.ghost_src != -1).any()


def test_renumbering_of_a_shuffled_mesh_gives_the_same_stencils():
    m, _, _ = inputs.workload("riemann201", 21)
    ms = inputs.shuffled(m, seed=9)
    S = lib_solver(ms, -1)
    topo = omesh.build(ms.xy, ms.tri, ms.ghost_src, ms.period)
    emap = edge_map(S, topo)
    _, st = S.export_edges()
    assert np.array_equal(topo.stencil[emap], st.astype(np.int64))
    # Hilbert order keeps neighbours close: mean index distance along edges
    ends, _ = S.export_edges()
    a, b = S.new_of_old[ends[:, 0]], S.new_of_old[ends[:, 1]]
    assert np.median(np.abs(a - b)) < 0.05 * S.nv
    # owned vertices first, then Dirichlet, then copying ghosts
    g = ms.ghost_src[S.old_of_new]
    assert (g[:S.n_owned] == -1).all() and (g[S.n_owned:] != -1).all()


def test_reverse_cuthill_mckee_bounds_the_bandwidth():
    """Reverse Cuthill-McKee numbering of a shuffled 41 x 41 lattice: every
    edge between owned vertices joins indices at most about two lattice
    rows apart (the breadth-first levels are anti-diagonals), against the
    whole index range for the shuffled input order; owned vertices first."""
    m, _, _ = inputs.workload("riemann201", 41)
    ms = inputs.shuffled(m, seed=9)
    band = {}
    for o in ("none", "rcm"):
        S = lib_solver(ms, -1, order=o)
        ends, _ = S.export_edges()
        a, b = S.new_of_old[ends[:, 0]], S.new_of_old[ends[:, 1]]
        own = (a < S.n_owned) & (b < S.n_owned)
        band[o] = int(np.abs(a - b)[own].max())
        g = ms.ghost_src[S.old_of_new]
        assert (g[:S.n_owned] == -1).all() and (g[S.n_owned:] != -1).all()
        assert sorted(S.old_of_new.tolist()) == list(range(S.nv))
    assert band["rcm"] <= 2 * 41
    assert band["none"] > 10 * band["rcm"]


def test_unknown_order_is_rejected():
    m, _, _ = inputs.workload("vortex21", 9)
    with pytest.raises(Exception):
        lib_solver(m, -1, order=5)


def test_sizes_match_the_lattice_recipe():
    m, _, _ = inputs.workload("riemann201", 201)
    S = lib_solver(m, -1)
    assert S.info["n_owned"] == 40401 and S.info["nv"] == 44521
    assert S.info["n_edges_mesh"] == 132720


def test_embedded_circle_mesh():
    """The circular Sod meshes (Section 3.3) carry the circle r = 0.5: every
    chord between consecutive circle vertices is a mesh edge, the circle
    vertices take the outer state and every other vertex the state its
    distance gives, and the triangles around owned vertices are not
    degenerate (smallest angle above 20 degrees)."""
    for n in (25, 51):
        m, circle = inputs.embedded_circle_grid(n)
        edges = set()
        for t in m.tri:
            for a, b in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0])):
                edges.add((min(a, b), max(a, b)))
        nc = circle.size
        assert nc == round(np.pi / m.h[0])
        r = np.hypot(m.xy[circle, 0] - 1.0, m.xy[circle, 1] - 1.0)
        assert np.allclose(r, 0.5, atol=1e-15)
        for k in range(nc):
            a, b = circle[k], circle[(k + 1) % nc]
            assert (min(a, b), max(a, b)) in edges
        U = inputs.circular_sod(m, on_circle=circle)
        assert np.all(U[0, circle] == 0.125)
        d = np.hypot(m.xy[:, 0] - 1.0, m.xy[:, 1] - 1.0)
        other = np.ones(m.nv, bool)
        other[circle] = False
        assert np.all(U[0, other & (d < 0.5)] == 1.0) and np.all(U[0, other & (d > 0.5)] == 0.125)
        x = m.xy[m.tri]
        ang = []
        for i in range(3):
            u = x[:, (i + 1) % 3] - x[:, i]
            v = x[:, (i + 2) % 3] - x[:, i]
            ang.append(np.degrees(np.arccos(np.clip(
                (u * v).sum(1) / np.linalg.norm(u, axis=1) / np.linalg.norm(v, axis=1), -1, 1))))
        near = (m.ghost_src[m.tri] == -1).any(1)
        assert np.min(np.minimum.reduce(ang)[near]) > 20.0
