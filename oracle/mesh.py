"""Oracle topology and stencils (test infrastructure only).

Follows Section 2.1 (a curvilinear stencil is assembled for each edge by
extending it twice from each end point along the incident edge of smallest
deflection) and Section 2.3 (the divergence stencil of a vertex holds two
levels of neighbouring vertices and all edges between them).

Readings where the paper is silent:

* edges are the unique vertex pairs of the triangles, oriented from the
  smaller to the larger original vertex id; n = unit vector from the first
  to the second end;
* periodic displacements use the minimum image, ``d -= P`` if ``d > P/2``,
  ``d += P`` if ``d < -P/2``;
* "smallest deflection" = largest cosine ``dot/(|d|*|e|)`` between the
  incoming direction d and the candidate edge e, evaluated in float64 in
  exactly that order; ties go to the smallest original id; vertices already
  in the stencil are excluded; no candidate left is a mesh error;
* the backward extension (i-1, then i-2) is done before the forward one
  (i+2, then i+3), and each excludes everything chosen before it;
* the divergence stencil S(v) is v, its neighbours and their neighbours,
  sorted by original id; M(v) holds every edge with both ends in S(v),
  sorted by (first, second) end;
* an edge is active if it is in M(v) of at least one owned vertex; only
  active edges get an edge stencil.

Every floating-point operation here is a plain Python float operation, so
the stencil choice is reproducible bit for bit by any IEEE-754 float64 code
that evaluates the same expressions in the same order without contraction.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


class MeshError(ValueError):
    pass


def minimg(d, P):
    """Minimum-image displacement along one periodic direction (P = 0: none)."""
    if P:
        if d > 0.5 * P:
            return d - P
        if d < -0.5 * P:
            return d + P
    return d


def disp(xy, period, a, b):
    """Displacement x_b - x_a with the minimum-image convention."""
    return (minimg(float(xy[b, 0]) - float(xy[a, 0]), period[0]),
            minimg(float(xy[b, 1]) - float(xy[a, 1]), period[1]))


@dataclasses.dataclass
class Topology:
    nv: int
    edges: np.ndarray        # [E, 2] int64, (a, b), a < b, sorted
    adj: "Adjacency"         # sorted neighbour lists
    owned: np.ndarray        # [V] bool
    active: np.ndarray       # [E] bool
    stencil: np.ndarray      # [E, 6] int64 (i-2, i-1, i, i+1, i+2, i+3); -1 if inactive
    vnodes: dict             # vertex -> sorted S(v) (for the vertices in ``verts``)
    vedges: dict             # vertex -> edge indices of M(v), sorted by (a, b)
    verts: np.ndarray        # vertices whose divergence stencil was built


def edges_from_triangles(tri):
    """Unique vertex pairs of the triangles as (smaller, larger) id, sorted."""
    t = np.asarray(tri, dtype=np.int64)
    pairs = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]])
    pairs.sort(axis=1)
    return np.unique(pairs, axis=0)


class Adjacency:
    """Sorted neighbour lists, stored compactly; ``adj[v]`` is a list."""

    def __init__(self, nv, edges):
        a = np.concatenate([edges[:, 0], edges[:, 1]])
        b = np.concatenate([edges[:, 1], edges[:, 0]])
        order = np.lexsort((b, a))
        self.nbr = b[order]
        self.ptr = np.zeros(nv + 1, dtype=np.int64)
        np.cumsum(np.bincount(a, minlength=nv), out=self.ptr[1:])

    def __getitem__(self, v):
        return [int(x) for x in self.nbr[self.ptr[v]:self.ptr[v + 1]]]

    def __len__(self):
        return self.ptr.size - 1


def adjacency(nv, edges):
    return Adjacency(nv, np.asarray(edges, dtype=np.int64))


def _extend(xy, period, adj, used, p, q):
    """Next node beyond q on the path p -> q: the neighbour c of q, not yet
    used, whose edge q -> c deviates least from the direction p -> q."""
    dx, dy = disp(xy, period, p, q)
    dn = math.sqrt(dx * dx + dy * dy)
    best = -1
    bestc = -math.inf
    for c in adj[q]:
        if c in used:
            continue
        ex, ey = disp(xy, period, q, c)
        cs = (dx * ex + dy * ey) / (dn * math.sqrt(ex * ex + ey * ey))
        if cs > bestc:
            best, bestc = c, cs
    if best < 0:
        raise MeshError(f"edge stencil dead end at vertex {q}")
    return best


def edge_stencil(xy, period, adj, a, b):
    """Six-node curvilinear stencil (i-2, i-1, i, i+1, i+2, i+3) of the edge
    i=a -> i+1=b (Section 2.1, Fig. of the assembled stencil)."""
    used = {a, b}
    im1 = _extend(xy, period, adj, used, b, a)
    used.add(im1)
    im2 = _extend(xy, period, adj, used, a, im1)
    used.add(im2)
    ip2 = _extend(xy, period, adj, used, a, b)
    used.add(ip2)
    ip3 = _extend(xy, period, adj, used, b, ip2)
    return (im2, im1, a, b, ip2, ip3)


def vertex_stencil(adj, v):
    """S(v): v, its first and second ring (Section 2.3, double-level
    stencil), sorted by id."""
    s = {v}
    r1 = adj[v]
    s.update(r1)
    for u in r1:
        s.update(adj[u])
    return sorted(s)


def build(xy, tri, ghost_src, period, verts=None):
    """Topology, vertex stencils of ``verts`` (default: every owned vertex)
    and edge stencils of the edges they use."""
    xy = np.asarray(xy, dtype=np.float64)
    nv = xy.shape[0]
    period = (float(period[0]), float(period[1]))
    edges = edges_from_triangles(tri)
    adj = adjacency(nv, edges)
    owned = np.asarray(ghost_src) == -1
    if verts is None:
        verts = np.nonzero(owned)[0]
    vnodes = {}
    vedges = {}
    active = np.zeros(edges.shape[0], dtype=bool)
    key = edges[:, 0] * nv + edges[:, 1]      # row of a pair in the sorted edge list
    for v in verts:
        v = int(v)
        S = vertex_stencil(adj, v)
        Sset = set(S)
        pairs = []
        for a in S:
            for b in adj[a]:
                if b > a and b in Sset:
                    pairs.append((a, b))
        pairs.sort()
        pa = np.array(pairs, dtype=np.int64)
        M = np.searchsorted(key, pa[:, 0] * nv + pa[:, 1])
        vnodes[v] = S
        vedges[v] = [int(m) for m in M]
        active[M] = True
    stencil = np.full((edges.shape[0], 6), -1, dtype=np.int64)
    for k in np.nonzero(active)[0]:
        a, b = int(edges[k, 0]), int(edges[k, 1])
        stencil[k] = edge_stencil(xy, period, adj, a, b)
    return Topology(nv=nv, edges=edges, adj=adj, owned=owned, active=active,
                    stencil=stencil, vnodes=vnodes, vedges=vedges,
                    verts=np.asarray(verts, dtype=np.int64))


def rel(xy, period, origin, nodes):
    """Minimum-image positions of ``nodes`` relative to vertex ``origin``
    (vectorised; same formula as :func:`minimg`)."""
    d = xy[np.asarray(nodes)] - xy[origin][None, :]
    for k in (0, 1):
        P = period[k]
        if P:
            d[:, k] = np.where(d[:, k] > 0.5 * P, d[:, k] - P,
                               np.where(d[:, k] < -0.5 * P, d[:, k] + P, d[:, k]))
    return d
