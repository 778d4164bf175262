"""Seeded synthetic inputs: triangle meshes and initial states.

This module is shared by the tests, the benchmark and the CPU oracle's
callers.  It holds no arithmetic of the numerical method itself: it only
generates meshes (jittered, randomly split lattices that stand in for the
Delaunay meshes of the paper's test cases) and evaluates closed-form
initial conditions (isentropic vortex of the paper's Section 3.1, a
four-quadrant 2D Riemann problem, a decaying Taylor-Green vortex, a
Mach 1.1 normal shock with an upstream vortex, and the steady Couette flow
of Section 3.2) together with their exact spatial derivatives, because the
method evolves w, w_x and w_y.

State layout everywhere: ``U[12, V]`` float64, rows ``q + 4*k`` with
``q`` = (rho, rho*u, rho*v, E) and ``k`` = (value, d/dx, d/dy).

Mesh recipe ``G(nx, ny, Lx, Ly, periodic, G, seed)``:

* lattice spacing ``h = L/(n-1)`` per direction;
* a periodic direction identifies the last row/column with the first
  (``n-1`` unique points, coordinates in ``[0, L)``);
* a non-periodic direction keeps all ``n`` points and adds ``G`` ghost rows
  outside the domain on each side; vertices on the domain's boundary lines
  are not jittered;
* ``numpy.random.default_rng(seed)`` draws, in this order, one diagonal bit
  per cell (0: triangles (a,b,d),(b,c,d); 1: (a,b,c),(a,c,d), counter-
  clockwise with a=(i,j), b=(i+1,j), c=(i+1,j+1), d=(i,j+1)), then a jitter
  ``U(-0.2h, 0.2h)`` per vertex and direction;
* vertex id ``= j*nxv + i`` (x fastest).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Mesh:
    xy: np.ndarray          # [V, 2] float64
    tri: np.ndarray         # [T, 3] int32, counter-clockwise
    ghost_src: np.ndarray   # [V] int32: -1 owned, >=0 copy source, -2 Dirichlet
    period: tuple           # (Px, Py), 0.0 = not periodic in that direction
    shape: tuple            # (nxv, nyv) lattice points actually stored
    h: tuple                # (hx, hy) lattice spacing
    ij: np.ndarray          # [V, 2] int lattice indices (ghosts negative / >= n)

    @property
    def nv(self):
        return self.xy.shape[0]

    @property
    def owned(self):
        return self.ghost_src == -1

    def n_owned(self):
        return int(np.count_nonzero(self.ghost_src == -1))


def jittered_grid(nx, ny, Lx, Ly, periodic=(True, True), ghost_layers=0,
                  seed=0, jitter=0.2, dirichlet_sides=()):
    """Jittered, randomly split lattice (recipe in the module docstring).

    ``dirichlet_sides`` lists sides among ('xlo', 'xhi', 'ylo', 'yhi') whose
    ghost vertices are Dirichlet (-2) instead of copies of the nearest
    boundary vertex (transmissive).
    """
    px, py = bool(periodic[0]), bool(periodic[1])
    G = int(ghost_layers)
    hx = Lx / (nx - 1)
    hy = Ly / (ny - 1)
    if px:
        ix = np.arange(nx - 1)
    else:
        ix = np.arange(-G, nx + G)
    if py:
        iy = np.arange(ny - 1)
    else:
        iy = np.arange(-G, ny + G)
    nxv, nyv = ix.size, iy.size
    I, J = np.meshgrid(ix, iy)          # [nyv, nxv]
    I = I.ravel()
    J = J.ravel()
    V = I.size
    ncx = nxv if px else nxv - 1
    ncy = nyv if py else nyv - 1

    rng = np.random.default_rng(seed)
    bits = rng.integers(0, 2, size=(ncy, ncx))
    jit = rng.uniform(-jitter, jitter, size=(V, 2))

    xy = np.empty((V, 2))
    xy[:, 0] = I * hx + jit[:, 0] * hx
    xy[:, 1] = J * hy + jit[:, 1] * hy
    on_line = np.zeros(V, dtype=bool)
    if not px:
        on_line |= (I == 0) | (I == nx - 1)
    if not py:
        on_line |= (J == 0) | (J == ny - 1)
    xy[on_line, 0] = I[on_line] * hx
    xy[on_line, 1] = J[on_line] * hy
    if px:
        xy[:, 0] = np.mod(xy[:, 0], Lx)
    if py:
        xy[:, 1] = np.mod(xy[:, 1], Ly)

    def vid(ci, cj):
        if px:
            ci = ci % nxv
        if py:
            cj = cj % nyv
        return cj * nxv + ci

    cj, ci = np.meshgrid(np.arange(ncy), np.arange(ncx), indexing="ij")
    a = vid(ci, cj)
    b = vid(ci + 1, cj)
    c = vid(ci + 1, cj + 1)
    d = vid(ci, cj + 1)
    b0 = bits == 0
    t1 = np.where(b0[..., None], np.stack([a, b, d], -1), np.stack([a, b, c], -1))
    t2 = np.where(b0[..., None], np.stack([b, c, d], -1), np.stack([a, c, d], -1))
    tri = np.stack([t1, t2], axis=2).reshape(-1, 3).astype(np.int32)

    ghost_src = np.full(V, -1, dtype=np.int32)
    gx = ((I < 0) | (I > nx - 1)) if not px else np.zeros(V, bool)
    gy = ((J < 0) | (J > ny - 1)) if not py else np.zeros(V, bool)
    ghost = gx | gy
    if np.any(ghost):
        ci_ = np.clip(I, 0, nx - 1) if not px else I
        cj_ = np.clip(J, 0, ny - 1) if not py else J
        src = (cj_ - iy[0]) * nxv + (ci_ - ix[0])
        ghost_src[ghost] = src[ghost].astype(np.int32)
        for side in dirichlet_sides:
            m = {"xlo": I < 0, "xhi": I > nx - 1,
                 "ylo": J < 0, "yhi": J > ny - 1}[side]
            ghost_src[ghost & m] = -2
    period = (Lx if px else 0.0, Ly if py else 0.0)
    return Mesh(xy=xy, tri=tri, ghost_src=ghost_src, period=period,
                shape=(nxv, nyv), h=(hx, hy), ij=np.stack([I, J], 1))


def equilateral_grid(nx, ny, Lx, jitter=0.0, seed=0):
    """Periodic lattice of equilateral triangles (every vertex of valence
    six, the ideal of an isotropic Delaunay mesh): ``nx`` points per row at
    spacing h = Lx/nx, ``ny`` rows (even) at spacing h sqrt(3)/2, odd rows
    shifted by h/2; period (Lx, ny h sqrt(3)/2).  ``jitter`` moves every
    vertex by U(-jitter h, jitter h) per direction
    (``numpy.random.default_rng(seed)``)."""
    if ny % 2:
        raise ValueError("ny must be even for a periodic equilateral lattice")
    h = Lx / nx
    hy = h * math.sqrt(3.0) / 2.0
    Ly = ny * hy
    J, I = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    I, J = I.ravel(), J.ravel()
    rng = np.random.default_rng(seed)
    jit = rng.uniform(-jitter, jitter, size=(I.size, 2)) * h
    xy = np.stack([np.mod((I + 0.5 * (J % 2)) * h + jit[:, 0], Lx),
                   np.mod(J * hy + jit[:, 1], Ly)], 1)
    vid = lambda i, j: (j % ny) * nx + (i % nx)
    tri = []
    for j in range(ny):
        for i in range(nx):
            if j % 2 == 0:
                tri.append((vid(i, j), vid(i + 1, j), vid(i, j + 1)))
                tri.append((vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)))
            else:
                tri.append((vid(i, j), vid(i + 1, j), vid(i + 1, j + 1)))
                tri.append((vid(i, j), vid(i + 1, j + 1), vid(i, j + 1)))
    return Mesh(xy=xy, tri=np.asarray(tri, dtype=np.int32),
                ghost_src=np.full(I.size, -1, dtype=np.int32), period=(Lx, Ly),
                shape=(nx, ny), h=(h, hy), ij=np.stack([I, J], 1))


def embedded_circle_grid(n, L=2.0, center=(1.0, 1.0), radius=0.5, ghost_layers=5, seed=7,
                         clearance=0.6):
    """The jittered lattice G(n, n, L, L, non-periodic, ghost_layers, seed)
    with a circle embedded in it (Section 3.3: the meshes of the circular Sod
    problem carry the circle r = radius so that the initial discontinuity
    lies on mesh edges).  Lattice vertices (owned, not on a boundary line)
    closer than ``clearance`` h to the circle are removed, round(2 pi r / h)
    vertices are placed on the circle at equal angles, and the whole point
    set is triangulated by Delaunay (scipy.spatial).  The circle vertices
    follow the lattice vertices; ``circle`` (returned with the mesh) lists
    them in angular order.  Ghost vertices keep their sources."""
    import scipy.spatial

    base = jittered_grid(n, n, L, L, (False, False), ghost_layers, seed=seed)
    h = base.h[0]
    c = np.asarray(center, dtype=np.float64)
    dist = np.abs(np.hypot(base.xy[:, 0] - c[0], base.xy[:, 1] - c[1]) - radius)
    I, J = base.ij[:, 0], base.ij[:, 1]
    interior = (base.ghost_src == -1) & (I > 0) & (I < n - 1) & (J > 0) & (J < n - 1)
    keep = ~(interior & (dist < clearance * h))
    old = np.nonzero(keep)[0]
    new_of_old = -np.ones(base.nv, dtype=np.int64)
    new_of_old[old] = np.arange(old.size)
    nc = int(round(2.0 * math.pi * radius / h))
    th = 2.0 * math.pi * np.arange(nc) / nc
    circ = np.stack([c[0] + radius * np.cos(th), c[1] + radius * np.sin(th)], 1)
    xy = np.concatenate([base.xy[old], circ])
    gs = base.ghost_src[old].astype(np.int64)
    gs = np.where(gs >= 0, new_of_old[np.maximum(gs, 0)], gs)
    if np.any(gs[base.ghost_src[old] >= 0] < 0):
        raise ValueError("a ghost source was removed")
    ghost_src = np.concatenate([gs, np.full(nc, -1)]).astype(np.int32)
    tri = scipy.spatial.Delaunay(xy).simplices.astype(np.int64)
    a, b, cc = xy[tri[:, 0]], xy[tri[:, 1]], xy[tri[:, 2]]
    cross = (b[:, 0] - a[:, 0]) * (cc[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (cc[:, 0] - a[:, 0])
    tri = np.where((cross < 0)[:, None], tri[:, [0, 2, 1]], tri).astype(np.int32)
    ij = np.concatenate([base.ij[old], np.full((nc, 2), np.iinfo(np.int64).min)])
    m = Mesh(xy=xy, tri=tri, ghost_src=ghost_src, period=(0.0, 0.0),
             shape=base.shape, h=base.h, ij=ij)
    return m, np.arange(old.size, old.size + nc)


def shuffled(mesh: Mesh, seed=0):
    """Same mesh with vertices renumbered by a seeded random permutation.

    Real mesh generators emit vertices in no useful order; this is the input
    that exercises a solver's own renumbering.
    """
    rng = np.random.default_rng(seed)
    perm = rng.permutation(mesh.nv)          # new position -> old id
    inv = np.empty_like(perm)
    inv[perm] = np.arange(mesh.nv)
    gs = mesh.ghost_src[perm].copy()
    gs[gs >= 0] = inv[gs[gs >= 0]]
    return Mesh(xy=mesh.xy[perm].copy(), tri=inv[mesh.tri].astype(np.int32),
                ghost_src=gs.astype(np.int32), period=mesh.period,
                shape=mesh.shape, h=mesh.h, ij=mesh.ij[perm].copy())


# ----------------------------------------------------------------------------
# Closed-form initial states with exact derivatives
# ----------------------------------------------------------------------------

def prim_to_state(gamma, rho, u, v, p, drho, du, dv, dp):
    """Conservative state and its gradient from primitive fields.

    ``d*`` are pairs (d/dx, d/dy).  Returns U[12, V].
    """
    V = np.broadcast_to(rho, np.shape(rho)).size
    U = np.zeros((12, V))
    q2 = u * u + v * v
    U[0] = rho
    U[1] = rho * u
    U[2] = rho * v
    U[3] = p / (gamma - 1.0) + 0.5 * rho * q2
    for k in (0, 1):
        r_, u_, v_, p_ = drho[k], du[k], dv[k], dp[k]
        U[4 * (k + 1) + 0] = r_
        U[4 * (k + 1) + 1] = r_ * u + rho * u_
        U[4 * (k + 1) + 2] = r_ * v + rho * v_
        U[4 * (k + 1) + 3] = (p_ / (gamma - 1.0) + 0.5 * r_ * q2
                              + rho * (u * u_ + v * v_))
    return U


def _rel(xy, center, period):
    d = xy - np.asarray(center)[None, :]
    for k in (0, 1):
        P = period[k]
        if P:
            d[:, k] -= P * np.round(d[:, k] / P)
    return d[:, 0], d[:, 1]


def _vortex_prims(xb, yb, beta, gamma, scale):
    """Isentropic vortex perturbation (paper Section 3.1) in coordinates
    scaled by ``scale``; returns temperature-like factor and velocity
    perturbation with derivatives w.r.t. physical x, y."""
    r2 = xb * xb + yb * yb
    kap = (gamma - 1.0) * beta * beta / (8.0 * gamma * math.pi ** 2)
    phi = np.exp(1.0 - r2)
    T = 1.0 - kap * phi
    dT = (2.0 * kap * phi * xb / scale, 2.0 * kap * phi * yb / scale)
    a = beta / (2.0 * math.pi)
    psi = np.exp(0.5 * (1.0 - r2))
    du_ = -a * yb * psi
    dv_ = a * xb * psi
    ddu = (a * xb * yb * psi / scale, -a * psi * (1.0 - yb * yb) / scale)
    ddv = (a * psi * (1.0 - xb * xb) / scale, -a * xb * yb * psi / scale)
    return T, dT, du_, ddu, dv_, ddv


def isentropic_vortex(mesh: Mesh, center=(5.0, 5.0), beta=5.0, gamma=1.4,
                      free=(1.0, 1.0), t=0.0):
    """Paper Section 3.1 vortex on a free stream (rho, u, v, p) =
    (1, free_u, free_v, 1), advected exactly to time ``t``."""
    c = (center[0] + free[0] * t, center[1] + free[1] * t)
    xb, yb = _rel(mesh.xy, c, mesh.period)
    T, dT, du_, ddu, dv_, ddv = _vortex_prims(xb, yb, beta, gamma, 1.0)
    g1 = 1.0 / (gamma - 1.0)
    rho = T ** g1
    drho = tuple(g1 * rho / T * d for d in dT)
    p = rho ** gamma
    dp = tuple(gamma * rho ** (gamma - 1.0) * d for d in drho)
    u = free[0] + du_
    v = free[1] + dv_
    return prim_to_state(gamma, rho, u, v, p, drho, ddu, ddv, dp)


def riemann_quadrants(mesh: Mesh, gamma=1.4, states=None, split=(0.5, 0.5)):
    """Four-quadrant piecewise-constant state, zero gradients.

    ``states`` (rho, u, v, p) in the order NE, NW, SW, SE; x >= split_x is
    east, y >= split_y is north.
    """
    if states is None:
        states = ((1.5, 0.0, 0.0, 1.5), (0.5323, 1.206, 0.0, 0.3),
                  (0.138, 1.206, 1.206, 0.029), (0.5323, 0.0, 1.206, 0.3))
    x, y = mesh.xy[:, 0], mesh.xy[:, 1]
    east = x >= split[0]
    north = y >= split[1]
    q = np.where(north & east, 0, np.where(north, 1, np.where(east, 3, 2)))
    S = np.asarray(states, dtype=np.float64)[q]
    z = np.zeros(mesh.nv)
    return prim_to_state(gamma, S[:, 0], S[:, 1], S[:, 2], S[:, 3],
                         (z, z), (z, z), (z, z), (z, z))


def taylor_green(mesh: Mesh, gamma=1.4, mach=0.1, rho0=1.0, U0=1.0, R=1.0,
                 t=0.0, nu=0.0):
    """Compressible decaying Taylor-Green vortex on [0, 2pi]^2 at low Mach
    number: p0 = rho0 U0^2/(gamma M^2), isothermal density rho = p/(R T0)
    with T0 = p0/(rho0 R).  With ``nu`` and ``t`` the incompressible decay
    factors exp(-2 nu t) (velocity) and exp(-4 nu t) (pressure perturbation)
    are applied."""
    p0 = rho0 * U0 * U0 / (gamma * mach * mach)
    T0 = p0 / (rho0 * R)
    fu = math.exp(-2.0 * nu * t)
    fp = fu * fu
    x, y = mesh.xy[:, 0], mesh.xy[:, 1]
    sx, cx, sy, cy = np.sin(x), np.cos(x), np.sin(y), np.cos(y)
    u = U0 * fu * sx * cy
    v = -U0 * fu * cx * sy
    du = (U0 * fu * cx * cy, -U0 * fu * sx * sy)
    dv = (U0 * fu * sx * sy, -U0 * fu * cx * cy)
    A = rho0 * U0 * U0 / 4.0 * fp
    p = p0 + A * (np.cos(2 * x) + np.cos(2 * y))
    dp = (-2.0 * A * np.sin(2 * x), -2.0 * A * np.sin(2 * y))
    rho = p / (R * T0)
    drho = (dp[0] / (R * T0), dp[1] / (R * T0))
    return prim_to_state(gamma, rho, u, v, p, drho, du, dv, dp)


def couette(mesh: Mesh, L=10.0, y0=5.0, u0=0.5, T_top=1.5, T_bottom=1.0, p=1.0,
            mu=0.1, K=0.01, cp=10.0, gamma=1.4):
    """Steady compressible Couette flow between the planes y - y0 = -L/2 and
    +L/2 (Section 3.2): u = 2 y' u0 / L, v = 0, constant p,
    T = (1/K) (-2 mu u0^2 y'^2 / L^2 + C1 y' + C0) with C1 = K (T_top -
    T_bottom)/L, C0 = (K (T_top + T_bottom) + mu u0^2)/2 (y' = y - y0; the
    sign of the printed C1, C0 taken so that T takes the wall values), and
    rho = gamma p / ((gamma - 1) cp T) = p / (R T).  Exact derivatives."""
    R = cp * (gamma - 1.0) / gamma
    y = mesh.xy[:, 1] - y0
    C1 = K * (T_top - T_bottom) / L
    C0 = 0.5 * (K * (T_top + T_bottom) + mu * u0 * u0)
    T = (-2.0 * mu * u0 * u0 * y * y / (L * L) + C1 * y + C0) / K
    Ty = (-4.0 * mu * u0 * u0 * y / (L * L) + C1) / K
    rho = p / (R * T)
    zero = np.zeros_like(y)
    u = 2.0 * y * u0 / L
    drho = (zero, -rho / T * Ty)
    du = (zero, np.full_like(y, 2.0 * u0 / L))
    return prim_to_state(gamma, rho, u, zero, np.full_like(y, p), drho, du, (zero, zero),
                         (zero, zero))


def circular_sod(mesh: Mesh, center=(1.0, 1.0), radius=0.5, gamma=1.4,
                 inner=(1.0, 0.0, 0.0, 1.0), outer=(0.125, 0.0, 0.0, 0.1), on_circle=None):
    """Circular Sod problem (Section 3.3): (rho, u, v, p) = ``inner`` for
    |x - c| < r, ``outer`` elsewhere, zero gradients.  ``on_circle``: ids of
    vertices placed on the circle itself, which take the outer state (the
    strict inequality) whatever their rounded distance."""
    d = mesh.xy - np.asarray(center)[None, :]
    inside = (d * d).sum(axis=1) < radius * radius
    if on_circle is not None:
        inside[np.asarray(on_circle)] = False
    S = np.where(inside[:, None], np.asarray(inner)[None, :], np.asarray(outer)[None, :])
    z = np.zeros(mesh.nv)
    return prim_to_state(gamma, S[:, 0], S[:, 1], S[:, 2], S[:, 3], (z, z), (z, z), (z, z),
                         (z, z))


def normal_shock_states(mach, gamma=1.4, rho1=1.0, p1=1.0):
    """Upstream/downstream (rho, u, v, p) of a stationary normal shock
    (Rankine-Hugoniot relations)."""
    c1 = math.sqrt(gamma * p1 / rho1)
    u1 = mach * c1
    m2 = mach * mach
    rho2 = rho1 * (gamma + 1.0) * m2 / ((gamma - 1.0) * m2 + 2.0)
    p2 = p1 * (1.0 + 2.0 * gamma / (gamma + 1.0) * (m2 - 1.0))
    u2 = u1 * rho1 / rho2
    return (rho1, u1, 0.0, p1), (rho2, u2, 0.0, p2)


def shock_vortex(mesh: Mesh, gamma=1.4, mach=1.1, x_shock=0.5,
                 center=(0.25, 0.5), beta=0.3, rc=0.05):
    """Stationary Mach ``mach`` normal shock at x = x_shock with the paper's
    isentropic vortex (strength ``beta``, coordinates scaled by ``rc``)
    superposed upstream as velocity and isentropic temperature perturbations
    of the pre-shock state (rho, p) = (1, 1)."""
    (r1, u1, _, p1), (r2, u2, _, p2) = normal_shock_states(mach, gamma)
    x = mesh.xy[:, 0]
    up = x < x_shock
    xb = (mesh.xy[:, 0] - center[0]) / rc
    yb = (mesh.xy[:, 1] - center[1]) / rc
    T, dT, du_, ddu, dv_, ddv = _vortex_prims(xb, yb, beta, gamma, rc)
    g1 = 1.0 / (gamma - 1.0)
    rho_v = T ** g1
    drho_v = tuple(g1 * rho_v / T * d for d in dT)
    p_v = rho_v ** gamma
    dp_v = tuple(gamma * rho_v ** (gamma - 1.0) * d for d in drho_v)
    z = np.zeros(mesh.nv)
    rho = np.where(up, rho_v, r2)
    p = np.where(up, p_v, p2)
    u = np.where(up, u1 + du_, u2)
    v = np.where(up, dv_, 0.0)
    drho = tuple(np.where(up, d, z) for d in drho_v)
    dp = tuple(np.where(up, d, z) for d in dp_v)
    du = tuple(np.where(up, d, z) for d in ddu)
    dv = tuple(np.where(up, d, z) for d in ddv)
    return prim_to_state(gamma, rho, u, v, p, drho, du, dv, dp)


def vertex_areas(mesh: Mesh):
    """One third of the areas of the triangles around each vertex (periodic
    displacements by the minimum image)."""
    t = mesh.tri.astype(np.int64)
    a = mesh.xy[t[:, 0]]
    d1 = mesh.xy[t[:, 1]] - a
    d2 = mesh.xy[t[:, 2]] - a
    for d in (d1, d2):
        for k in (0, 1):
            P = mesh.period[k]
            if P:
                d[:, k] -= P * np.round(d[:, k] / P)
    area = 0.5 * np.abs(d1[:, 0] * d2[:, 1] - d1[:, 1] * d2[:, 0])
    out = np.zeros(mesh.nv)
    for k in range(3):
        np.add.at(out, t[:, k], area / 3.0)
    return out


# ----------------------------------------------------------------------------
# Named workloads (mesh recipe + initial state), sizes as stated per case
# ----------------------------------------------------------------------------

def workload(name, scale=None):
    """Return (mesh, U0, params) for a named workload.

    ``scale`` overrides the lattice size n (n x n, or (2n-1) x n for the
    shock-vortex case) to build a smaller instance of the same recipe.
    """
    if name == "vortex21":
        n = scale or 21
        m = jittered_grid(n, n, 10.0, 10.0, (True, True), 0, seed=1)
        U = isentropic_vortex(m, center=(5.0, 5.0), beta=5.0)
        prm = dict(gamma=1.4, mu=0.0, switch="paper", cfl=0.3, steps=20)
    elif name == "riemann201":
        n = scale or 201
        m = jittered_grid(n, n, 1.0, 1.0, (False, False), 5, seed=2)
        U = riemann_quadrants(m)
        prm = dict(gamma=1.4, mu=0.0, switch="paper", cfl=0.3, steps=10)
    elif name == "tgv513":
        n = scale or 513
        L = 2.0 * math.pi
        m = jittered_grid(n, n, L, L, (True, True), 0, seed=3)
        U = taylor_green(m)
        prm = dict(gamma=1.4, mu=0.01, prandtl=0.72, gas_R=1.0,
                   switch="smooth", cfl=0.3, steps=500)
    elif name == "vortex257":
        n = scale or 257
        m = jittered_grid(n, n, 10.0, 10.0, (True, True), 0, seed=4)
        U = isentropic_vortex(m, center=(5.0, 5.0), beta=5.0)
        prm = dict(gamma=1.4, mu=0.0, switch="paper", cfl=0.3, steps=200)
    elif name == "shockvortex2049":
        n = scale or 1025
        m = jittered_grid(2 * n - 1, n, 2.0, 1.0, (False, False), 5, seed=5,
                          dirichlet_sides=("xlo",))
        U = shock_vortex(m)
        prm = dict(gamma=1.4, mu=0.0, switch="paper", cfl=0.3, steps=10)
    elif name == "couette":
        # x periodic on [0, 10), walls at y = 0 and 10 with Dirichlet ghost
        # regions holding the exact solution (the paper's ghost regions)
        n = scale or 141
        m = jittered_grid(n, n, 10.0, 10.0, (True, False), 5, seed=6,
                          dirichlet_sides=("ylo", "yhi"))
        U = couette(m)
        gamma, cp, K, mu = 1.4, 10.0, 0.01, 0.1
        prm = dict(gamma=gamma, mu=mu, prandtl=mu * cp / K, gas_R=cp * (gamma - 1.0) / gamma,
                   switch="smooth", cfl=0.3, steps=20)
    elif name == "sod_circle":
        # the 2 x 2 square of the paper's circular Sod problem with the circle
        # r = 0.5 embedded in the mesh, transmissive
        n = scale or 101
        m, circle = embedded_circle_grid(n, 2.0, (1.0, 1.0), 0.5, 5, seed=7)
        U = circular_sod(m, on_circle=circle)
        prm = dict(gamma=1.4, mu=0.0, switch="paper", cfl=0.3, steps=40, t_end=0.2)
    else:
        raise KeyError(name)
    return m, U, prm
