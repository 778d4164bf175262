"""Pins of the oracle's midpoint derivatives (the second and third rows of
the 5-node Hermite operator of Section 2.2, eq. hintp_5, and the gradient of
the 3-node interpolants of eq. 3nodes_intp), against exact derivatives of
polynomials computed by numpy.polynomial -- not by the oracle's basis."""
import math

import numpy as np
import numpy.polynomial.polynomial as npp
import pytest
import torch

from oracle import basis, weights as ow
from paper_2109_01286_amd import inputs
from tests.test_oracle_pins import _random_stencils
from tests._helpers import oracle_scheme


def _rand_poly(rng, deg):
    m = np.zeros((deg + 1, deg + 1))
    for a in range(deg + 1):
        for b in range(deg + 1 - a):
            m[a, b] = rng.standard_normal()
    return m


def _hermite_data(m, x, y):
    return np.stack([npp.polyval2d(x, y, m), npp.polyval2d(x, y, npp.polyder(m, axis=0)),
                     npp.polyval2d(x, y, npp.polyder(m, axis=1))], 1).ravel()


@pytest.mark.parametrize("deg", [1, 2, 3])
def test_hermite_gradient_rows_reproduce_cubics(deg):
    """The derivative rows give the exact gradient at the midpoint of any
    polynomial of degree <= 3 whenever at most five directions are dropped
    (the graded operator then recovers all cubic coefficients), and zero for
    a constant (the fold)."""
    rng = np.random.default_rng(20 + deg)
    S = _random_stencils(rng, 200, sd_ang=math.pi / 6)
    w, r, g = ow.hermite_weights(S, grad=True)
    assert ((r < 14) & (r >= 10)).any()
    for j in np.nonzero(r >= 10)[0]:
        m = _rand_poly(rng, deg)
        x, y = S[j, :, 0], S[j, :, 1]
        d = _hermite_data(m, x, y)
        want = np.array([m[1, 0], m[0, 1]])       # gradient at the origin
        assert np.abs(g[j] @ d - want).max() <= 1e-10 * (1 + np.abs(m).sum()), (j, r[j])
    const = np.tile([1.0, 0.0, 0.0], 5)
    assert np.abs(g @ const).max() <= 1e-12


def test_three_node_gradient_rows():
    """Non-collinear nodes: the gradient of the planar interpolant, exact for
    linear fields.  Collinear uniform nodes along x: the derivative of the 1D
    quadratic through them at the midpoint (Lagrange basis derivatives), and
    zero across the line (the graded solution has no y term)."""
    rng = np.random.default_rng(31)
    for _ in range(50):
        pts = rng.uniform(-2, 2, size=(1, 3, 2))
        a, bx, by = rng.standard_normal(3)
        f = a + bx * pts[0, :, 0] + by * pts[0, :, 1]
        _, g = ow.three_node_weights(pts, anchor=2, grad=True)
        assert np.allclose(g[0] @ f, [bx, by], rtol=1e-9, atol=1e-9)
    xs = np.array([-2.5, -1.5, -0.5])
    pts = np.stack([xs, np.zeros(3)], 1)[None]
    _, g = ow.three_node_weights(pts, anchor=2, grad=True)
    # derivative at 0 of the Lagrange basis polynomials through xs
    dl = []
    for k in range(3):
        others = [xs[m] for m in range(3) if m != k]
        coef = npp.polyfromroots(others) / np.prod([xs[k] - o for o in others])
        dl.append(npp.polyval(0.0, npp.polyder(coef)))
    assert np.allclose(g[0, 0], dl, atol=1e-13)
    assert np.allclose(g[0, 1], 0.0, atol=1e-13)


def _poly_state(rng, m, deg):
    """Each conservative component a random polynomial of degree ``deg`` in
    (x, y) (period-free: used away from any wrap), exact gradients."""
    polys = [_rand_poly(rng, deg) * 0.05 for _ in range(4)]
    polys[0][0, 0] += 1.0                      # rho ~ 1
    polys[3][0, 0] += 3.0                      # E ~ 3
    x, y = m.xy[:, 0], m.xy[:, 1]
    U = np.zeros((12, m.nv))
    for q, pq in enumerate(polys):
        U[q] = npp.polyval2d(x, y, pq)
        U[4 + q] = npp.polyval2d(x, y, npp.polyder(pq, axis=0))
        U[8 + q] = npp.polyval2d(x, y, npp.polyder(pq, axis=1))
    return U, polys


@pytest.mark.parametrize("switch,deg", [("smooth", 3), ("weno", 1), ("mask", 1)])
def test_edge_midpoint_gradients_of_polynomial_states(switch, deg):
    """On a jittered non-periodic lattice with polynomial conservative fields
    and exact gradients, both sides' midpoint derivatives equal the exact
    gradient at the edge midpoint: cubics on the 5-node branch, linear fields
    on the 3-node branch and on a random per-component mix of the two (which
    exercises the characteristic projection and the back-projection)."""
    rng = np.random.default_rng(40)
    m = inputs.jittered_grid(15, 15, 1.4, 1.4, (False, False), 5, seed=8)
    m.ghost_src = np.where(m.ghost_src >= 0, -2, m.ghost_src)   # ghosts keep the field
    U, polys = _poly_state(rng, m, deg)
    sc = oracle_scheme(m)
    sw = switch
    if switch == "mask":
        sw = rng.integers(0, 256, size=sc.st.shape[0]).astype(np.uint8)
    wl, wr, mask, h, gl, gr = sc.edge_states(torch.as_tensor(U), sw, grad=True)
    st = sc.topo.stencil[sc.ew.edges]
    mid = 0.5 * (m.xy[st[:, 2]] + m.xy[st[:, 3]])
    want = np.stack([np.stack([npp.polyval2d(mid[:, 0], mid[:, 1], npp.polyder(pq, axis=a))
                               for pq in polys], 1) for a in (0, 1)], 1)   # [E, 2, 4]
    keep = np.ones(st.shape[0], dtype=bool)
    if switch != "smooth":
        # three collinear nodes (the boundary lines are not jittered) fix no
        # derivative across their line: leave out edges with such a substencil
        P = m.xy[st]                                     # [E, 6, 2]
        for j in range(4):
            a, b, c = P[:, j], P[:, j + 1], P[:, j + 2]
            cross = np.abs((b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1])
                           - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0]))
            keep &= cross > 1e-3 * np.sum((c - a) ** 2, axis=1)
        assert keep.mean() > 0.3
    scale = np.abs(want).max()
    err = max(np.abs(gl.numpy() - want)[keep].max(), np.abs(gr.numpy() - want)[keep].max())
    assert err <= 1e-8 * scale, err
