"""Pins of the oracle's literal reading of Section 2.2 (``hermite="physical"``):
the plain pseudo-inverse rows of the 15 x 15 Hermite system and of the 3 x 6
system of eq. 3nodes_intp, in physical units with the origin at the edge
midpoint.

The minimum-norm solution of a consistent system is the exact coefficient
vector minus its component in the null space.  So for a polynomial of the
fit's degree, the midpoint value and derivatives that the rows give differ
from the exact ones by that null component, evaluated at the midpoint.  The
null spaces here are built from the geometry alone, not from the oracle's
matrices:

* 5 nodes with values and gradients (rank 14): the square of the conic
  through the five nodes, whose value and gradient vanish at every node;
* 3 non-collinear nodes with values (rank 3): the three products of two of
  the lines through pairs of nodes, each vanishing at all three nodes.

A dropped term of the basis, a transposed row, a row taken from the wrong
factor or another choice among the solutions changes the error away from
this multiple of the null component and fails the check.
"""
import math

import numpy as np
import numpy.polynomial.polynomial as npp

from oracle import basis, weights as ow

from .test_oracle_pins import _random_stencils


def _taylor(m, deg):
    """Taylor coefficients (the basis order of Section 2.2) of the 2D
    monomial coefficient array ``m``."""
    return np.array([math.factorial(a) * math.factorial(b) * m[a, b]
                     for a, b in basis.exponents(deg)])


def _poly_mul(c1, c2):
    out = np.zeros((c1.shape[0] + c2.shape[0] - 1, c1.shape[1] + c2.shape[1] - 1))
    for (a1, b1), v1 in np.ndenumerate(c1):
        for (a2, b2), v2 in np.ndenumerate(c2):
            out[a1 + a2, b1 + b2] += v1 * v2
    return out


def _conic_square(x, y):
    """Monomial coefficients (5 x 5) of the square of the conic through the
    five points (null vector of the 5 x 6 conic matrix)."""
    Q = np.stack([np.ones(5), x, y, x * x, x * y, y * y], 1)
    q = np.linalg.svd(Q)[2][-1]
    c = np.zeros((3, 3))
    c[0, 0], c[1, 0], c[0, 1], c[2, 0], c[1, 1], c[0, 2] = q
    return _poly_mul(c, c)


def test_physical_hermite_rows_miss_by_the_conic_square_component():
    """On stencils where the literal reading keeps rank 14 (no singular
    value dropped), the value row and both derivative rows applied to the
    data of a random quartic give its exact midpoint value and gradient
    minus n_j (n . c) / |n|^2, with c its Taylor coefficients and n those of
    the conic's square (n_0 = C(0)^2, n_1 and n_2 its midpoint gradient).
    Physical units: the stencils are scaled by h = 0.5 and h = 1."""
    rng = np.random.default_rng(23)
    checked = 0
    for h in (0.5, 1.0):
        S = h * _random_stencils(rng, 80, sd_ang=math.pi / 8)
        w, r, g = ow.hermite_weights_physical(S, grad=True)
        for j in np.nonzero(r == 14)[0]:
            x, y = S[j, :, 0], S[j, :, 1]
            n = _taylor(_conic_square(x, y), 4)
            m = np.zeros((5, 5))
            for a, b in basis.exponents(4):
                m[a, b] = rng.standard_normal()
            c = _taylor(m, 4)
            data = np.stack([npp.polyval2d(x, y, m),
                             npp.polyval2d(x, y, npp.polyder(m, axis=0)),
                             npp.polyval2d(x, y, npp.polyder(m, axis=1))], 1).ravel()
            t = (n @ c) / (n @ n)
            got = np.array([w[j] @ data, g[j, 0] @ data, g[j, 1] @ data])
            want = c[:3] - n[:3] * t
            scale = 1.0 + np.abs(c).sum()
            assert np.abs(got - want).max() <= 1e-8 * scale, (h, j, got, want)
            checked += 1
    assert checked >= 80
    # the null component is not zero in general: the literal rows do not
    # reproduce cubics either (the conic square has lower-degree terms)
    assert abs(n[0] * t) > 1e-6


def test_physical_hermite_dropping_rule_leaves_every_entry_below_one():
    """The literal dropping rule tests all 15 entries of the stored row:
    after it, every entry is below one in magnitude unless the rank reached
    one; on the stencils of Section 2.2's protocol scaled by 0.05 the
    derivative weights carry the length scale and the rule fires."""
    rng = np.random.default_rng(29)
    for h in (0.05, 1.0):
        S = h * _random_stencils(rng, 200, sd_ang=math.pi / 6)
        w, r = ow.hermite_weights_physical(S)
        ok = (np.abs(w).max(axis=1) < 1.0) | (r == 1)
        assert ok.all(), (h, np.nonzero(~ok)[0][:5])
        assert (r <= 14).all()


def _line(p, q):
    """Monomial coefficients (2 x 2, degree 1) of the line through p and q."""
    a, b = q[1] - p[1], p[0] - q[0]
    c = np.zeros((2, 2))
    c[0, 0], c[1, 0], c[0, 1] = -(a * p[0] + b * p[1]), a, b
    return c


def test_physical_three_node_rows_are_the_minimum_norm_fit():
    """For three non-collinear nodes the 3 x 6 system of eq. 3nodes_intp has
    a three-dimensional null space, the quadratics vanishing at the nodes:
    L12 L13, L12 L23 and L13 L23 (Lij the line through nodes i and j).  The
    plain pseudo-inverse picks the coefficient vector orthogonal to it, so
    on any quadratic the value row and the derivative rows give the exact
    midpoint value and gradient minus those of the projection of its Taylor
    coefficients onto that null space.  Physical units, nodes at distances
    0.3 to 2 from the midpoint."""
    rng = np.random.default_rng(31)
    P = rng.uniform(-1.5, 1.5, size=(60, 3, 2))
    area = 0.5 * np.abs((P[:, 1, 0] - P[:, 0, 0]) * (P[:, 2, 1] - P[:, 0, 1])
                        - (P[:, 2, 0] - P[:, 0, 0]) * (P[:, 1, 1] - P[:, 0, 1]))
    P = P[area > 0.2]
    w, g = ow.three_node_weights_physical(P, grad=True)
    for j in range(P.shape[0]):
        a, b, c3 = P[j]
        l12, l13, l23 = _line(a, b), _line(a, c3), _line(b, c3)
        Z = np.stack([_taylor(_poly_mul(l12, l13), 2), _taylor(_poly_mul(l12, l23), 2),
                      _taylor(_poly_mul(l13, l23), 2)], 1)          # [6, 3]
        Qz = np.linalg.qr(Z)[0]
        m = np.zeros((3, 3))
        for e1, e2 in basis.exponents(2):
            m[e1, e2] = rng.standard_normal()
        c = _taylor(m, 2)
        data = npp.polyval2d(P[j, :, 0], P[j, :, 1], m)
        want = (c - Qz @ (Qz.T @ c))[:3]
        got = np.array([w[j] @ data, g[j, 0] @ data, g[j, 1] @ data])
        assert np.abs(got - want).max() <= 1e-11 * (1.0 + np.abs(c).sum()), (j, got, want)
    assert P.shape[0] >= 30
    # linear data are not reproduced exactly: the literal rows miss even
    # constants (the null space is not orthogonal to the constant term)
    one = w.sum(axis=1)
    assert np.abs(one - 1.0).max() > 1e-3
