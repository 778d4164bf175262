"""Oracle polynomial basis (test infrastructure only).

Section 2.2 defines the degree-4 basis p(x, y) = [1, x, y, x^2/2, xy, y^2/2,
x^3/6, ...] and its exact derivatives p_x, p_y.  Its pattern: monomials in
order of total degree, within a degree by decreasing power of x, each term
x^a y^b divided by a! b!, so that the coefficients are the Taylor
derivatives at the origin.  The same pattern gives the degree-2 basis p_3
of eq. 3nodes_intp and the degree-5 basis used for the divergence.
"""
from __future__ import annotations

import math

import numpy as np


def exponents(deg):
    return [(d - j, j) for d in range(deg + 1) for j in range(d + 1)]


def nterms(deg):
    return (deg + 1) * (deg + 2) // 2


def _mono(x, y, a, b):
    if a < 0 or b < 0:
        return np.zeros_like(x)
    return x ** a * y ** b / (math.factorial(a) * math.factorial(b))


def p(x, y, deg):
    """Basis values, shape [..., nterms(deg)]."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    return np.stack([_mono(x, y, a, b) for a, b in exponents(deg)], axis=-1)


def px(x, y, deg):
    """d/dx of every basis term: x^(a-1) y^b / ((a-1)! b!)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    return np.stack([_mono(x, y, a - 1, b) for a, b in exponents(deg)], axis=-1)


def py(x, y, deg):
    """d/dy of every basis term: x^a y^(b-1) / (a! (b-1)!)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    return np.stack([_mono(x, y, a, b - 1) for a, b in exponents(deg)], axis=-1)


def degree_block(deg):
    """Indices of the terms of exactly total degree ``deg``."""
    return list(range(nterms(deg - 1), nterms(deg)))
