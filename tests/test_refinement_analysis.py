"""The refinement analysis of Section 2.1 (the leading error term of an
interpolation in the curve coordinate xi, and its transformation under the
two kinds of refinement, eq. err_term ... eq. scaled_dx), as a test.

A p-th order Lagrange interpolation in xi along a curved five-node stencil
(the 1D curve-coordinate approach the paper abandons) converges at order p
when the same curve is discretised with more nodes ("inserting"), but only
at first order when the stencil pattern shrinks ("shrunk", how unstructured
meshes refine): the error term carries d^p x / d xi^p, which scales like 1/N.
The 2D Hermite least-squares interpolation of Section 2.2 (the oracle's
graded pseudo-inverse) stays high order under shrinking, which is why the
paper uses it.  CPU only; the interpolation here is written out in the test.
"""
import numpy as np

from oracle import weights as ow


def curve(xi):
    """A generic smooth curve (its fifth xi-derivative is far from zero)."""
    return np.stack([xi + 0.1 * xi * xi, 0.3 * np.sin(1.3 * xi + 0.4)], axis=-1)


def u(p):
    x, y = p[..., 0], p[..., 1]
    return np.exp(0.3 * x) * np.sin(y + 0.2)


def grad_u(p):
    x, y = p[..., 0], p[..., 1]
    return np.stack([0.3 * np.exp(0.3 * x) * np.sin(y + 0.2), np.exp(0.3 * x) * np.cos(y + 0.2)],
                    axis=-1)


XI = np.array([-2.0, -1.0, 0.0, 1.0, 2.0])  # nodes i-2 .. i+2
XI_STAR = 0.5                               # the edge midpoint between i and i+1


def lagrange_weights(nodes, x):
    w = np.ones(len(nodes))
    for j in range(len(nodes)):
        for k in range(len(nodes)):
            if k != j:
                w[j] *= (x - nodes[k]) / (nodes[j] - nodes[k])
    return w


def order(Ns, errs):
    """Observed order: minus the slope of log(error) against log(N)."""
    return -np.polyfit(np.log(Ns), np.log(errs), 1)[0]


NS = np.array([8.0, 16.0, 32.0, 64.0, 128.0])


def test_xi_lagrange_inserting_refinement_is_fifth_order():
    errs = []
    for N in NS:
        nodes = XI / N                      # more nodes on the same curve
        w = lagrange_weights(nodes, XI_STAR / N)
        errs.append(abs(w @ u(curve(nodes)) - u(curve(np.array(XI_STAR / N)))))
    assert order(NS, errs) > 4.5


def test_xi_lagrange_shrunk_refinement_is_first_order():
    w = lagrange_weights(XI, XI_STAR)       # the xi spacing does not change
    errs = []
    for N in NS:
        pts = curve(XI) / N                  # the whole pattern shrinks
        errs.append(abs(w @ u(pts) - u(curve(np.array(XI_STAR)) / N)))
    s = order(NS, errs)
    assert 0.8 < s < 1.2, s


def test_hermite_least_squares_stays_high_order_when_shrunk():
    errs = []
    for N in NS[:4]:  # (at N = 128 the error nears float64 rounding)
        pts = curve(XI) / N
        mid = 0.5 * (pts[2] + pts[3])       # midpoint of the edge (i, i+1)
        h = np.linalg.norm(pts[3] - pts[2])
        frame = (pts - mid) / h
        w, rank = ow.hermite_weights(frame[None])
        w = w[0]
        g = grad_u(pts) * h                  # gradients in the edge frame
        val = w[0::3] @ u(pts) + w[1::3] @ g[:, 0] + w[2::3] @ g[:, 1]
        errs.append(abs(val - u(mid)))
    assert order(NS[:4], errs) > 3.5
