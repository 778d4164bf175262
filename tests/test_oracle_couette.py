"""Viscous pin of the oracle (Section 3.2): the steady compressible Couette
flow is an exact solution of the Navier-Stokes equations, so the discrete
residual at that state is the scheme's truncation error and must vanish
under refinement at high order (the paper reports fourth-order convergence
of the density error).  Dirichlet ghost regions hold the exact solution, as
in the paper.  A dropped viscous term, a wrong sign in the heat flux or in
the work of the stresses, or an inconsistent exact state would leave an O(1)
residual."""
import numpy as np

from oracle import scheme as osch
from paper_2109_01286_amd import inputs


def residual_max(n):
    m, U, prm = inputs.workload("couette", n)
    o = osch.Options(gamma=prm["gamma"], mu=prm["mu"], prandtl=prm["prandtl"],
                     gas_R=prm["gas_R"])
    sc = osch.Scheme(m.xy, m.tri, m.ghost_src, m.period, o)
    R = np.asarray(sc.residual(U, "smooth"))
    own = m.ghost_src == -1
    return np.abs(R[:, own]).max(axis=1), m.h[1]


def test_exact_couette_residual_converges_at_high_order():
    (r1, h1), (r2, h2) = residual_max(31), residual_max(61)
    order = np.log(r1 / r2) / np.log(h1 / h2)
    print("Couette residual orders (values, d/dx, d/dy rows):", np.round(order, 2))
    # rho, rho u, E rows of the values and of both gradients (rho v is ~0)
    for q in (0, 1, 3):
        assert order[q] > 4.0, order
        assert order[4 + q] > 3.5 and order[8 + q] > 3.5, order
    assert np.all(np.isfinite(r2)) and r2[[0, 1, 3]].max() < 1e-2
