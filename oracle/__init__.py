"""CPU FP64 oracle of the Hermite finite-difference method (arXiv 2109.01286).

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, calls or
links anything here; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library: topology, stencils, least-squares weights and the residual are
written again here from the paper, plainly and slowly, in float64.

Modules (each function cites the passage of the paper it follows):

``mesh``     edges, adjacency, periodic minimum image, curvilinear edge
             stencils (Section 2.1, first paragraph) and double-level vertex
             stencils (Section 2.3, "Computing Divergence with Least-Square
             Method").
``basis``    Taylor-scaled monomial basis p, p_x, p_y (Section 2.2).
``weights``  graded SVD pseudo-inverse, 5-node Hermite weights with the
             singular-value dropping rule (Section 2.2), 3-node substencil
             weights (eq. 3nodes_intp), divergence rows d0, dx, dy
             (eq. flux_polynomials and the three row vectors after it),
             viscous vertex-only rows (Section 2.3, "Computing Viscous Flux").
``gas``      Euler/Navier-Stokes fluxes, Roe average, characteristic
             eigenvectors, Rusanov flux.
``scheme``   WENO switch and interpolation (eq. 2d_hweno_intp, Algorithm 1),
             residual of eq. HWENO, three-stage TVD Runge-Kutta, time step.

Readings of passages the paper leaves open are listed in the headers of the
modules that take them.
"""
