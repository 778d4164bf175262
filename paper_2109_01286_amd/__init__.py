"""Hermite finite-difference method for 2D Euler/Navier-Stokes on
unstructured triangle meshes, MI355X (gfx950) HIP implementation.

``inputs``  seeded synthetic meshes and initial states.
``hfd``     ctypes binding of the C-ABI library ``libhfd.so`` (built from
            ``csrc/``); every step of the solver runs in its HIP kernels.
"""
