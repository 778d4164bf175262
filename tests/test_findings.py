"""Findings about the method as read, reproduced on the oracle (CPU).  They
are properties of the scheme under the readings, not of the GPU path (which
reproduces the oracle); each test states one so that it can be checked:

1. the smooth (5-node Hermite) path is linearly unstable: the residual
   linearised about a uniform flow has an eigenvalue with a positive real
   part of order 1/h, whose eigenvector lies mostly in the gradient unknowns;
2. planar 3-node interpolation on path substencils is ill-conditioned
   (weights of order 10^4 on a jittered lattice), which the w3_cap option
   bounds;
3. the switch on omega_1 alone keeps the Hermite value when the jump lies in
   the third substencil (omega_1 = 1/11), while it catches jumps in the first
   two."""
import numpy as np
import pytest
import torch

from oracle import mesh as omesh
from oracle import scheme as osch
from oracle import weights as ow
from paper_2109_01286_amd import inputs


def test_smooth_path_has_a_growing_gradient_mode():
    n = 11
    m = inputs.jittered_grid(n, n, 10.0, 10.0, (True, True), 0, seed=1)
    sc = osch.Scheme(m.xy, m.tri, m.ghost_src, m.period, osch.Options(switch="smooth"))
    V = m.nv
    U0 = np.zeros((12, V))
    U0[0], U0[1], U0[2], U0[3] = 1.0, 1.0, 1.0, 1.0 / 0.4 + 1.0
    J = torch.autograd.functional.jacobian(
        lambda x: sc.residual(x.reshape(12, V), "smooth").reshape(-1),
        torch.as_tensor(U0).reshape(-1), vectorize=True).numpy()
    ev, vec = np.linalg.eig(J)
    k = int(np.argmax(ev.real))
    h = 10.0 / (n - 1)
    v = vec[:, k].reshape(12, V)
    blocks = np.array([np.linalg.norm(v[4 * b:4 * b + 4]) for b in range(3)])
    print(f"[findings] max Re(lambda) h = {ev.real[k] * h:.3f}, "
          f"eigenvector blocks (w, w_x, w_y) {np.round(blocks / blocks.max(), 3)}")
    assert ev.real[k] * h > 0.5
    assert blocks[0] < 0.7 * max(blocks[1], blocks[2])


def test_planar_three_node_weights_are_ill_conditioned_and_capped():
    m = inputs.jittered_grid(21, 21, 10.0, 10.0, (True, True), 0, seed=1)
    topo = omesh.build(m.xy, m.tri, m.ghost_src, m.period)
    free = np.abs(ow.edge_weights(topo, m.xy, m.period, w3_cap=0.0).w3).max()
    capped = np.abs(ow.edge_weights(topo, m.xy, m.period, w3_cap=2.0).w3).max()
    print(f"[findings] largest 3-node weight: {free:.3g} without the cap, {capped:.3g} with 2")
    assert free > 1e3
    assert capped <= 2.0


@pytest.mark.parametrize("jump_after,weno", [(0, True), (1, True), (2, True), (3, False)])
def test_omega1_switch_misses_a_jump_in_the_third_substencil(jump_after, weno):
    """Five projected values with a unit jump after position `jump_after`.
    Substencils (c0 c1 c2), (c1 c2 c3), (c2 c3 c4): a jump after c3 lies in
    the third only, the other two are flat, and omega_1 = d1/(d1 + d2) =
    1/11 falls inside the Hermite interval (0.01, 0.79)."""
    c = torch.zeros(5, dtype=torch.float64)
    c[jump_after + 1:] = 1.0
    om = osch.weno_omega(c, 1e-6)
    o1 = float(om[0])
    takes_weno = not (0.01 < o1 < 0.79)
    print(f"[findings] jump after c{jump_after}: omega_1 = {o1:.4f}")
    assert takes_weno == weno
    if jump_after == 3:
        assert abs(o1 - 1.0 / 11.0) < 1e-9
