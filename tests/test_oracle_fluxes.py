"""Pins of the oracle's Riemann fluxes (Rusanov, Roe with Harten's entropy
fix, HLLC) against properties fixed by the mathematics: consistency, the
defining property of Roe's linearisation, upwinding in supersonic flow, and
exact resolution of a stationary contact/shear layer and of a stationary
shock (Rankine-Hugoniot)."""
import numpy as np
import torch

from oracle import gas
from paper_2109_01286_amd import inputs

G = 1.4


def state(rho, u, v, p):
    return torch.tensor([rho, rho * u, rho * v, p / (G - 1.0) + 0.5 * rho * (u * u + v * v)],
                        dtype=torch.float64)


def random_states(n, seed):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.2, 3.0, n)
    u, v = rng.normal(0.0, 1.0, n), rng.normal(0.0, 1.0, n)
    p = rng.uniform(0.2, 3.0, n)
    return torch.stack([state(*a) for a in zip(rho, u, v, p)])


def random_normals(n, seed):
    a = np.random.default_rng(seed).uniform(0.0, 2 * np.pi, n)
    return torch.as_tensor(np.stack([np.cos(a), np.sin(a)], axis=-1))


FLUXES = {"rusanov": gas.rusanov, "roe": gas.roe_flux, "hllc": gas.hllc_flux}


def close(a, b, tol=1e-12):
    return torch.max(torch.abs(a - b)) <= tol * max(1.0, float(torch.max(torch.abs(b))))


def test_consistency_h_of_equal_states_is_the_physical_flux():
    w = random_states(64, 1)
    n = random_normals(64, 2)
    for name, f in FLUXES.items():
        assert close(f(w, w, n, G), gas.normal_flux(w, n, G)), name


def test_roe_linearisation_property():
    """R diag(lambda) R^-1 (wR - wL) = F(wR).n - F(wL).n at the Roe average."""
    wl, wr = random_states(64, 3), random_states(64, 4)
    n = random_normals(64, 5)
    u, v, H, c = gas.roe_average(wl, wr, G)
    un = u * n[:, 0] + v * n[:, 1]
    lam = torch.stack([un - c, un, un + c, un], dim=-1)
    R = gas.roe_eigenvectors(wl, wr, n, G)
    a = torch.linalg.solve(R, (wr - wl)[..., None])[..., 0]
    jump = (R @ (lam * a)[..., None])[..., 0]
    assert close(jump, gas.normal_flux(wr, n, G) - gas.normal_flux(wl, n, G), 1e-11)


def test_supersonic_flow_is_fully_upwind():
    n = random_normals(16, 6)
    for sign in (1.0, -1.0):
        wl, wr = [], []
        rng = np.random.default_rng(7)
        for k in range(16):
            # velocity along +-n at Mach 2.5 .. 3.5 on both sides, any tangential part
            for lst in (wl, wr):
                rho, p = rng.uniform(0.5, 2.0), rng.uniform(0.5, 2.0)
                c = np.sqrt(G * p / rho)
                m, t = sign * rng.uniform(2.5, 3.5) * c, rng.normal()
                nx, ny = float(n[k, 0]), float(n[k, 1])
                lst.append(state(rho, m * nx - t * ny, m * ny + t * nx, p))
        wl, wr = torch.stack(wl), torch.stack(wr)
        up = gas.normal_flux(wl if sign > 0 else wr, n, G)
        for name in ("roe", "hllc"):
            assert close(FLUXES[name](wl, wr, n, G), up), (name, sign)


def test_stationary_contact_and_shear_are_exact():
    """u.n = 0 on both sides, equal pressure, different density and
    tangential velocity: the exact flux is (0, p n, 0)."""
    n = random_normals(16, 8)
    rng = np.random.default_rng(9)
    wl, wr, ex = [], [], []
    for k in range(16):
        nx, ny = float(n[k, 0]), float(n[k, 1])
        p = rng.uniform(0.5, 2.0)
        tl, tr = rng.normal(), rng.normal()
        wl.append(state(rng.uniform(0.3, 1.0), -tl * ny, tl * nx, p))
        wr.append(state(rng.uniform(1.5, 3.0), -tr * ny, tr * nx, p))
        ex.append(torch.tensor([0.0, p * nx, p * ny, 0.0], dtype=torch.float64))
    wl, wr, ex = torch.stack(wl), torch.stack(wr), torch.stack(ex)
    assert close(gas.hllc_flux(wl, wr, n, G), ex)
    assert close(gas.roe_flux(wl, wr, n, G), ex)
    # Rusanov diffuses the contact
    assert not close(gas.rusanov(wl, wr, n, G), ex, 1e-3)


def test_stationary_shock_is_exact():
    """Upstream Mach 2 along n, downstream from the Rankine-Hugoniot
    relations: F(wL).n = F(wR).n, and HLLC and Roe's flux without the entropy
    fix return it (the entropy fix adds dissipation to the stationary
    acoustic wave by design)."""
    (r1, u1, _, p1), (r2, u2, _, p2) = inputs.normal_shock_states(2.0)
    n = random_normals(8, 10)
    wl = torch.stack([state(r1, u1 * float(a[0]), u1 * float(a[1]), p1) for a in n])
    wr = torch.stack([state(r2, u2 * float(a[0]), u2 * float(a[1]), p2) for a in n])
    fl, fr = gas.normal_flux(wl, n, G), gas.normal_flux(wr, n, G)
    assert close(fl, fr, 1e-13)
    assert close(gas.roe_flux(wl, wr, n, G, delta=0.0), fl, 1e-11)
    assert close(gas.hllc_flux(wl, wr, n, G), fl, 1e-11)
