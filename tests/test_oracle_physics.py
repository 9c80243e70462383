"""Pins for the oracle's physical and numerical fluxes (Sections 2.2, 3 and 5.2)."""
import math

import numpy as np
import pytest
import torch

from oracle.physics import Physics, EQ_EULER, EQ_NS, EQ_POISSON

DT = torch.float64


def cons(rho, vel, p, gamma=1.4):
    vel = torch.as_tensor(vel, dtype=DT)
    E = p / (gamma - 1) + 0.5 * rho * float((vel * vel).sum())
    return torch.cat([torch.tensor([rho], dtype=DT), rho * vel, torch.tensor([E], dtype=DT)])


def random_states(dim, n, seed, mach=0.5):
    g = torch.Generator().manual_seed(seed)
    rho = 0.5 + torch.rand(n, generator=g, dtype=DT)
    vel = (torch.rand(n, dim, generator=g, dtype=DT) - 0.5) * 2 * mach
    p = 0.5 + torch.rand(n, generator=g, dtype=DT)
    E = p / 0.4 + 0.5 * rho * (vel * vel).sum(-1)
    return torch.cat([rho[:, None], rho[:, None] * vel, E[:, None]], dim=-1)


@pytest.mark.parametrize("dim", [2, 3])
def test_euler_flux_closed_form(dim):
    ph = Physics(EQ_EULER, dim)
    vel = [0.3, -0.2, 0.1][:dim]
    u = cons(1.2, vel, 0.9)
    F = ph.flux_inv(u)
    for d in range(dim):
        assert abs(F[0, d] - 1.2 * vel[d]) < 1e-15
        for i in range(dim):
            ref = 1.2 * vel[i] * vel[d] + (0.9 if i == d else 0.0)
            assert abs(F[1 + i, d] - ref) < 1e-15
        H = (float(u[-1]) + 0.9) / 1.2
        assert abs(F[-1, d] - 1.2 * vel[d] * H) < 1e-14


@pytest.mark.parametrize("dim", [2, 3])
def test_roe_flux_pins(dim):
    ph = Physics(EQ_EULER, dim)
    uL = random_states(dim, 64, 1)
    uR = random_states(dim, 64, 2)
    g = torch.Generator().manual_seed(3)
    n = torch.randn(64, dim, generator=g, dtype=DT)
    nn = torch.linalg.norm(n, dim=-1, keepdim=True)
    nbar = n / nn
    # Roe property: A_roe (uR - uL) = (F(uR) - F(uL)) . nbar
    absA, A = ph.roe_abs_matrix(uR, uL, nbar)
    lhs = (A @ (uR - uL)[..., None])[..., 0]
    rhs = ph.flux_inv_n(uR, nbar) - ph.flux_inv_n(uL, nbar)
    assert torch.allclose(lhs, rhs, atol=1e-12, rtol=1e-12)
    # |A|^2 = A^2 and |A| commutes with A
    assert torch.allclose(absA @ absA, A @ A, atol=1e-10)
    assert torch.allclose(absA @ A, A @ absA, atol=1e-10)
    # consistency: Fhat(u, u; n) = F(u) . n
    assert torch.allclose(ph.roe_flux(uL, uL, n), ph.flux_inv_n(uL, n), atol=1e-13)
    # scaling with |n| and antisymmetry Fhat(uR,uL;n) = -Fhat(uL,uR;-n)
    assert torch.allclose(ph.roe_flux(uR, uL, 3.0 * n), 3.0 * ph.roe_flux(uR, uL, n), atol=1e-12)
    assert torch.allclose(ph.roe_flux(uR, uL, n), -ph.roe_flux(uL, uR, -n), atol=1e-12)


def test_roe_supersonic_upwinding():
    ph = Physics(EQ_EULER, 2)
    uL = cons(1.0, [3.0, 0.1], 1.0)  # Mach ~ 2.5 towards +x
    uR = cons(0.9, [2.8, -0.1], 0.8)
    n = torch.tensor([2.0, 0.0], dtype=DT)
    assert torch.allclose(ph.roe_flux(uR[None], uL[None], n[None])[0], ph.flux_inv_n(uL, n), atol=1e-12)
    n2 = -n
    assert torch.allclose(ph.roe_flux(uL[None], uR[None], n2[None])[0], ph.flux_inv_n(uL, n2), atol=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_viscous_flux_couette(dim):
    """Simple shear u_0 = a x_1 at constant rho, p: tau_01 = mu a, heat flux 0."""
    mu, a = 0.3, 2.0
    ph = Physics(EQ_NS, dim, mu=mu, prandtl=0.72)
    x1 = 0.4
    vel = torch.zeros(dim, dtype=DT)
    vel[0] = a * x1
    u = cons(1.1, vel, 1.3)
    q = torch.zeros(dim + 2, dim, dtype=DT)
    # conserved gradients at constant rho, p: d(rho u0)/dx1 = rho a, d(rho E)/dx1 = rho u0 a
    q[1, 1] = 1.1 * a
    q[-1, 1] = 1.1 * vel[0] * a
    Fv = ph.flux_vis(u, q)
    ref = torch.zeros(dim + 2, dim, dtype=DT)
    ref[1, 1] = -mu * a
    ref[2, 0] = -mu * a
    ref[-1, 1] = -vel[0] * mu * a
    assert torch.allclose(Fv, ref, atol=1e-14)


@pytest.mark.parametrize("dim", [2, 3])
def test_viscous_flux_heat_conduction(dim):
    """Fluid at rest with a temperature gradient: only the heat flux -(mu/Pr) dh/dx."""
    mu, pr, g = 0.2, 0.72, 1.4
    ph = Physics(EQ_NS, dim, mu=mu, prandtl=pr)
    rho, p = 1.3, 1.0
    u = cons(rho, torch.zeros(dim), p)
    # at fixed p, a density gradient drho/dx0 = s changes h = gamma p/((gamma-1) rho)
    s = 0.25
    q = torch.zeros(dim + 2, dim, dtype=DT)
    q[0, 0] = s
    Fv = ph.flux_vis(u, q)
    dh = -g * p / ((g - 1) * rho ** 2) * s
    ref = torch.zeros(dim + 2, dim, dtype=DT)
    ref[-1, 0] = -(mu / pr) * dh
    assert torch.allclose(Fv, ref, atol=1e-14)


def test_viscous_flux_dilatation():
    """Pure expansion u = a x in 2-D: tau_00 = mu (2a - 2a/3), tau_11 = -2 mu a/3."""
    mu, a = 0.5, 1.5
    ph = Physics(EQ_NS, 2, mu=mu)
    u = cons(1.0, [0.0, 0.0], 1.0)  # at x = 0
    q = torch.zeros(4, 2, dtype=DT)
    q[1, 0] = a  # d(rho u)/dx at rho = 1, u = 0
    Fv = ph.flux_vis(u, q)
    assert abs(Fv[1, 0] + mu * (2 * a - 2 * a / 3)) < 1e-14
    assert abs(Fv[2, 1] + mu * (-2 * a / 3)) < 1e-14
    assert abs(Fv[1, 1]) < 1e-15 and abs(Fv[2, 0]) < 1e-15


def test_poisson_flux():
    ph = Physics(EQ_POISSON, 2)
    q = torch.randn(5, 1, 2, dtype=DT)
    assert torch.equal(ph.flux_vis(torch.zeros(5, 1, dtype=DT), q), -q)
    assert ph.m == 1 and not ph.has_inviscid and ph.has_viscous
