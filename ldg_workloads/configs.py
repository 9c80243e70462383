"""The five synthetic workloads, with their sizes and physical parameters.

C1  2-D Poisson, 8x8 uniform quads on [0,1]^2, p=3, Dirichlet, u = sin(pi x) sin(pi y).
C2  2-D Euler isentropic vortex (strength 5, centre (5,5)), 32x32 quads on [0,10]^2 with
    interior vertices perturbed by up to 20% of h (seed 0), p=4, periodic, RK4 dt=2e-3.
C3  3-D Navier-Stokes Taylor-Green, M=0.2, Re=400, Pr=0.72, 16^3 hexes of [0,2pi]^3 curved by
    x + 0.1 sin x sin y sin z, p=3, periodic, one BDF2 Newton step with dt=0.05.
C4  As C3 on 32^3 hexes at p=4, Re=1600, dt=0.02.
C5  24^3 hexes, p=3, Navier-Stokes with seeded Re in [200,2000], M in [0.1,0.4] and a low-mode
    perturbation of the Taylor-Green field (learned-preconditioner data).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import fields
from .mesh import Mesh, hex_mesh, quad_mesh

EQ_POISSON, EQ_EULER, EQ_NS = 0, 1, 2


@dataclasses.dataclass
class Problem:
    name: str
    mesh: Mesh
    equation: int
    m: int
    U0: np.ndarray
    gamma: float = 1.4
    mu: float = 0.0
    prandtl: float = 0.72
    c11_interior: float = 0.0
    c11_dirichlet: float = 10.0
    source: np.ndarray | None = None
    gD: np.ndarray | None = None
    gN: np.ndarray | None = None
    dt: float = 0.0
    extra: dict = dataclasses.field(default_factory=dict)

    @property
    def n_dof(self) -> int:
        return self.mesh.n_elem * self.m * self.mesh.np_


def poisson(n: int = 8, p: int = 3, kind: str = "sine", c11_dirichlet: float = 10.0) -> Problem:
    mesh = quad_mesh(n, n, p, box=((0.0, 1.0), (0.0, 1.0)), periodic=(False, False),
                     name=f"poisson{n}x{n}p{p}")
    if kind == "sine":
        u, f, g = fields.poisson_sine(mesh)
    else:
        u, f, g = fields.poisson_polynomial(mesh, degs=(min(p, 3), min(p, 2)))
    gD = fields.face_values(mesh, u)
    return Problem(mesh.name, mesh, EQ_POISSON, 1, np.zeros_like(u), c11_dirichlet=c11_dirichlet,
                   source=np.ascontiguousarray(f), gD=gD,
                   extra=dict(u_exact=u, grad_exact=g))


def config1() -> Problem:
    return poisson(8, 3)


def euler_vortex(n: int = 32, p: int = 4, perturb: float = 0.2, seed: int = 0) -> Problem:
    L = 10.0
    mesh = quad_mesh(n, n, p, box=((0.0, L), (0.0, L)), periodic=(True, True), perturb=perturb,
                     seed=seed, name=f"vortex{n}x{n}p{p}")
    U0 = fields.vortex(mesh, 0.0, beta=5.0, center=(5.0, 5.0), period=(L, L))
    return Problem(mesh.name, mesh, EQ_EULER, 4, U0, gamma=1.4, dt=2e-3,
                   extra=dict(n_steps=100, period=(L, L)))


def config2() -> Problem:
    return euler_vortex(32, 4)


def euler_vortex_tiled(n: int = 512, p: int = 4, perturb: float = 0.2, seed: int = 0) -> Problem:
    """The vortex workload scaled up for a bandwidth measurement: n x n perturbed quads of the same
    size as the 32 x 32 one (h = 10/32) on [0, 10 n / 32]^2, with the vortex repeated in every
    10 x 10 tile (periodic), p = 4: 26.2 M unknowns at n = 512."""
    L = 10.0 * n / 32
    mesh = quad_mesh(n, n, p, box=((0.0, L), (0.0, L)), periodic=(True, True), perturb=perturb, seed=seed,
                     name=f"vortex-tiled{n}x{n}p{p}")
    U0 = fields.vortex(mesh, 0.0, beta=5.0, center=(5.0, 5.0), period=(10.0, 10.0))
    return Problem(mesh.name, mesh, EQ_EULER, 4, U0, gamma=1.4, dt=2e-3, extra=dict(period=(L, L)))


def taylor_green(n: int, p: int, re: float, mach: float = 0.2, dt: float = 0.05,
                 perturb_amp: float = 0.0, seed: int | None = None) -> Problem:
    mesh = hex_mesh(n, p, name=f"tgv{n}^3p{p}")
    U0 = fields.taylor_green(mesh, mach=mach, perturb_amp=perturb_amp, seed=seed)
    return Problem(mesh.name, mesh, EQ_NS, 5, U0, gamma=1.4, mu=1.0 / re, prandtl=0.72, dt=dt,
                   extra=dict(re=re, mach=mach))


def config3() -> Problem:
    return taylor_green(16, 3, 400.0, dt=0.05)


def config4() -> Problem:
    return taylor_green(32, 4, 1600.0, dt=0.02)


def config5_sample(seed: int, n: int = 24, p: int = 3) -> Problem:
    """One learned-preconditioner run: seeded Re ~ U[200,2000], M ~ U[0.1,0.4]."""
    rng = np.random.default_rng(seed)
    re = float(rng.uniform(200.0, 2000.0))
    mach = float(rng.uniform(0.1, 0.4))
    pr = taylor_green(n, p, re, mach=mach, dt=0.05, perturb_amp=0.05, seed=seed + 7919)
    pr.extra.update(seed=seed)
    return pr


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4}
