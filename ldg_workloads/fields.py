"""Analytic initial data, boundary data and sources, sampled at mesh nodes.

Inputs only: every function evaluates a closed-form field at the node
coordinates of a :class:`ldg_workloads.mesh.Mesh` and returns arrays in the
``[E, m, Np]`` (volume) or ``[E, 2D, m, Nf]`` (face) layouts.
"""
from __future__ import annotations

import math

import numpy as np

from .mesh import Mesh, line_end_node


def face_node_table(mesh: Mesh) -> np.ndarray:
    """``tab[f, l]`` = local node index of face node ``l`` on face ``f``."""
    d, p = mesh.dim, mesh.p
    return np.array([[line_end_node(d, p, f // 2, l, p if f % 2 else 0) for l in range(mesh.nf)]
                     for f in range(2 * d)], dtype=np.int64)


def face_values(mesh: Mesh, vol: np.ndarray) -> np.ndarray:
    """Restrict a nodal field ``[E, m, Np]`` to face nodes ``[E, 2D, m, Nf]``."""
    tab = face_node_table(mesh)
    return np.ascontiguousarray(np.transpose(vol[:, :, tab], (0, 2, 1, 3)))


def axis_normal_face_values(mesh: Mesh, grad: np.ndarray) -> np.ndarray:
    """grad . nhat at face nodes [E, 2D, m, Nf] for axis-aligned faces: face 2n+s has outward unit
    normal (2s - 1) e_n (rectangular elements).  grad is [E, m, D, Np]."""
    tab = face_node_table(mesh)
    E, m, D = grad.shape[0], grad.shape[1], mesh.dim
    out = np.empty((E, 2 * D, m, tab.shape[1]))
    for f in range(2 * D):
        n, s = divmod(f, 2)
        out[:, f] = (2 * s - 1) * grad[:, :, n, tab[f]]
    return out


# ---------------------------------------------------------------- Poisson
def poisson_sine(mesh: Mesh):
    """u = sin(pi x) sin(pi y), f = 2 pi^2 u (so that -Lap u = f)."""
    x, y = mesh.xyz[:, 0], mesh.xyz[:, 1]
    u = np.sin(math.pi * x) * np.sin(math.pi * y)
    grad = np.stack([math.pi * np.cos(math.pi * x) * np.sin(math.pi * y),
                     math.pi * np.sin(math.pi * x) * np.cos(math.pi * y)], axis=1)
    return u[:, None, :], 2 * math.pi ** 2 * u[:, None, :], grad[:, None, :, :]


def poisson_polynomial(mesh: Mesh, degs=(3, 2)):
    """u = x^a y^b (a, b <= p is inside Q_p), f = -Lap u, and grad u."""
    a, b = degs
    x, y = mesh.xyz[:, 0], mesh.xyz[:, 1]
    u = x ** a * y ** b
    ux = a * x ** max(a - 1, 0) * y ** b if a > 0 else 0 * x
    uy = b * x ** a * y ** max(b - 1, 0) if b > 0 else 0 * y
    uxx = a * (a - 1) * x ** max(a - 2, 0) * y ** b if a > 1 else 0 * x
    uyy = b * (b - 1) * x ** a * y ** max(b - 2, 0) if b > 1 else 0 * y
    f = -(uxx + uyy)
    grad = np.stack([ux, uy], axis=1)
    return u[:, None, :], f[:, None, :], grad[:, None, :, :]


def poisson_polynomial_3d(mesh: Mesh, degs=(2, 1, 2)):
    a, b, c = degs
    x, y, z = mesh.xyz[:, 0], mesh.xyz[:, 1], mesh.xyz[:, 2]

    def mono(v, k, der):
        if der == 0:
            return v ** k
        if der == 1:
            return k * v ** (k - 1) if k >= 1 else 0 * v
        return k * (k - 1) * v ** (k - 2) if k >= 2 else 0 * v

    u = mono(x, a, 0) * mono(y, b, 0) * mono(z, c, 0)
    gx = mono(x, a, 1) * mono(y, b, 0) * mono(z, c, 0)
    gy = mono(x, a, 0) * mono(y, b, 1) * mono(z, c, 0)
    gz = mono(x, a, 0) * mono(y, b, 0) * mono(z, c, 1)
    lap = (mono(x, a, 2) * mono(y, b, 0) * mono(z, c, 0) + mono(x, a, 0) * mono(y, b, 2) * mono(z, c, 0)
           + mono(x, a, 0) * mono(y, b, 0) * mono(z, c, 2))
    return u[:, None, :], -lap[:, None, :], np.stack([gx, gy, gz], axis=1)[:, None, :, :]


# ---------------------------------------------------------------- Euler vortex
def vortex(mesh: Mesh, t: float = 0.0, beta: float = 5.0, center=(5.0, 5.0), gamma: float = 1.4,
           uinf=(1.0, 1.0), period=None, images: int = 0) -> np.ndarray:
    """Isentropic vortex of strength ``beta`` advected with ``uinf``.

    Free stream rho = p = 1, velocity ``uinf``; velocity perturbation
    ``beta/(2 pi) exp((1-r^2)/2) (-dy, dx)`` and temperature
    ``1 - (gamma-1) beta^2/(8 gamma pi^2) exp(1-r^2)``.  With ``period`` and
    ``images > 0`` the perturbations of periodic images are summed (the exact
    periodic solution to the accuracy of the far-field tails).
    Returns conserved variables ``[E, 4, Np]``.
    """
    x, y = mesh.xyz[:, 0], mesh.xyz[:, 1]
    du = np.zeros_like(x)
    dv = np.zeros_like(x)
    dT = np.zeros_like(x)
    shifts = [(0.0, 0.0)]
    if period is not None and images > 0:
        shifts = [(i * period[0], j * period[1]) for i in range(-images, images + 1)
                  for j in range(-images, images + 1)]
    for sx, sy in shifts:
        xc = x - center[0] - uinf[0] * t - sx
        yc = y - center[1] - uinf[1] * t - sy
        if period is not None and images == 0:
            xc = (xc + period[0] / 2) % period[0] - period[0] / 2
            yc = (yc + period[1] / 2) % period[1] - period[1] / 2
        r2 = xc * xc + yc * yc
        g = np.exp(0.5 * (1.0 - r2))
        du += -beta / (2 * math.pi) * yc * g
        dv += beta / (2 * math.pi) * xc * g
        dT += -(gamma - 1) * beta ** 2 / (8 * gamma * math.pi ** 2) * g * g
    T = 1.0 + dT
    rho = T ** (1.0 / (gamma - 1))
    u = uinf[0] + du
    v = uinf[1] + dv
    p = rho * T
    E = p / (gamma - 1) + 0.5 * rho * (u * u + v * v)
    return np.ascontiguousarray(np.stack([rho, rho * u, rho * v, E], axis=1))


# ---------------------------------------------------------------- Taylor-Green
def taylor_green(mesh: Mesh, mach: float = 0.2, gamma: float = 1.4, rho0: float = 1.0,
                 v0: float = 1.0, perturb_amp: float = 0.0, seed: int | None = None) -> np.ndarray:
    """Classical Taylor-Green vortex in conserved variables ``[E, 5, Np]``.

    u = V0 sin x cos y cos z, v = -V0 cos x sin y cos z, w = 0,
    p = p0 + rho0 V0^2/16 (cos 2x + cos 2y)(cos 2z + 2), rho = rho0 p / p0 with
    p0 = rho0 V0^2 / (gamma M^2).  With ``perturb_amp`` a seeded low-mode
    velocity perturbation (wavenumbers 1..2, random phases) is added.
    """
    x, y, z = mesh.xyz[:, 0], mesh.xyz[:, 1], mesh.xyz[:, 2]
    p0 = rho0 * v0 ** 2 / (gamma * mach ** 2)
    u = v0 * np.sin(x) * np.cos(y) * np.cos(z)
    v = -v0 * np.cos(x) * np.sin(y) * np.cos(z)
    w = np.zeros_like(x)
    if perturb_amp > 0:
        rng = np.random.default_rng(seed)
        for comp in (u, v, w):
            for _ in range(3):
                kx, ky, kz = rng.integers(1, 3, size=3)
                ph = rng.uniform(0, 2 * math.pi, size=3)
                a = rng.uniform(-1, 1)
                comp += perturb_amp * v0 * a * (np.sin(kx * x + ph[0]) * np.sin(ky * y + ph[1])
                                                * np.sin(kz * z + ph[2]))
    p = p0 + rho0 * v0 ** 2 / 16.0 * (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0)
    rho = rho0 * p / p0
    E = p / (gamma - 1) + 0.5 * rho * (u * u + v * v + w * w)
    return np.ascontiguousarray(np.stack([rho, rho * u, rho * v, rho * w, E], axis=1))


def constant_state(mesh: Mesh, state) -> np.ndarray:
    st = np.asarray(state, dtype=np.float64)
    return np.ascontiguousarray(np.broadcast_to(st[None, :, None], (mesh.n_elem, st.size, mesh.np_)).copy())


def random_smooth_state(mesh: Mesh, m: int, seed: int, base=None, amp: float = 0.1) -> np.ndarray:
    """A seeded smooth positive state (for Jacobian / invariance tests)."""
    rng = np.random.default_rng(seed)
    xyz = mesh.xyz
    out = np.empty((mesh.n_elem, m, mesh.np_))
    for c in range(m):
        acc = np.zeros(xyz.shape[0:1] + xyz.shape[2:])
        for _ in range(3):
            k = rng.uniform(0.5, 2.0, size=mesh.dim)
            ph = rng.uniform(0, 2 * math.pi)
            arg = sum(k[d] * xyz[:, d] for d in range(mesh.dim)) + ph
            acc += rng.uniform(-1, 1) * np.sin(arg)
        b = 0.0 if base is None else base[c]
        out[:, c] = b + amp * acc
    return out
