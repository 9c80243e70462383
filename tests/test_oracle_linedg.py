"""Pins for the oracle's line-DG residual, gradient and Jacobians (Sections 2-4)."""
import math
import os

import numpy as np
import pytest
import torch

from ldg_workloads import (BC_NEUMANN, BC_SLIP, configs, fields, hex_mesh, quad_mesh, reorient_elements,
                           with_boundary_kinds)
from oracle import LineDG, Physics
from oracle.basis import LineOps
from oracle.physics import EQ_EULER, EQ_NS, EQ_POISSON
from oracle import solver

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def disc(mesh, eq, mu=0.0, **kw):
    ph = Physics(eq, mesh.dim, mu=mu)
    return LineDG(mesh.dim, mesh.p, mesh.xyz, mesh.face_nbr, mesh.nbr_node, mesh.switch_plus, ph, **kw)


def base_state(dim):
    return [1.0, 0.3, -0.2, 2.6] if dim == 2 else [1.0, 0.3, -0.2, 0.1, 2.6]


# ------------------------------------------------------------------ P2: Q_p exactness
@pytest.mark.parametrize("p", [2, 3, 4])
def test_poisson_qp_exactness_2d(p):
    """u in Q_p on an affine mesh with g_D = u, f = -Lap u: q = grad u and R = 0."""
    mesh = quad_mesh(3, 3, p, box=((0.2, 1.4), (-0.3, 0.9)))
    u, f, g = fields.poisson_polynomial(mesh, degs=(p, p - 1))
    d = disc(mesh, EQ_POISSON, source=f, gD=fields.face_values(mesh, u))
    Q = d.gradient(u).numpy()
    assert np.abs(Q - g).max() <= 1e-11 * np.abs(g).max()
    R, mag = d.residual(u, return_abs=True)
    assert R.abs().max() <= 1e-11 * mag.max()


def test_poisson_qp_exactness_3d():
    mesh = hex_mesh(2, 2, length=1.0, periodic=False, amp=0.0)
    u, f, g = fields.poisson_polynomial_3d(mesh, degs=(2, 1, 2))
    d = disc(mesh, EQ_POISSON, source=f, gD=fields.face_values(mesh, u))
    Q = d.gradient(u).numpy()
    assert np.abs(Q - g).max() <= 1e-11 * np.abs(g).max()
    R, mag = d.residual(u, return_abs=True)
    assert R.abs().max() <= 1e-11 * mag.max()


# ------------------------------------------------------------------ P3: stencil count
def test_costtab_closed_forms():
    tab = np.loadtxt(os.path.join(GOLDEN, "costtab.txt"), dtype=np.int64)
    p = tab[:, 0]
    assert np.array_equal(tab[:, 1], 2 * p + 1 + 4)          # 2-D Line-DG: D p + 1 + 2D
    assert np.array_equal(tab[:, 4], 3 * p + 1 + 6)          # 3-D Line-DG
    assert np.array_equal(tab[:, 2], 2 * p + 1 + 4 * (p + 1))  # 2-D DGSEM/SD
    assert np.array_equal(tab[:, 5], 3 * p + 1 + 6 * (p + 1))  # 3-D DGSEM/SD
    assert np.array_equal(tab[:, 3], (p + 1) ** 2 + 4)
    assert np.array_equal(tab[:, 6], (p + 1) ** 3 + 6 * (p + 1))
    assert tab[2, 6] / tab[2, 4] == 5.5                        # "5.5 times sparser" at p = 3
    assert 37 < tab[9, 6] / tab[9, 4] < 40                     # "almost 40 times" at p = 10


@pytest.mark.parametrize("dim,p", [(2, 1), (2, 2), (2, 3), (2, 4), (3, 1), (3, 2)])
def test_k11_stencil_count(dim, p):
    """Every node row of K11 has exactly D p + 1 + 2D nonzero m x m blocks (periodic mesh)."""
    tab = np.loadtxt(os.path.join(GOLDEN, "costtab.txt"), dtype=np.int64)
    expect = int(tab[p - 1, 1 if dim == 2 else 4])
    if dim == 2:
        mesh = quad_mesh(3, 3, p, box=((0, 3), (0, 3)), periodic=(True, True), perturb=0.2, seed=5)
    else:
        mesh = hex_mesh(3, p)
    d = disc(mesh, EQ_NS, mu=0.05)
    U = fields.random_smooth_state(mesh, d.m, seed=2, base=base_state(dim), amp=0.05)
    K11, K12, K21 = d.jacobian(U)
    nz = (K11.abs().amax(dim=(-1, -2)) > 0)
    cols = d.column_nodes("K11")
    # distinct column nodes per row
    assert np.all((cols >= 0).sum(-1) == expect)
    assert torch.all(nz.sum(-1) == expect)
    # K12 and K21 rows couple D p + 1 + D node blocks
    assert torch.all((K12.abs().amax(dim=(-1, -2)) > 0).sum(-1) == dim * p + 1 + dim)
    assert torch.all((K21.abs().amax(dim=-1) > 0).sum(-1) == dim * p + 1 + dim)


# ------------------------------------------------------------------ P4: freestream
def flux_scale(d, state):
    """|F(u)| |a_n| / J: the size of each directional flux derivative for a constant state."""
    geo = d.geometry(torch.arange(d.E))
    F = d.ph.flux_inv(torch.as_tensor(state, dtype=torch.float64))
    amax = max(float(torch.linalg.norm(a, dim=-1).max()) for a in geo["ag"])
    return float(F.abs().max()) * amax / float(geo["J"].abs().min())


def curved_quad(n, p):
    L = 4.0
    def curve(x, y):
        return (x + 0.15 * np.sin(math.pi * x / 2) * np.sin(math.pi * y / 2),
                y - 0.1 * np.sin(math.pi * x / 2) * np.sin(math.pi * y))
    return quad_mesh(n, n, p, box=((0, L), (0, L)), periodic=(True, True), perturb=0.15, seed=3, curve=curve)


@pytest.mark.parametrize("p", [2, 3, 4])
def test_freestream_curved_2d(p):
    mesh = curved_quad(4, p)
    d = disc(mesh, EQ_EULER)
    U = fields.constant_state(mesh, base_state(2))
    R = d.residual(U)
    assert R.abs().max() <= 1e-12 * flux_scale(d, base_state(2))


def test_freestream_3d():
    """Exact on affine hexes and on the workload map X + b(X) (b added to every coordinate,
    whose cofactor metric is linear in grad b); on a general curved Q_p hex the
    metric terms along a line have degree 2p, so freestream holds only up to
    truncation error, which must decay under refinement."""
    for amp in (0.0, 0.1):
        mesh = hex_mesh(2, 3, amp=amp)
        d = disc(mesh, EQ_EULER)
        R = d.residual(fields.constant_state(mesh, base_state(3)))
        assert R.abs().max() <= 1e-12 * flux_scale(d, base_state(3))

    def general(X, Y, Z):
        return (X + 0.1 * np.sin(Y) * np.sin(Z) * np.sin(X),
                Y + 0.08 * np.sin(X) * np.sin(Z),
                Z + 0.05 * np.sin(2 * X) * np.sin(Y))
    errs = []
    for n in (4, 8):
        mesh = hex_mesh(n, 2, curve=general)
        d = disc(mesh, EQ_EULER)
        R = d.residual(fields.constant_state(mesh, base_state(3)))
        errs.append(float(R.abs().max()) / flux_scale(d, base_state(3)))
    assert errs[0] > 1e-6
    assert errs[1] < errs[0] / 8  # decays at least like h^3


# ------------------------------------------------------------------ P5: conservation
def weights3(d):
    W = d.ops.M.sum(1)
    co = d.node_coords()
    return torch.as_tensor(np.prod(W[co], axis=1))


@pytest.mark.parametrize("dim,eq", [(2, EQ_EULER), (2, EQ_NS), (3, EQ_NS)])
def test_discrete_conservation(dim, eq):
    if dim == 2:
        mesh = quad_mesh(4, 3, 3, box=((0, 4), (0, 3)), periodic=(True, True), perturb=0.2, seed=7)
    else:
        mesh = hex_mesh(2, 2)
    d = disc(mesh, eq, mu=0.05)
    U = fields.random_smooth_state(mesh, d.m, seed=9, base=base_state(dim), amp=0.1)
    R, mag = d.residual(U, return_abs=True)
    geo = d.geometry(torch.arange(d.E))
    w = weights3(d)
    tot = (R * geo["J"][:, None, :] * w).sum(dim=(0, 2))
    scale = (mag * geo["J"][:, None, :].abs() * w).sum(dim=(0, 2))
    assert torch.all(tot.abs() <= 1e-13 * scale)


# ------------------------------------------------------------------ P8: Jacobian vs FD
@pytest.mark.parametrize("dim,eq,p", [(2, EQ_EULER, 2), (2, EQ_NS, 3), (2, EQ_POISSON, 2), (3, EQ_NS, 2)])
def test_jacobian_vs_finite_differences(dim, eq, p):
    if dim == 2:
        mesh = quad_mesh(2, 2, p, box=((0, 2), (0, 2)), periodic=(True, eq != EQ_POISSON), perturb=0.2, seed=1)
    else:
        mesh = hex_mesh(2, p)
    kw = {}
    if eq == EQ_POISSON:
        kw = dict(gD=np.zeros((mesh.n_elem, 2 * dim, 1, mesh.nf)), c11_interior=0.3)
    d = disc(mesh, eq, mu=0.1, **kw)
    base = [0.4] if eq == EQ_POISSON else base_state(dim)
    U = fields.random_smooth_state(mesh, d.m, seed=3, base=base, amp=0.05)
    K11, K12, K21 = d.jacobian(U)
    A = solver.dense_operator(d, K11, K12, K21)
    rng = np.random.default_rng(0)
    for _ in range(2):
        v = rng.standard_normal(U.shape)
        eps = 1e-6
        fd = ((d.residual(U + eps * v) - d.residual(U - eps * v)) / (2 * eps)).numpy().reshape(-1)
        assert np.abs(fd - A @ v.reshape(-1)).max() <= 1e-6 * np.abs(fd).max()
    # K21 is linear: the homogeneous gradient of a combination
    x, y = rng.standard_normal(U.shape), rng.standard_normal(U.shape)
    lhs = d.gradient(2.0 * x - 0.5 * y, homogeneous=True)
    rhs = 2.0 * d.gradient(x, homogeneous=True) - 0.5 * d.gradient(y, homogeneous=True)
    assert torch.allclose(lhs, rhs, atol=1e-13 * float(rhs.abs().max()))


# ------------------------------------------------------------------ P9: NS at mu = 0
@pytest.mark.parametrize("dim", [2, 3])
def test_ns_zero_viscosity_equals_euler(dim):
    mesh = quad_mesh(3, 3, 2, box=((0, 3), (0, 3)), periodic=(True, True), perturb=0.2) if dim == 2 \
        else hex_mesh(2, 2)
    U = fields.random_smooth_state(mesh, dim + 2, seed=4, base=base_state(dim), amp=0.1)
    Re = disc(mesh, EQ_EULER).residual(U)
    ph = Physics(EQ_NS, dim, mu=0.0)
    ph.has_viscous = True  # evaluate the viscous terms with mu = 0
    dn = LineDG(dim, mesh.p, mesh.xyz, mesh.face_nbr, mesh.nbr_node, mesh.switch_plus, ph)
    Rn = dn.residual(U)
    assert torch.allclose(Rn, Re, atol=1e-14 * float(Re.abs().max()))
    # a constant state has zero gradient
    Uc = fields.constant_state(mesh, base_state(dim))
    assert dn.gradient(Uc).abs().max() < 1e-12


# ------------------------------------------------------------------ NS consistency
def test_ns_residual_consistency_with_divergence():
    """R_h(u) -> -div F(u, grad u) under refinement for a smooth field (affine 2-D mesh).

    The exact divergence is formed by automatic differentiation of the same
    physical flux evaluated on the analytic field, so this pins the
    discretisation (not the flux formula, which has its own closed-form pins).
    """
    mu = 0.05
    ph = Physics(EQ_NS, 2, mu=mu)

    def field(X):  # X [..., 2] -> conserved state [..., 4]
        x, y = X[..., 0], X[..., 1]
        rho = 1.0 + 0.2 * torch.sin(x) * torch.cos(y)
        u = 0.3 + 0.1 * torch.cos(x + y)
        v = -0.2 + 0.1 * torch.sin(x - 2 * y)
        p = 1.0 + 0.1 * torch.cos(2 * x) * torch.sin(y)
        E = p / 0.4 + 0.5 * rho * (u * u + v * v)
        return torch.stack([rho, rho * u, rho * v, E], dim=-1)

    def flux_at(X):
        Xr = X.clone().requires_grad_(True)
        U = field(Xr)
        q = torch.stack([torch.autograd.grad(U[..., c].sum(), Xr, create_graph=True)[0] for c in range(4)], -2)
        return ph.flux_total(U, q), Xr

    def div_exact(X):
        F, Xr = flux_at(X)
        out = []
        for c in range(4):
            g0 = torch.autograd.grad(F[..., c, 0].sum(), Xr, retain_graph=True)[0][..., 0]
            g1 = torch.autograd.grad(F[..., c, 1].sum(), Xr, retain_graph=True)[0][..., 1]
            out.append(g0 + g1)
        return torch.stack(out, -1).detach()

    errs = []
    for n in (8, 16):
        mesh = quad_mesh(n, n, 3, box=((0, 2 * math.pi), (0, 2 * math.pi)), periodic=(True, True))
        X = torch.as_tensor(mesh.xyz).permute(0, 2, 1)  # [E, Np, 2]
        U = field(X).permute(0, 2, 1).detach()
        d = LineDG(2, 3, mesh.xyz, mesh.face_nbr, mesh.nbr_node, mesh.switch_plus, ph)
        R = d.residual(U)
        ref = -div_exact(X).permute(0, 2, 1)
        errs.append(float((R - ref).abs().max() / ref.abs().max()))
    # the viscous terms differentiate q = D(u) once more: truncation order p - 1 = 2
    assert errs[1] < errs[0] / 2 ** 1.7
    assert errs[1] < 0.02


# ------------------------------------------------------------------ P11: relabelling invariance
@pytest.mark.parametrize("eq", [EQ_EULER, EQ_NS])
def test_relabelling_invariance(eq):
    mesh = quad_mesh(4, 4, 3, box=((0, 4), (0, 4)), periodic=(True, True), perturb=0.2, seed=11)
    U = fields.random_smooth_state(mesh, 4, seed=12, base=base_state(2), amp=0.1)
    R = disc(mesh, eq, mu=0.05).residual(U).numpy()
    rng = np.random.default_rng(13)
    flips = np.zeros((mesh.n_elem, 2), dtype=bool)
    rot = rng.random(mesh.n_elem) < 0.5
    flips[rot] = True  # 180 degree rotation of about half the elements
    perm = rng.permutation(mesh.n_elem)
    m2 = reorient_elements(mesh, flips, perm)
    # relabel the state the same way
    U2 = np.empty_like(U)
    n1 = mesh.n1
    idx = np.arange(mesh.np_)
    i, j = idx % n1, idx // n1
    for e in range(mesh.n_elem):
        ii = np.where(flips[e, 0], mesh.p - i, i)
        jj = np.where(flips[e, 1], mesh.p - j, j)
        U2[perm[e]] = U[e][:, ii + n1 * jj]
    R2 = disc(m2, eq, mu=0.05).residual(U2).numpy()
    Rback = np.empty_like(R)
    for e in range(mesh.n_elem):
        ii = np.where(flips[e, 0], mesh.p - i, i)
        jj = np.where(flips[e, 1], mesh.p - j, j)
        Rback[e][:, ii + n1 * jj] = R2[perm[e]]
    assert np.abs(Rback - R).max() <= 1e-12 * np.abs(R).max()
    assert np.any(m2.switch_plus < 0)


# ------------------------------------------------------------------ K21 weights = homogeneous gradient
def flip_mesh(mesh, seed, frac=0.5):
    from tests.gpu_cases import flip_mesh as fm
    return fm(mesh, seed, frac)[0]


def apply_k21(d, W, x):
    """w[e, c, dd, a] = sum over slots of W[e, a, slot, dd] x[column node of the slot, c]."""
    cols = d.column_nodes("K21")
    E, m, Np = d.E, d.m, d.Np
    xf = torch.as_tensor(x, dtype=torch.float64).reshape(E, m, Np).permute(0, 2, 1).reshape(E * Np, m)
    c = torch.as_tensor(cols)
    ok = (c >= 0)
    xs = xf[torch.where(ok, c, torch.zeros_like(c))] * ok[..., None].to(torch.float64)  # [E, Np, ns, m]
    return torch.einsum("easd,easc->ecda", W, xs)


@pytest.mark.parametrize("kind", ["quad_dirichlet_flipped", "hex_periodic", "hex_flipped"])
def test_k21_weights_apply_as_homogeneous_gradient(kind):
    """The stored K21 weights (line slots and the switch-side neighbour slot) reproduce
    D(x) with zero boundary data for any x (Section 4.1: K21 = dD/dU, D linear in U),
    including elements whose local axes are reversed so that S = -1 occurs."""
    if kind == "quad_dirichlet_flipped":
        mesh = flip_mesh(quad_mesh(3, 3, 3, box=((0, 3), (0, 3)), perturb=0.2, seed=8), seed=9)
    elif kind == "hex_periodic":
        mesh = hex_mesh(2, 2)
    else:
        mesh = flip_mesh(hex_mesh(2, 2, amp=0.15), seed=10)
    d = disc(mesh, EQ_NS, mu=0.05)
    W = d.k21()
    x = torch.randn(d.E, d.m, d.Np, generator=torch.Generator().manual_seed(4), dtype=torch.float64)
    w = apply_k21(d, W, x)
    ref = d.gradient(x, homogeneous=True)
    assert float((w - ref).abs().max()) <= 1e-12 * float(ref.abs().max())
    if kind != "hex_periodic":
        assert np.any(mesh.switch_plus < 0)
    # the Jacobian's own K21 output is the same operator
    _, _, K21 = d.jacobian(fields.random_smooth_state(mesh, d.m, seed=5, base=base_state(mesh.dim), amp=0.05))
    assert torch.allclose(K21, W, rtol=0, atol=1e-13 * float(W.abs().max()))



# ------------------------------------------------------------------ Neumann faces and slip walls (Section 3)
@pytest.mark.parametrize("dim,p", [(2, 2), (2, 3), (3, 2)])
def test_poisson_qp_exactness_mixed_dirichlet_neumann(dim, p):
    """u in Q_p on a mesh of rectangular elements: g_D = u on the faces xi_n = 0 of the box and the
    Neumann data g_N = F(u, grad u) . nhat = -grad u . nhat on the faces xi_n = 1 (eqs. neumann1/2
    with C22 = 0): the discrete gradient is grad u and R = 0 at every node."""
    if dim == 2:
        base = quad_mesh(3, 3, p, box=((0.2, 1.4), (-0.3, 0.9)))
        u, f, g = fields.poisson_polynomial(base, degs=(p, p - 1))
    else:
        base = hex_mesh(2, p, length=1.0, periodic=False, amp=0.0)
        u, f, g = fields.poisson_polynomial_3d(base, degs=(p, 1, p))
    mesh = with_boundary_kinds(base, {2 * n + 1: BC_NEUMANN for n in range(dim)})
    gN = -fields.axis_normal_face_values(mesh, g)
    d = disc(mesh, EQ_POISSON, source=f, gD=fields.face_values(mesh, u), gN=gN)
    Q = d.gradient(u).numpy()
    assert np.abs(Q - g).max() <= 1e-11 * np.abs(g).max()
    R, mag = d.residual(u, return_abs=True)
    assert R.abs().max() <= 1e-11 * mag.max()
    # the Neumann data enters: other data changes R on the Neumann faces only
    d2 = disc(mesh, EQ_POISSON, source=f, gD=fields.face_values(mesh, u), gN=gN + 1.0)
    R2 = d2.residual(u)
    assert R2.abs().max() > 1e-3


def channel(p=3, eq=EQ_EULER, perturb=0.2):
    """Periodic in x, slip walls at y = 0 and y = 2 (straight: boundary vertices are not moved)."""
    base = quad_mesh(4, 3, p, box=((0, 4), (0, 2)), periodic=(True, False), perturb=perturb, seed=3)
    return with_boundary_kinds(base, {0 + 2: BC_SLIP, 1 + 2: BC_SLIP})


@pytest.mark.parametrize("eq", [EQ_EULER, EQ_NS])
def test_slip_wall_uniform_flow_along_the_wall(eq):
    """Flow parallel to a slip wall is its own mirror state, so the wall flux is the physical
    pressure flux and a uniform flow stays steady (R = 0) on the perturbed channel mesh."""
    mesh = channel(eq=eq)
    U = fields.constant_state(mesh, [1.0, 0.5, 0.0, 2.6])
    d = disc(mesh, eq, mu=0.05)
    R = d.residual(U)
    assert float(R.abs().max()) <= 1e-12 * flux_scale(d, [1.0, 0.5, 0.0, 2.6])


@pytest.mark.parametrize("eq", [EQ_EULER, EQ_NS])
def test_slip_wall_conserves_mass_and_energy(eq):
    """Through a slip wall the Roe flux of the mirror state carries no mass and no energy (its
    central part and its dissipation both vanish there), so on the channel mass and energy are
    conserved discretely while the wall-normal momentum is not (the wall pressure force)."""
    mesh = channel(eq=eq)
    d = disc(mesh, eq, mu=0.05)
    U = fields.random_smooth_state(mesh, d.m, seed=9, base=base_state(2), amp=0.1)
    R, mag = d.residual(U, return_abs=True)
    geo = d.geometry(torch.arange(d.E))
    w = weights3(d)
    tot = (R * geo["J"][:, None, :] * w).sum(dim=(0, 2))
    scale = (mag * geo["J"][:, None, :].abs() * w).sum(dim=(0, 2))
    assert abs(float(tot[0])) <= 1e-13 * float(scale[0])
    assert abs(float(tot[3])) <= 1e-13 * float(scale[3])
    assert abs(float(tot[2])) > 1e-6 * float(scale[2])


@pytest.mark.parametrize("eq,kind", [(EQ_EULER, BC_SLIP), (EQ_NS, BC_SLIP), (EQ_POISSON, BC_NEUMANN),
                                     (EQ_NS, BC_NEUMANN)])
def test_jacobian_vs_finite_differences_with_boundaries(eq, kind):
    """Jacobians (dual numbers) against central differences of the residual on a mesh with
    Dirichlet faces and Neumann faces or slip walls (P8 with boundaries)."""
    p = 2
    base = quad_mesh(2, 2, p, box=((0, 2), (0, 2)), periodic=(True, False), perturb=0.2, seed=1)
    mesh = with_boundary_kinds(base, {3: kind})
    m = 1 if eq == EQ_POISSON else 4
    state = [0.4] if eq == EQ_POISSON else base_state(2)
    gD = fields.face_values(mesh, fields.random_smooth_state(mesh, m, seed=5, base=state, amp=0.05))
    gN = 0.1 * fields.face_values(mesh, fields.random_smooth_state(mesh, m, seed=6, base=None, amp=1.0))
    d = disc(mesh, eq, mu=0.1, gD=gD, gN=gN, c11_interior=0.3 if eq == EQ_POISSON else 0.0)
    U = fields.random_smooth_state(mesh, m, seed=3, base=state, amp=0.05)
    K11, K12, K21 = d.jacobian(U)
    A = solver.dense_operator(d, K11, K12, K21)
    rng = np.random.default_rng(0)
    for _ in range(2):
        v = rng.standard_normal(U.shape)
        eps = 1e-6
        fd = ((d.residual(U + eps * v) - d.residual(U - eps * v)) / (2 * eps)).numpy().reshape(-1)
        assert np.abs(fd - A @ v.reshape(-1)).max() <= 1e-6 * np.abs(fd).max()
    # K21 weights reproduce the homogeneous gradient (inside traces on Neumann faces and walls)
    x = torch.as_tensor(rng.standard_normal(U.shape))
    w = apply_k21(d, d.k21(), x)
    ref = d.gradient(x, homogeneous=True)
    assert float((w - ref).abs().max()) <= 1e-12 * float(ref.abs().max())
