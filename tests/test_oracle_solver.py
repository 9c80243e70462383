"""Pins for the oracle's solvers: Poisson rates, vortex rates, BILU(0), GMRES, Newton (Sections 4-5)."""
import math
import os

import numpy as np
import pytest
import torch

from ldg_workloads import configs, fields, hex_mesh, quad_mesh
from oracle import LineDG, Physics
from oracle import solver
from oracle.physics import EQ_EULER, EQ_NS, EQ_POISSON

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def disc_of(pr):
    me = pr.mesh
    ph = Physics(pr.equation, me.dim, gamma=pr.gamma, mu=pr.mu, prandtl=pr.prandtl)
    return LineDG(me.dim, me.p, me.xyz, me.face_nbr, me.nbr_node, me.switch_plus, ph,
                  pr.c11_interior, pr.c11_dirichlet, pr.source, pr.gD)


# ------------------------------------------------------------------ P6: Poisson rates
def test_poisson_convergence_rates():
    rates = {}
    for line in open(os.path.join(GOLDEN, "poisson_p3_rates.txt")):
        if line.strip() and not line.startswith("#"):
            k, r, s = line.split()
            rates[k] = (float(r), float(s))
    eu, eq = [], []
    for n in (4, 8, 16, 32):
        pr = configs.poisson(n, 3)
        d = disc_of(pr)
        U = solver.steady_direct_solve(d)
        eu.append(np.abs(U.numpy() - pr.extra["u_exact"]).max())
        eq.append(np.abs(d.gradient(U).numpy() - pr.extra["grad_exact"]).max())
    ru = np.log2(np.array(eu[:-1]) / np.array(eu[1:]))
    rq = np.log2(np.array(eq[:-1]) / np.array(eq[1:]))
    assert np.all(ru[1:] >= rates["u"][0] - rates["u"][1])
    assert np.all(rq[1:] >= rates["q"][0] - rates["q"][1])
    # the 8x8 workload error lies on the fitted line between its neighbours
    assert eu[2] < eu[1] < eu[0]


# ------------------------------------------------------------------ P7: vortex
def test_vortex_convergence_and_conservation():
    """Isentropic vortex (Section 5.2): error against the exact translated vortex.

    The initial data are nodal values, so after a short time the nodal error is
    time x local truncation error, which converges like h^p; the h^{p+1} of the
    paper's long-time errors needs far more steps than a CPU test affords.
    Conserved totals (weights W_i W_j J) must not drift on the periodic mesh.
    """
    errs = []
    p = 3
    for n in (16, 32):
        pr = configs.euler_vortex(n, p, perturb=0.2, seed=0)
        d = disc_of(pr)
        U = torch.as_tensor(pr.U0)
        dt, steps = 2e-3, 10
        geo = d.geometry(torch.arange(d.E))
        W = d.ops.M.sum(1)
        w = torch.as_tensor(np.prod(W[d.node_coords()], axis=1))
        tot0 = (U * geo["J"][:, None, :] * w).sum(dim=(0, 2))
        for _ in range(steps):
            U = solver.rk4_step(d, U, dt)
        tot1 = (U * geo["J"][:, None, :] * w).sum(dim=(0, 2))
        assert torch.all((tot1 - tot0).abs() <= 1e-12 * tot0.abs())
        exact = fields.vortex(pr.mesh, dt * steps, period=(10.0, 10.0), images=1)
        errs.append(np.abs(U.numpy() - exact).max())
    assert math.log2(errs[0] / errs[1]) > p - 0.3


# ------------------------------------------------------------------ P10: BILU(0), GMRES, Newton
def small_ns(seed=0, p=2):
    mesh = quad_mesh(2, 2, p, box=((0, 2), (0, 2)), periodic=(True, True), perturb=0.2, seed=seed)
    ph = Physics(EQ_NS, 2, mu=0.05)
    d = LineDG(2, p, mesh.xyz, mesh.face_nbr, mesh.nbr_node, mesh.switch_plus, ph)
    U = fields.random_smooth_state(mesh, 4, seed=seed + 1, base=[1.0, 0.3, -0.2, 2.6], amp=0.05)
    return mesh, d, U


def test_bilu0_matches_on_pattern_and_is_exact_when_dense():
    mesh, d, U = small_ns()
    K11, K12, K21 = d.jacobian(U)
    At = solver.precond_matrix(d, K11, K12, K21, gamma=0.05)
    pat = solver.line_pattern(d)
    F = solver.bilu0(At, pat)
    Np, m = d.Np, d.m
    eye = torch.eye(m, dtype=torch.float64)
    L = torch.zeros_like(F)
    Uu = torch.zeros_like(F)
    for i in range(Np):
        for j in range(Np):
            if j < i:
                L[:, i, :, j, :] = F[:, i, :, j, :]
            else:
                Uu[:, i, :, j, :] = F[:, i, :, j, :]
        L[:, i, :, i, :] = eye
    E = F.shape[0]
    LU = (L.reshape(E, Np * m, Np * m) @ Uu.reshape(E, Np * m, Np * m)).reshape(F.shape)
    mask = torch.as_tensor(pat)[None, :, None, :, None]
    assert torch.allclose(LU * mask, At * mask, atol=1e-12)
    # factor pattern is the matrix pattern (no fill)
    assert torch.all(F * ~mask == 0)
    # the triangular solves invert L U
    r = torch.randn(E, m, Np, dtype=torch.float64)
    z = solver.bilu0_apply(F, pat, r)
    zz = z.permute(0, 2, 1).reshape(E, Np * m, 1)
    back = (LU.reshape(E, Np * m, Np * m) @ zz).reshape(E, Np, m).permute(0, 2, 1)
    assert torch.allclose(back, r, atol=1e-11)
    # with a full pattern ILU(0) is the exact block LU
    full = np.ones_like(pat)
    F2 = solver.bilu0(At, full)
    z2 = solver.bilu0_apply(F2, full, r)
    assert torch.allclose(z2, solver.dense_block_solve(At, r), atol=1e-11)


def test_gmres_matches_dense_solve():
    mesh, d, U = small_ns(3)
    K11, K12, K21 = d.jacobian(U)
    gamma = 0.05
    A = solver.dense_operator(d, K11, K12, K21)
    M = np.eye(A.shape[0]) - gamma * A
    b = torch.randn(d.E, d.m, d.Np, dtype=torch.float64)
    x_ref = np.linalg.solve(M, b.reshape(-1).numpy())
    pat = solver.line_pattern(d)
    F = solver.bilu0(solver.precond_matrix(d, K11, K12, K21, gamma), pat)
    mv = lambda x: solver.split_matvec(d, K11, K12, x, gamma)
    x, its, rel = solver.gmres(mv, lambda r: solver.bilu0_apply(F, pat, r), b, rtol=1e-10, restart=20)
    kappa = np.linalg.cond(M)
    assert rel <= 1e-10
    assert np.abs(x.reshape(-1).numpy() - x_ref).max() <= 1e-10 * kappa * np.abs(x_ref).max()
    # the preconditioner helps: fewer iterations than without it
    _, its_none, _ = solver.gmres(mv, lambda r: r, b, rtol=1e-10, restart=20, max_iters=400)
    assert its < its_none


def test_poisson_newton_step_is_the_linear_solve():
    pr = configs.poisson(4, 3)
    d = disc_of(pr)
    res = solver.newton_step(d, pr.U0, None, gamma=1.0, alpha=0.0, rtol=1e-12, max_iters=3000)
    Ud = solver.steady_direct_solve(d)
    assert res["lin_relres"] <= 1e-12
    assert torch.allclose(res["U"], Ud, atol=1e-9 * float(Ud.abs().max()))
    assert res["G1"] <= 1e-9 * res["G0"]


def test_bdf2_newton_step_converges_quadratically():
    mesh, d, U = small_ns(5)
    dt = 0.05
    gamma = 2 * dt / 3
    Ucomb = U.clone() if torch.is_tensor(U) else torch.as_tensor(U)
    r1 = solver.newton_step(d, U, Ucomb, gamma, rtol=1e-12)
    assert r1["lin_relres"] <= 1e-12
    r2 = solver.newton_step(d, r1["U"], Ucomb, gamma, rtol=1e-12)
    assert r1["G1"] < 1e-2 * r1["G0"]
    assert r2["G1"] < 1e-3 * r2["G0"]
    # exact-block preconditioner needs no more iterations than BILU(0)
    r3 = solver.newton_step(d, U, Ucomb, gamma, rtol=1e-12, precond="exact")
    assert r3["iters"] <= r1["iters"]


def test_dirk3_coefficients():
    """Section 4.1 tableau: alpha is a root of x^3 - 3x^2 + 3x/2 - 1/6 and b1 + b2 + alpha = 1."""
    a = 0.435866521508459
    b1 = -(6 * a * a - 16 * a + 1) / 4
    b2 = (6 * a * a - 20 * a + 5) / 4
    assert abs(b1 + b2 + a - 1) < 1e-15
    assert abs(a ** 3 - 3 * a ** 2 + 1.5 * a - 1 / 6) < 1e-15


# ------------------------------------------------------------------ A~ against its definition (Section 4.2)
def _intra_element_columns(d, K11, K12, gamma, alpha, e):
    """Columns of alpha I - gamma (K11_ee + K12_ee K21_ee) for element e, one unit vector at a
    time: x = e_(b,k) on element e, w = D(x) with zero boundary data kept on element e only
    (K21 taken inside the element), y = alpha x - gamma (K11 x + K12 w) read on element e."""
    E, m, Np, D = d.E, d.m, d.Np, d.D
    c11, c12 = d.column_nodes("K11"), d.column_nodes("K12")
    out = torch.zeros(Np, m, Np, m, dtype=torch.float64)
    for b in range(Np):
        for k in range(m):
            x = torch.zeros(E, m, Np, dtype=torch.float64)
            x[e, k, b] = 1.0
            w = d.gradient(x, homogeneous=True)
            keep = torch.zeros(E, 1, 1, 1, dtype=torch.float64)
            keep[e] = 1.0
            w = (w * keep).reshape(E, m * D, Np)
            y = alpha * x - gamma * (solver.blocks_apply(d, K11, c11, x, m) + solver.blocks_apply(d, K12, c12, w, m * D))
            out[:, :, b, k] = y[e].T
    return out


def test_precond_matrix_is_the_masked_operator_of_an_isolated_element():
    """A single element with Dirichlet faces couples to nothing else, so A = K11 + K12 K21 is
    element-local and A~ must be alpha I - gamma A masked to the line pattern (Section 4.2)."""
    mesh = hex_mesh(1, 2, length=1.0, periodic=False, amp=0.05)
    ph = Physics(EQ_NS, 3, mu=0.05)
    U = fields.random_smooth_state(mesh, 5, seed=3, base=[1.0, 0.3, -0.2, 0.1, 2.6], amp=0.05)
    # Dirichlet data: a valid gas state (the inviscid boundary flux is Roe(g_D, u_in))
    gD = fields.face_values(mesh, fields.random_smooth_state(mesh, 5, seed=4, base=[1.0, 0.2, 0.1, -0.1, 2.5],
                                                               amp=0.05))
    d = LineDG(3, 2, mesh.xyz, mesh.face_nbr, mesh.nbr_node, mesh.switch_plus, ph, 0.0, 10.0, None, gD)
    K11, K12, K21 = d.jacobian(U)
    gamma, alpha = 0.05, 1.0
    At = solver.precond_matrix(d, K11, K12, K21, gamma, alpha)
    Ad = solver.dense_operator(d, K11, K12, K21)  # [E m Np] ordering
    Np, m = d.Np, d.m
    A5 = torch.as_tensor(Ad).reshape(m, Np, m, Np).permute(1, 0, 3, 2)  # [a, c, b, k]
    ref = alpha * torch.eye(Np * m, dtype=torch.float64).reshape(Np, m, Np, m) - gamma * A5
    mask = torch.as_tensor(solver.line_pattern(d))[:, None, :, None].to(torch.float64)
    assert torch.allclose(At[0], ref * mask, rtol=0, atol=1e-12 * float(ref.abs().max()))
    # and the masked part is not trivially the whole operator: K12 K21 fills outside the pattern
    assert float((ref * (1 - mask)).abs().max()) > 1e-6


@pytest.mark.parametrize("dim", [2, 3])
def test_precond_matrix_is_the_intra_element_restriction(dim):
    """On a periodic mesh with reversed element axes (S = -1 faces), A~_e equals the line-pattern
    mask of alpha I - gamma (K11_ee + K12_ee K21_ee), built here from the split product with the
    gradient of unit vectors kept inside the element."""
    from tests.test_oracle_linedg import flip_mesh
    if dim == 2:
        mesh = flip_mesh(quad_mesh(3, 3, 2, box=((0, 3), (0, 3)), periodic=(True, True), perturb=0.2, seed=1), 2)
        base = [1.0, 0.3, -0.2, 2.6]
    else:
        mesh = flip_mesh(hex_mesh(2, 1, amp=0.15), 3)
        base = [1.0, 0.3, -0.2, 0.1, 2.6]
    ph = Physics(EQ_NS, dim, mu=0.05)
    d = LineDG(dim, mesh.p, mesh.xyz, mesh.face_nbr, mesh.nbr_node, mesh.switch_plus, ph)
    U = fields.random_smooth_state(mesh, d.m, seed=4, base=base, amp=0.05)
    K11, K12, K21 = d.jacobian(U)
    gamma, alpha = 0.05, 1.0
    At = solver.precond_matrix(d, K11, K12, K21, gamma, alpha)
    mask = torch.as_tensor(solver.line_pattern(d))[:, None, :, None].to(torch.float64)
    flipped = np.nonzero((mesh.switch_plus < 0).any(1))[0]
    assert len(flipped) > 0
    for e in sorted({0, int(flipped[0]), d.E - 1}):
        ref = _intra_element_columns(d, K11, K12, gamma, alpha, e) * mask
        assert torch.allclose(At[e], ref, rtol=0, atol=1e-12 * float(ref.abs().max())), e


def _heat_problem():
    """Poisson operator with zero Dirichlet data and no source: dU/dt = R(U) = A U is linear."""
    mesh = quad_mesh(2, 2, 2, box=((0, 1), (0, 1)), perturb=0.1, seed=3)
    ph = Physics(EQ_POISSON, 2)
    d = LineDG(2, 2, mesh.xyz, mesh.face_nbr, mesh.nbr_node, mesh.switch_plus, ph, 0.0, 10.0)
    U0 = torch.as_tensor(np.sin(3.0 * mesh.xyz[:, 0:1]) * np.cos(2.0 * mesh.xyz[:, 1:2]))
    K11, K12, K21 = d.jacobian(U0)
    A = solver.dense_operator(d, K11, K12, K21)
    return d, U0, A


def test_dirk3_is_third_order_against_the_matrix_exponential():
    """On the linear system dU/dt = A U the DIRK3 step reproduces expm(t A) U0 with error
    O(dt^3) at fixed t (the tableau's order), so halving dt divides the error by about 8."""
    import scipy.linalg
    d, U0, A = _heat_problem()
    lam = float(np.abs(np.linalg.eigvals(A)).max())
    T = 4.0 / lam
    exact = scipy.linalg.expm(T * A) @ U0.reshape(-1).numpy()
    errs = []
    for nsteps in (4, 8, 16):
        U = U0.clone()
        for _ in range(nsteps):
            U, st = solver.dirk3_step(d, U, T / nsteps, newton_tol=1e-10)
        errs.append(float(np.abs(U.reshape(-1).numpy() - exact).max()))
    r1, r2 = np.log2(errs[0] / errs[1]), np.log2(errs[1] / errs[2])
    assert r1 > 2.6 and r2 > 2.7, (errs, r1, r2)


def test_dirk3_is_l_stable():
    """A single step with dt far beyond the stiffest mode damps every mode (L-stability:
    the stability function vanishes at -infinity), where Crank-Nicolson would not."""
    d, U0, A = _heat_problem()
    lam = float(np.abs(np.linalg.eigvals(A)).max())
    lam_min = float(np.abs(np.linalg.eigvals(A)).min())
    U1, _ = solver.dirk3_step(d, U0, 1e4 / lam_min)
    assert float(U1.abs().max()) < 1e-3 * float(U0.abs().max())
