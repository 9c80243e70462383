"""The coupled (U, Q) system with C22 != 0 (Section 4.1; the C22 terms of eqs. ldgflux1/2 and
neumann1/2) solved on the GPU against the oracle's dense solve of the same system.

Bound (2-norm over all unknowns x = [U; Q]): the GPU stops with the true residual
||b - A_g x_g|| = rho ||b|| of its own FP64 operator A_g, and A_g differs from the exact A by the
rounding of the residual and gradient kernels, ||A - A_g|| <= delta ||A||, delta = 2 n_row u with
n_row the largest number of non-zeros in a row of A.  So
  ||x_g - x|| <= kappa_2(A) (rho + delta ||A|| ||x_g|| / ||b||) ||x||   (to first order),
and the oracle's LU solve adds at most kappa_2(A) n u ||x||; the test allows twice the sum.
Q_p exactness (polynomial data of degree p on affine elements): every jump of the normal flux
vanishes, so the coupled solution is u and grad u at the nodes for any C22.
"""
import numpy as np
import pytest
import torch
from torch.func import jacfwd

from ldg_workloads import BC_NEUMANN, configs, fields, hex_mesh, quad_mesh, with_boundary_kinds
from oracle import solver
from oracle.linedg import LineDG
from oracle.physics import EQ_POISSON, Physics
from paper_1204_1533_amd.ldg import LDG_PRECOND_BLOCK_LU, LDGError
from tests.gpu_cases import gpu_of, record

pytestmark = pytest.mark.gpu
U53 = 2.0 ** -53


def poisson_problem(name):
    """Poisson problems of the coupled tests: (Problem, C11 interior, C22)."""
    if name == "quad4p3_pert":
        mesh = quad_mesh(4, 4, 3, box=((0, 1), (0, 1)), perturb=0.2, seed=2)
        u, f, g = fields.poisson_sine(mesh)
        pr = configs.Problem(name, mesh, EQ_POISSON, 1, 0 * u, c11_interior=1 / 20, source=f,
                             gD=fields.face_values(mesh, u))
        return pr, 1 / 20
    if name == "quad4p2_pert_neumann":
        base = quad_mesh(4, 4, 2, box=((0, 1), (0, 1)), perturb=0.25, seed=5)
        u, f, g = fields.poisson_sine(base)
        mesh = with_boundary_kinds(base, {1: BC_NEUMANN, 3: BC_NEUMANN})
        pr = configs.Problem(name, mesh, EQ_POISSON, 1, 0 * u, c11_interior=1 / 20, source=f,
                             gD=fields.face_values(mesh, u), gN=-fields.axis_normal_face_values(mesh, g))
        return pr, 1 / 20
    if name == "hex2p2_curved":
        mesh = hex_mesh(2, 2, length=1.0, periodic=False, amp=0.05)
        u, f, g = fields.poisson_polynomial_3d(mesh, degs=(2, 1, 2))
        pr = configs.Problem(name, mesh, EQ_POISSON, 1, 0 * u, c11_interior=1 / 20, source=f,
                             gD=fields.face_values(mesh, u))
        return pr, 1 / 20
    if name == "hex2p2_curved_neumann":
        base = hex_mesh(2, 2, length=1.0, periodic=False, amp=0.05)
        u, f, g = fields.poisson_polynomial_3d(base, degs=(2, 1, 2))
        mesh = with_boundary_kinds(base, {1: BC_NEUMANN, 3: BC_NEUMANN, 5: BC_NEUMANN})
        # the axis-normal gradient as Neumann data (not the exact flux on curved faces; both sides
        # solve the same discrete problem)
        pr = configs.Problem(name, mesh, EQ_POISSON, 1, 0 * u, c11_interior=1 / 20, source=f,
                             gD=fields.face_values(mesh, u), gN=-fields.axis_normal_face_values(mesh, g))
        return pr, 1 / 20
    if name == "quad4p3_pert_c22_0":
        pr, _ = poisson_problem("quad4p3_pert")
        pr.name = name
        return pr, 0.0
    raise KeyError(name)


def oracle_coupled(pr, c22):
    me = pr.mesh
    return LineDG(me.dim, me.p, me.xyz, me.face_nbr, me.nbr_node, me.switch_plus, Physics(EQ_POISSON, me.dim),
                  pr.c11_interior, pr.c11_dirichlet, pr.source, pr.gD, gN=pr.gN, c22=c22)


def coupled_matrix(d):
    E, m, D, Np = d.E, d.m, d.D, d.Np
    nu, nq = E * m * Np, E * m * D * Np

    def F(x):
        R, RQ = solver.coupled_residuals(d, x[:nu].reshape(E, m, Np), x[nu:].reshape(E, m, D, Np))
        return torch.cat([-R.reshape(-1), RQ.reshape(-1)])
    x0 = torch.zeros(nu + nq, dtype=torch.float64)
    return jacfwd(F)(x0), -F(x0)


def gpu_coupled(pr, c22, rtol, kind=None):
    ctx = gpu_of(pr)
    if kind is not None:
        ctx.ldg_set_preconditioner(kind)
    ctx.ldg_set_c22(c22)
    E, Np, D = pr.mesh.n_elem, pr.mesh.np_, pr.mesh.dim
    U = torch.full((E, 1, Np), float("nan"), dtype=torch.float64, device="cuda")
    Q = torch.full((E, 1, D, Np), float("nan"), dtype=torch.float64, device="cuda")
    rep = ctx.ldg_coupled_solve(U, Q, rtol=rtol, inner_rtol=1e-2, restart=60, max_iters=500)
    torch.cuda.synchronize()
    ctx.close()
    return U.cpu(), Q.cpu(), rep


@pytest.mark.parametrize("name,kind", [("quad4p3_pert", None), ("quad4p2_pert_neumann", None),
                                       ("hex2p2_curved", None), ("hex2p2_curved_neumann", None),
                                       ("quad4p3_pert_c22_0", None),
                                       ("quad4p3_pert", LDG_PRECOND_BLOCK_LU)])
def test_coupled_solve_matches_oracle(name, kind):
    print(f"[gpu] coupled solve {name} precond {kind}", flush=True)
    pr, c22 = poisson_problem(name)
    rtol = 1e-10
    Ug, Qg, rep = gpu_coupled(pr, c22, rtol, kind)
    assert rep["relres"] <= rtol
    d = oracle_coupled(pr, c22)
    A, b = coupled_matrix(d)
    x = torch.linalg.solve(A, b)
    xg = torch.cat([Ug.reshape(-1), Qg.reshape(-1)])
    An = A.numpy()
    s = np.linalg.svd(An, compute_uv=False)
    kappa, normA = s[0] / s[-1], s[0]
    n_row = int((An != 0).sum(axis=1).max())
    delta = 2 * n_row * U53
    xn, bn = float(x.norm()), float(b.norm())
    bound = 2 * kappa * (rep["relres"] + delta * normA * float(xg.norm()) / bn + An.shape[0] * U53) * xn
    err = float((xg - x).norm())
    record(name, f"coupled solve (C22 = {c22})", err, bound)
    print(f"  FGMRES {rep['iters']} its ({rep['inner_iters']} inner), relres {rep['relres']:.2e}, kappa {kappa:.2e}",
          flush=True)
    assert err <= bound


def test_coupled_c22_zero_equals_reduced_newton():
    """With C22 = 0 the coupled solution's U is the steady solution of the reduced system (one
    Newton step of alpha = 0, gamma = 1 from zero on the linear problem), and Q = D(U)."""
    print("[gpu] coupled C22 = 0 vs reduced", flush=True)
    pr, _ = poisson_problem("quad4p3_pert")
    Ug, Qg, rep = gpu_coupled(pr, 0.0, 1e-12)
    ctx = gpu_of(pr)
    U = torch.zeros(pr.mesh.n_elem, 1, pr.mesh.np_, dtype=torch.float64, device="cuda")
    r2 = ctx.ldg_newton_step(U, U.clone(), 0.0, 1.0, restart=60, max_iters=2000, rtol=1e-12)
    assert r2["lin_relres"] <= 1e-12
    Q = torch.empty(Qg.shape, dtype=torch.float64, device="cuda")
    ctx.ldg_gradient(U, Q)
    torch.cuda.synchronize()
    ctx.close()
    d = oracle_coupled(pr, 0.0)
    A, b = coupled_matrix(d)
    kappa = float(np.linalg.cond(A.numpy()))
    tol = 4 * kappa * 1e-12
    eu = float((Ug - U.cpu()).abs().max()) / float(U.abs().max())
    eq = float((Qg - Q.cpu()).abs().max()) / float(Q.abs().max())
    record("quad4p3_pert", "coupled C22=0 vs reduced (rel)", max(eu, eq), tol)
    assert eu <= tol and eq <= tol


@pytest.mark.parametrize("neumann", [False, True])
def test_coupled_qp_exactness(neumann):
    """u in Q_p with exact data on rectangles: U = u and Q = grad u with C22 = 1/20."""
    print(f"[gpu] coupled Q_p exactness neumann={neumann}", flush=True)
    p = 3
    base = quad_mesh(3, 3, p, box=((0.2, 1.4), (-0.3, 0.9)))
    u, f, g = fields.poisson_polynomial(base, degs=(p, p - 1))
    mesh = with_boundary_kinds(base, {1: BC_NEUMANN, 3: BC_NEUMANN}) if neumann else base
    gN = -fields.axis_normal_face_values(mesh, g) if neumann else None
    pr = configs.Problem("qp", mesh, EQ_POISSON, 1, 0 * u, c11_interior=1 / 20, source=f,
                         gD=fields.face_values(mesh, u), gN=gN)
    Ug, Qg, rep = gpu_coupled(pr, 1 / 20, 1e-12)
    eu = np.abs(Ug.numpy() - u).max() / np.abs(u).max()
    eq = np.abs(Qg.numpy() - g).max() / np.abs(g).max()
    record("qp_neumann" if neumann else "qp", "coupled Q_p exactness (rel)", max(eu, eq), 1e-8)
    assert eu <= 1e-8 and eq <= 1e-8


def test_coupled_argument_errors():
    print("[gpu] coupled argument errors", flush=True)
    pr, _ = poisson_problem("quad4p3_pert")
    ctx = gpu_of(pr)
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(LDGError):
            ctx.ldg_set_c22(bad)
    U = torch.zeros(pr.mesh.n_elem, 1, pr.mesh.np_, dtype=torch.float64, device="cuda")
    Q = torch.zeros(pr.mesh.n_elem, 1, 2, pr.mesh.np_, dtype=torch.float64, device="cuda")
    with pytest.raises(LDGError):
        ctx.ldg_coupled_solve(U, Q, rtol=0.0)
    with pytest.raises(LDGError):
        ctx.ldg_coupled_solve(U, Q, restart=0)
    with pytest.raises(LDGError):
        ctx.ldg_coupled_solve(U, Q, inner_rtol=1.0)
    with pytest.raises(LDGError):
        ctx.ldg_coupled_solve(U, U)
    ctx.close()
    from tests.gpu_cases import case
    ns = gpu_of(case("ns2d_p2"))
    with pytest.raises(LDGError):
        ns.ldg_set_c22(0.05)
    ns.ldg_set_c22(0.0)
    ns.close()


def test_coupled_c22_improves_q_rates():
    """Section 5.1 (Table poitab1) on the GPU: C11 = C22 = 1/20 gives a smaller q error and a higher
    q convergence rate than C11 = C22 = 0 (perturbed quads, p = 1, 8^2 -> 16^2 -> 32^2; the oracle
    pins the same comparison at 8^2 and 16^2)."""
    print("[gpu] coupled q rates", flush=True)
    err = {}
    for c in (0.0, 1 / 20):
        for n in (8, 16, 32):
            mesh = quad_mesh(n, n, 1, box=((0, 1), (0, 1)), perturb=0.25, seed=3)
            u, f, g = fields.poisson_sine(mesh)
            pr = configs.Problem(f"rates{n}", mesh, EQ_POISSON, 1, 0 * u, c11_interior=c, source=f,
                                 gD=fields.face_values(mesh, u))
            Ug, Qg, rep = gpu_coupled(pr, c, 1e-11)
            err[c, n] = float(np.abs(Qg.numpy() - g).max())
    r0 = [np.log2(err[0.0, n] / err[0.0, 2 * n]) for n in (8, 16)]
    r1 = [np.log2(err[1 / 20, n] / err[1 / 20, 2 * n]) for n in (8, 16)]
    print(f"  |q - grad u| C=0: {[err[0.0, n] for n in (8, 16, 32)]}, rates {r0}", flush=True)
    print(f"  |q - grad u| C=1/20: {[err[1 / 20, n] for n in (8, 16, 32)]}, rates {r1}", flush=True)
    record("rates_p1", "q error ratio C22=1/20 / C22=0 at 32^2", err[1 / 20, 32] / err[0.0, 32], 0.75)
    assert err[1 / 20, 32] < 0.75 * err[0.0, 32]
    assert r1[0] > r0[0] + 0.2 and r1[1] > r0[1]
