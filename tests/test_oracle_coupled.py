"""Pins of the oracle's coupled (U, Q) system with C22 != 0 (Section 4.1; Section 3 eqs.
ldgflux1/2, neumann1/2; Section 5.1 Table poitab1)."""
import numpy as np
import pytest
import torch
from torch.func import jacfwd

from ldg_workloads import BC_NEUMANN, configs, fields, quad_mesh, with_boundary_kinds
from oracle import solver
from oracle.linedg import LineDG
from oracle.physics import EQ_POISSON, Physics


def poisson_dg(mesh, c11=0.0, c22=0.0, kind="sine", neumann=False):
    """LineDG for -Lap u = f on the unit box with exact data (Dirichlet, or Neumann on xi_n = 1)."""
    if kind == "sine":
        u, f, g = fields.poisson_sine(mesh)
    else:
        u, f, g = fields.poisson_polynomial(mesh, degs=(mesh.p, mesh.p - 1))
    gN = None
    if neumann:
        mesh = with_boundary_kinds(mesh, {1: BC_NEUMANN, 3: BC_NEUMANN})
        gN = -fields.axis_normal_face_values(mesh, g)
    d = LineDG(2, mesh.p, mesh.xyz, mesh.face_nbr, mesh.nbr_node, mesh.switch_plus, Physics(EQ_POISSON, 2),
               c11, 10.0, f, fields.face_values(mesh, u), gN=gN, c22=c22)
    return d, u, g


def test_c22_zero_coupled_system_equals_reduced_system():
    """With C22 = 0 the coupled system's solution is the reduced system's (Q = D(U) eliminated),
    solved here by a different route (sparse split matrices)."""
    mesh = quad_mesh(4, 4, 2, box=((0, 1), (0, 1)), perturb=0.2, seed=2)
    d, u, g = poisson_dg(mesh)
    U, Q = solver.coupled_steady_solve(d)
    Ud = solver.steady_direct_solve(d)
    assert float((U - Ud).abs().max()) <= 1e-12 * float(Ud.abs().max())
    assert float((Q - d.gradient(Ud)).abs().max()) <= 1e-11 * float(Q.abs().max())


@pytest.mark.parametrize("neumann", [False, True])
def test_c22_keeps_qp_exactness(neumann):
    """For u in Q_p with its exact data, q = grad u is in Q_p too: every jump of F . n vanishes,
    so the C22 terms do, and the coupled solution is the exact u and grad u at the nodes."""
    mesh = quad_mesh(3, 3, 3, box=((0.2, 1.4), (-0.3, 0.9)), perturb=0.0)
    d, u, g = poisson_dg(mesh, c11=1 / 20, c22=1 / 20, kind="poly", neumann=neumann)
    U, Q = solver.coupled_steady_solve(d)
    assert np.abs(U.numpy() - u).max() <= 1e-10 * np.abs(u).max()
    assert np.abs(Q.numpy() - g).max() <= 1e-9 * np.abs(g).max()


@pytest.mark.parametrize("neumann", [False, True])
def test_c22_is_dissipative(neumann):
    """With Q eliminated, the operator for U has eigenvalues in the right half plane for every
    C22 >= 0 (the stability of LDG with C22 >= 0); the opposite sign convention of the jump gives
    eigenvalues far in the left half plane already at C22 = 0.05 (checked through -C22)."""
    mesh = quad_mesh(3, 3, 2, box=((0, 1), (0, 1)), perturb=0.25, seed=5)
    mins = {}
    for c22 in (0.0, 1 / 20, 1.0, -1 / 20):
        d, _, _ = poisson_dg(mesh, c22=c22, neumann=neumann)
        E, m, D, Np = d.E, d.m, d.D, d.Np
        nu, nq = E * m * Np, E * m * D * Np

        def F(x):
            U = x[:nu].reshape(E, m, Np)
            Q = x[nu:].reshape(E, m, D, Np)
            R, RQ = solver.coupled_residuals(d, U, Q)
            return torch.cat([-R.reshape(-1), RQ.reshape(-1)])
        A = jacfwd(F)(torch.zeros(nu + nq, dtype=torch.float64)).numpy()
        S = A[:nu, :nu] - A[:nu, nu:] @ np.linalg.solve(A[nu:, nu:], A[nu:, :nu])
        mins[c22] = float(np.linalg.eigvals(S).real.min())
    assert mins[0.0] > 0 and mins[1 / 20] > 0 and mins[1.0] > 0
    assert mins[-1 / 20] < 0


def test_c22_improves_q_on_perturbed_meshes():
    """Section 5.1 (Table poitab1): C11 = C22 = 1/20 gives better q than C11 = C22 = 0.  On
    perturbed quads with p = 1 the q error at 16^2 is smaller and converges faster from 8^2."""
    err = {}
    for c in (0.0, 1 / 20):
        for n in (8, 16):
            mesh = quad_mesh(n, n, 1, box=((0, 1), (0, 1)), perturb=0.25, seed=3)
            d, u, g = poisson_dg(mesh, c11=c, c22=c)
            U, Q = solver.coupled_steady_solve(d)
            err[c, n] = float(np.abs(Q.numpy() - g).max())
    rate0 = np.log2(err[0.0, 8] / err[0.0, 16])
    rate1 = np.log2(err[1 / 20, 8] / err[1 / 20, 16])
    assert err[1 / 20, 16] < 0.75 * err[0.0, 16]
    assert rate1 > rate0 + 0.2
