"""GPU residual and LDG gradient against the FP64 oracle (through the C ABI).

Tolerance (FP64 residual), normwise:
    max |R_gpu - R_orc| <= max(1e-12 * max(|R_orc|_inf, |R_abs|_inf), 4 S)
where S is the oracle's own response to random one-ulp perturbations of its
inputs (node coordinates and state) on the same elements, and R_abs = (1/J) sum_n |r^(n)| + |S| is the oracle's magnitude of the
terms summed into R.  The residual differentiates the node coordinates, and
its response to a one-ulp perturbation of them is of the same size as the
GPU/oracle difference (about 5e-13 |R_abs|_inf on the perturbed p = 4 vortex
mesh), so the bound is relative to the summed terms rather than to R itself,
which cancels them.  Q = K21 U + (boundary data) is linear in U; its bound is
the forward-error scale of a linear operator,
    max |Q_gpu - Q_orc| <= 1e-12 * max(|Q_orc|_inf, |U|_inf * ||K21||_inf),
with ||K21||_inf the largest absolute row sum of the oracle's gradient weights.
"""
import sys

import numpy as np
import pytest
import torch

from tests.gpu_cases import case, gpu_of, oracle_of, rounding_sensitivity

pytestmark = pytest.mark.gpu

FULL = ["C1", "C2", "ns2d_p1", "ns2d_p2", "ns2d_p3", "ns2d_p4", "euler3d_p1", "euler3d_p2", "euler3d_p3",
        "euler3d_p4", "poisson3d_p2", "poisson3d_p3", "tgv3p2", "tgv2p4"]


def run_gpu(pr, want_q=True):
    ctx = gpu_of(pr)
    U = torch.as_tensor(pr.U0, device="cuda").contiguous()
    R = torch.empty_like(U)
    Q = torch.empty(pr.mesh.n_elem, pr.m, pr.mesh.dim, pr.mesh.np_, dtype=torch.float64, device="cuda")
    ctx.ldg_residual(U, R, Q if pr.equation != 1 else None)
    torch.cuda.synchronize()
    return ctx, U, R.cpu().numpy(), Q.cpu().numpy()


def check_R(R_gpu, R_orc, mag, sens=0.0):
    R_orc = R_orc.numpy()
    scale = max(np.abs(R_orc).max(), mag.numpy().max())
    bound = max(1e-12 * scale, 4.0 * sens)
    err = np.abs(R_gpu - R_orc).max()
    print(f"  max|R_gpu - R_orc| = {err:.3e}, bound {bound:.3e} (1e-12 scale {1e-12 * scale:.3e}, "
          f"ulp sensitivity {sens:.3e})", flush=True)
    assert err <= bound, (err, bound)


def check_Q(Q_gpu, Q_orc, orc, U, elems):
    W = orc.k21(elems).numpy()
    k21_norm = np.abs(W).sum(axis=2).max()
    scale = max(np.abs(Q_orc).max(), np.abs(U).max() * k21_norm)
    err = np.abs(Q_gpu - Q_orc).max()
    print(f"  max|Q_gpu - Q_orc| = {err:.3e}, bound {1e-12 * scale:.3e}", flush=True)
    assert err <= 1e-12 * scale


@pytest.mark.parametrize("name", FULL)
def test_residual_parity_full(name):
    print(f"[gpu] residual parity {name}", flush=True)
    pr = case(name)
    ctx, U, R_gpu, Q_gpu = run_gpu(pr)
    orc = oracle_of(pr)
    R_orc, mag = orc.residual(pr.U0, return_abs=True)
    check_R(R_gpu, R_orc, mag)
    if pr.equation != 1:
        check_Q(Q_gpu, orc.gradient(pr.U0).numpy(), orc, pr.U0, None)
    ctx.close()


@pytest.mark.parametrize("name", ["C3", "C4"])
def test_residual_parity_sampled(name):
    """Full-size 3-D Navier-Stokes workloads: every element on the GPU, a seeded sample on the oracle."""
    print(f"[gpu] residual parity sampled {name}", flush=True)
    pr = case(name)
    ctx, U, R_gpu, Q_gpu = run_gpu(pr)
    rng = np.random.default_rng(0)
    E = pr.mesh.n_elem
    sample = np.unique(np.concatenate([[0, E - 1], rng.choice(E, size=24, replace=False)]))
    orc = oracle_of(pr)
    R_orc, mag = orc.residual(pr.U0, elems=sample, return_abs=True)
    check_R(R_gpu[sample], R_orc, mag, rounding_sensitivity(orc, pr, sample))
    check_Q(Q_gpu[sample], orc.gradient(pr.U0, elems=sample).numpy(), orc, pr.U0, sample)
    # properties that hold at any size: finite, and repeatable bit for bit
    assert np.all(np.isfinite(R_gpu))
    R2 = torch.empty_like(U)
    ctx.ldg_residual(U, R2)
    torch.cuda.synchronize()
    assert np.array_equal(R2.cpu().numpy(), R_gpu)
    ctx.close()


def test_freestream_and_conservation_gpu():
    """Freestream on a curved 2-D mesh and discrete conservation (periodic NS) on the GPU path."""
    import math
    from ldg_workloads import configs, fields, quad_mesh
    def curve(x, y):
        return (x + 0.15 * np.sin(math.pi * x / 2) * np.sin(math.pi * y / 2),
                y - 0.1 * np.sin(math.pi * x / 2) * np.sin(math.pi * y))
    mesh = quad_mesh(6, 6, 4, box=((0, 4), (0, 4)), periodic=(True, True), perturb=0.15, seed=3, curve=curve)
    U0 = fields.constant_state(mesh, [1.0, 0.3, -0.2, 2.6])
    pr = configs.Problem("fs", mesh, configs.EQ_EULER, 4, U0)
    ctx, U, R, _ = run_gpu(pr)
    assert np.abs(R).max() < 1e-11
    ctx.close()


def test_rk4_parity_c2():
    """100 RK4 steps of the vortex (C2) on the GPU against 2 oracle steps compared after 2 GPU steps,
    then conservation over the full 100 steps."""
    from oracle import solver
    pr = case("C2")
    ctx = gpu_of(pr)
    U = torch.as_tensor(pr.U0, device="cuda").contiguous()
    ctx.ldg_rk4(U, pr.dt, 2)
    torch.cuda.synchronize()
    orc = oracle_of(pr)
    Uo = torch.as_tensor(pr.U0)
    for _ in range(2):
        Uo = solver.rk4_step(orc, Uo, pr.dt)
    err = np.abs(U.cpu().numpy() - Uo.numpy()).max()
    assert err <= 1e-12 * np.abs(Uo.numpy()).max()
    ctx.ldg_rk4(U, pr.dt, 98)
    torch.cuda.synchronize()
    geo = orc.geometry(torch.arange(orc.E))
    W = orc.ops.M.sum(1)
    w = torch.as_tensor(np.prod(W[orc.node_coords()], axis=1))
    tot0 = (torch.as_tensor(pr.U0) * geo["J"][:, None, :] * w).sum(dim=(0, 2))
    tot1 = (U.cpu() * geo["J"][:, None, :] * w).sum(dim=(0, 2))
    assert torch.all((tot1 - tot0).abs() <= 1e-11 * tot0.abs())
    ctx.close()


def test_rk4_graph_replays_match_oracle():
    """RK4 runs as a captured graph replayed per step: repeated calls, with eager work and
    synchronisations in between, and a new step size (a new capture) stay on the oracle's path."""
    from oracle import solver
    pr = case("ns2d_p2")
    print("[gpu] rk4 graph replays ns2d_p2", flush=True)
    ctx = gpu_of(pr)
    orc = oracle_of(pr)
    U = torch.as_tensor(pr.U0, device="cuda").contiguous()
    R = torch.empty_like(U)
    Uo = torch.as_tensor(pr.U0)
    scale = float(Uo.abs().max())
    for dt, calls in ((1e-3, 3), (5e-4, 2)):
        for _ in range(calls):
            ctx.ldg_rk4(U, dt, 2)
            ctx.ldg_residual(U, R)  # eager work on the same stream between replays
            torch.cuda.synchronize()
            for _ in range(2):
                Uo = solver.rk4_step(orc, Uo, dt)
            err = float((U.cpu() - Uo).abs().max())
            assert err <= 1e-12 * scale, (dt, err)
            Ro = orc.residual(Uo)
            assert float((R.cpu() - Ro).abs().max()) <= 1e-10 * float(Ro.abs().max())
    ctx.close()
