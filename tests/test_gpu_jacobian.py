"""GPU Jacobian blocks, split product, BILU(0) and Newton step against the FP64 oracle.

Bounds (written per check below):
* FP64 K11 / K12 blocks, row-normwise: max over a node's block row of
  |K_gpu - K_orc| <= 1e-11 * max over the same row of |K_orc|.
* Stored FP32 / BF16 blocks, elementwise: |K_gpu - K_orc| <= u |K_orc| + 1e-300
  with u = 2^-24 (FP32) and 2^-8 + 2^-24 (BF16, rounded through FP32).
* FP64 BILU(0) factors (diagonal slot = inverse of the U block):
  row-normwise 1e-10.
* Products y = (alpha I - gamma A) x with FP64 blocks and the exact tangent:
  max |y_gpu - y_orc| <= 1e-12 * (|x|_inf + gamma |A|_row |x|_inf) with
  |A|_row the largest absolute row sum of K11 + |K12| |K21|.
* Preconditioner apply (FP64): max |z_gpu - z_orc| <= 1e-10 |z_orc|_inf.
* Newton step: linear residual <= 1e-8 on both sides, and
  |U_gpu - U_orc| / |U| <= 1e-7.
"""
import numpy as np
import pytest
import torch

from oracle import solver
from tests.gpu_cases import case, gpu_of, oracle_of

pytestmark = pytest.mark.gpu

SMALL = ["C1", "ns2d_p1", "ns2d_p2", "ns2d_p3", "euler3d_p2", "poisson3d_p2", "tgv2p2", "tgv2p3"]
PREC = {"f64": 0, "f32": 1, "bf16": 2}


def assemble(pr, alpha, gamma, prec=0):
    ctx = gpu_of(pr)
    U = torch.as_tensor(pr.U0, device="cuda").contiguous()
    ctx.ldg_jacobian_assemble(U, alpha, gamma, prec)
    ns11, ns12, nsf = ctx.nslots()
    E, Np, m, D = pr.mesh.n_elem, pr.mesh.np_, pr.m, pr.mesh.dim
    K11 = torch.empty(E, Np, ns11, m, m, dtype=torch.float64, device="cuda")
    K12 = torch.empty(E, Np, ns12, m, m * D, dtype=torch.float64, device="cuda")
    F = torch.empty(E, Np, nsf, m, m, dtype=torch.float64, device="cuda")
    ctx.ldg_export_operators(K11, K12 if pr.equation != 1 else None, F)
    torch.cuda.synchronize()
    return ctx, U, K11.cpu(), K12.cpu(), F.cpu()


def rownorm_check(Kg, Ko, tol, what):
    err = (Kg - Ko).abs().amax(dim=(2, 3, 4))
    scale = Ko.abs().amax(dim=(2, 3, 4)).clamp_min(1e-300)
    worst = float((err / scale).max())
    print(f"  {what}: worst row-relative error {worst:.3e} (bound {tol:.1e})", flush=True)
    assert worst <= tol, what


@pytest.mark.parametrize("name", SMALL)
def test_jacobian_blocks_fp64(name):
    print(f"[gpu] jacobian fp64 {name}", flush=True)
    pr = case(name)
    ctx, U, K11, K12, F = assemble(pr, 1.0, 0.02)
    orc = oracle_of(pr)
    O11, O12, O21 = orc.jacobian(pr.U0)
    rownorm_check(K11, O11, 1e-11, "K11")
    if pr.equation != 1:
        rownorm_check(K12, O12, 1e-11, "K12")
    ctx.close()


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_jacobian_stored_precision(prec):
    pr = case("ns2d_p3")
    print(f"[gpu] jacobian {prec}", flush=True)
    ctx, U, K11, K12, F = assemble(pr, 1.0, 0.02, PREC[prec])
    orc = oracle_of(pr)
    O11, O12, _ = orc.jacobian(pr.U0)
    u = 2.0 ** -24 if prec == "f32" else 2.0 ** -8 + 2.0 ** -24
    for Kg, Ko in ((K11, O11), (K12, O12)):
        # the FP64 values themselves agree to 1e-11 row-relative; add that slack to the rounding bound
        slack = 1e-11 * Ko.abs().amax(dim=(2, 3, 4), keepdim=True)
        assert torch.all((Kg - Ko).abs() <= u * Ko.abs() + slack + 1e-300)
    ctx.close()


def oracle_factors_in_slots(orc, F_dense):
    """Dense oracle BILU(0) factors -> line-slot layout with inverted diagonal blocks."""
    cols = orc.column_nodes("K11")[:, :, :orc.nslot_line]
    E, Np, m = F_dense.shape[0], orc.Np, orc.m
    out = torch.zeros(E, Np, orc.nslot_line, m, m, dtype=torch.float64)
    for a in range(Np):
        for s in range(orc.nslot_line):
            b = int(cols[0, a, s] % Np)
            blk = F_dense[:, a, :, b, :]
            out[:, a, s] = torch.linalg.inv(blk) if b == a else blk
    return out


@pytest.mark.parametrize("name", ["C1", "ns2d_p2", "ns2d_p3", "euler3d_p2", "tgv2p2"])
def test_precond_factors_and_apply_fp64(name):
    print(f"[gpu] bilu0 {name}", flush=True)
    pr = case(name)
    alpha, gamma = (0.0, 1.0) if name == "C1" else (1.0, 0.02)
    ctx, U, K11, K12, F = assemble(pr, alpha, gamma)
    orc = oracle_of(pr)
    O11, O12, O21 = orc.jacobian(pr.U0)
    At = solver.precond_matrix(orc, O11, O12, O21, gamma, alpha)
    pat = solver.line_pattern(orc)
    Fo = solver.bilu0(At, pat)
    rownorm_check(F, oracle_factors_in_slots(orc, Fo), 1e-10, "BILU(0) factors")
    # apply
    g = torch.Generator().manual_seed(5)
    r = torch.randn(pr.mesh.n_elem, pr.m, pr.mesh.np_, dtype=torch.float64, generator=g)
    z = torch.empty(r.shape, dtype=torch.float64, device="cuda")
    ctx.ldg_precond_apply(r.cuda(), z)
    zo = solver.bilu0_apply(Fo, pat, r)
    err = float((z.cpu() - zo).abs().max())
    assert err <= 1e-10 * float(zo.abs().max()), err
    ctx.close()


@pytest.mark.parametrize("name", ["C1", "ns2d_p3", "euler3d_p2", "tgv2p3", "poisson3d_p2"])
def test_jacvec_fp64_and_exact(name):
    print(f"[gpu] jacvec {name}", flush=True)
    pr = case(name)
    alpha, gamma = 1.0, 0.02
    ctx, U, K11, K12, F = assemble(pr, alpha, gamma)
    orc = oracle_of(pr)
    O11, O12, O21 = orc.jacobian(pr.U0)
    g = torch.Generator().manual_seed(7)
    x = torch.randn(pr.mesh.n_elem, pr.m, pr.mesh.np_, dtype=torch.float64, generator=g)
    yo = solver.split_matvec(orc, O11, O12, x, gamma, alpha)
    # |A| row-sum scale
    a11 = O11.abs().sum(dim=(2, 4)).amax()
    a12 = O12.abs().sum(dim=(2, 4)).amax() * O21.abs().sum(dim=(2, 3)).amax()
    scale = float(x.abs().max()) * (1 + gamma * float(a11 + a12))
    for exact in (False, True):
        y = torch.empty(x.shape, dtype=torch.float64, device="cuda")
        ctx.ldg_jacvec(x.cuda(), y, exact)
        err = float((y.cpu() - yo).abs().max())
        print(f"  exact={exact}: max err {err:.3e}, bound {1e-12 * scale:.3e}", flush=True)
        assert err <= 1e-12 * scale
    ctx.close()


def test_jacvec_not_assembled_and_alias_errors():
    from paper_1204_1533_amd import LDGError
    pr = case("ns2d_p2")
    ctx = gpu_of(pr)
    x = torch.zeros(pr.mesh.n_elem, pr.m, pr.mesh.np_, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(LDGError):
        ctx.ldg_jacvec(x, y)
    with pytest.raises(LDGError):
        ctx.ldg_precond_apply(x, y)
    ctx.ldg_jacobian_assemble(torch.as_tensor(pr.U0, device="cuda").contiguous(), 1.0, 0.01)
    with pytest.raises(LDGError):
        ctx.ldg_jacvec(x, x)
    ctx.close()


@pytest.mark.parametrize("name,prec", [("ns2d_p3", "f64"), ("ns2d_p3", "f32"), ("ns2d_p3", "bf16"),
                                       ("tgv2p3", "f64"), ("tgv2p3", "bf16")])
def test_bdf2_newton_step(name, prec):
    print(f"[gpu] newton {name} {prec}", flush=True)
    pr = case(name)
    dt = 0.02
    gamma = 2 * dt / 3
    ctx = gpu_of(pr)
    U = torch.as_tensor(pr.U0, device="cuda").contiguous()
    Ucomb = U.clone()
    rep = ctx.ldg_newton_step(U, Ucomb, 1.0, gamma, restart=30, max_iters=600, storage_prec=PREC[prec], rtol=1e-8)
    torch.cuda.synchronize()
    print("  report", rep, flush=True)
    assert rep["converged"] == 1 and rep["lin_relres"] <= 1e-8
    orc = oracle_of(pr)
    res = solver.newton_step(orc, pr.U0, pr.U0, gamma, rtol=1e-10, restart=30)
    Uo = res["U"].numpy()
    rel = np.abs(U.cpu().numpy() - Uo).max() / np.abs(Uo).max()
    print(f"  |U_gpu - U_orc|/|U| = {rel:.3e}; G0 gpu {rep['newton_res_before']:.4e} orc {res['G0']:.4e}; "
          f"G1 gpu {rep['newton_res_after']:.4e} orc {res['G1']:.4e}", flush=True)
    assert rel <= 1e-7
    assert abs(rep["newton_res_before"] - res["G0"]) <= 1e-10 * res["G0"]
    ctx.close()


def test_poisson_steady_newton_is_direct_solve():
    pr = case("C1")
    pr.U0 = np.zeros_like(pr.U0)
    ctx = gpu_of(pr)
    U = torch.zeros(pr.U0.shape, dtype=torch.float64, device="cuda")
    rep = ctx.ldg_newton_step(U, None, 0.0, 1.0, restart=50, max_iters=3000, storage_prec=0, rtol=1e-10)
    torch.cuda.synchronize()
    orc = oracle_of(pr)
    Ud = solver.steady_direct_solve(orc).numpy()
    err = np.abs(U.cpu().numpy() - Ud).max()
    print(f"  poisson: iters {rep['gmres_iters']} |U_gpu - U_direct| {err:.3e}", flush=True)
    assert err <= 1e-8 * np.abs(Ud).max()
    # and the discrete solution is close to sin(pi x) sin(pi y)
    assert np.abs(U.cpu().numpy() - pr.extra["u_exact"]).max() < 1e-4
    ctx.close()
