"""GPU learned preconditioner correction against the oracle (network, loss, gradients, samples, apply).

Bounds (written per check below):
* Network output, FP32 mode vs the FP64 oracle: max|Y_gpu - Y_orc| <= 1e-5 max|Y_orc|
  (FP32 accumulation over at most 1920 terms of O(1) products).
* BF16 mode vs the oracle's BF16 emulation (same rounding points): 1e-2 max|Y_orc|
  (FP32 accumulation order can flip a BF16 rounding of an activation by 2^-8).
* Loss and gradients, FP32 mode: loss 1e-5 relative, each parameter block
  max|g_gpu - g_orc| <= 1e-4 max|g_orc|; BF16 mode vs emulation: loss 1e-2, blocks 5e-2.
* Samples: A~ rows rounded to FP32 (2^-24 relative plus the 1e-11 row-relative agreement
  of the FP64 assembly); features 1e-6 absolute (they are at most 1 in size); s and t
  1e-5 relative to the element's largest entry (A~ is applied in FP32).
* Corrected apply (FP32 network, FP32 copy of A~):
  max|z_gpu - z_orc| <= 1e-10 max|z_orc| + 1e-4 max|z_orc - z0_orc| (z0 = plain ILU(0)).
* Adam: one and two steps equal the bias-corrected update of the GPU's own
  gradients to 1e-6 of the learning rate.
"""
import numpy as np
import pytest
import torch

from oracle import learned as LN
from oracle import solver
from paper_1204_1533_amd import LDG_BF16, LDG_F32, Net
from tests.gpu_cases import case, gpu_of, oracle_of

pytestmark = pytest.mark.gpu
DT = torch.float64


def stream():
    return torch.cuda.current_stream().cuda_stream


def flat_params(P):
    return LN.flatten(P).to(torch.float32)


def random_params(n_in, h, n_out, seed, zero_out=False):
    g = torch.Generator().manual_seed(seed)
    P = {}
    for k, shp in LN.param_shapes(n_in, h, n_out):
        fan = shp[0] if len(shp) == 2 else 1
        P[k] = torch.randn(shp, generator=g, dtype=DT) * (1.0 / np.sqrt(fan) if len(shp) == 2 else 0.1)
    if zero_out:
        P["W3"].zero_()
        P["b3"].zero_()
    # parameters as the GPU sees them (FP32)
    return {k: v.to(torch.float32).to(DT) for k, v in P.items()}


def line_rows(orc, At):
    """Dense oracle A~ [E, Np, m, Np, m] -> line-pattern rows [E, Np, Dp+1, m, m] (slot order of ldg.h)."""
    cols = orc.column_nodes("K11")[:, :, :orc.nslot_line]
    E, Np, m = At.shape[0], orc.Np, orc.m
    out = torch.zeros(E, Np, orc.nslot_line, m, m, dtype=DT)
    for a in range(Np):
        for s in range(orc.nslot_line):
            b = int(cols[0, a, s] % Np)
            out[:, a, s] = At[:, a, :, b, :]
    return out


def oracle_system(pr, gamma, alpha=1.0):
    orc = oracle_of(pr)
    O11, O12, O21 = orc.jacobian(pr.U0)
    At = solver.precond_matrix(orc, O11, O12, O21, gamma, alpha)
    pat = solver.line_pattern(orc)
    F = solver.bilu0(At, pat)
    G = -gamma * orc.residual(pr.U0)
    X, Dinv, _ = LN.features(At, G)
    return orc, At, pat, F, X, Dinv


# ------------------------------------------------------------------ network forward
@pytest.mark.parametrize("shape", [(2, 1, 4, 32, 70), (3, 3, 5, 256, 300)])
def test_net_forward_matches_oracle(shape):
    dim, p, m, h, n = shape
    print(f"[gpu] net forward {shape}", flush=True)
    net = Net(dim, p, m, hidden=h, seed=3, stream=stream())
    np_ = (p + 1) ** dim
    n_in, n_out = np_ * m * m + np_ * m, np_ * m * m
    P = random_params(n_in, h, n_out, seed=4)
    assert net.ldg_net_num_params() == sum(int(np.prod(s)) for _, s in LN.param_shapes(n_in, h, n_out))
    net.ldg_net_set_params(flat_params(P).cuda())
    g = torch.Generator().manual_seed(5)
    X = (2 * torch.rand(n, n_in, generator=g, dtype=DT) - 1).to(torch.float32).to(DT)
    for prec, bf16, tol in ((LDG_F32, False, 1e-5), (LDG_BF16, True, 1e-2)):
        Y = torch.empty(n, n_out, device="cuda")
        net.ldg_net_forward(X.float().cuda(), n, prec, Y)
        Yo, _ = LN.mlp_forward(P, X, bf16=bf16)
        err = float((Y.cpu().to(DT) - Yo).abs().max()) / float(Yo.abs().max())
        print(f"  prec {prec}: relative error {err:.2e} (bound {tol:.0e})", flush=True)
        assert err <= tol
    # parameters round-trip
    w = torch.empty(net.ldg_net_num_params(), device="cuda")
    net.ldg_net_get_params(w)
    assert torch.equal(w.cpu(), flat_params(P))
    net.close()


# ------------------------------------------------------------------ samples
@pytest.mark.parametrize("name", ["tgv2p3", "ns2d_p2"])
def test_samples_match_oracle(name):
    print(f"[gpu] learned samples {name}", flush=True)
    pr = case(name)
    gamma = 0.03
    orc, At, pat, F, X, Dinv = oracle_system(pr, gamma)
    E, m, Np = pr.mesh.n_elem, pr.m, pr.mesh.np_
    ctx = gpu_of(pr)
    ctx.ldg_learned_collect(True)
    U = torch.as_tensor(pr.U0, device="cuda").contiguous()
    ctx.ldg_jacobian_assemble(U, 1.0, gamma, 0)
    K = 3
    V = torch.randn(K, E, m, Np, generator=torch.Generator().manual_seed(8), dtype=DT)
    el = np.array(sorted(set(np.random.default_rng(1).choice(E, size=min(E, 6), replace=False))), dtype=np.int64)
    n = len(el)
    nsl = orc.nslot_line
    Xg = torch.empty(n, X.shape[1], device="cuda")
    Ag = torch.empty(n, Np, nsl, m, m, device="cuda")
    Sg = torch.empty(n, K, Np, m, device="cuda")
    Tg = torch.empty(n, K, Np, m, device="cuda")
    ctx.ldg_learned_samples(el, V.cuda(), K, Xg, Ag, Sg, Tg)
    torch.cuda.synchronize()
    Ao = line_rows(orc, At)[el]
    err_a = (Ag.cpu().to(DT) - Ao).abs()
    bound_a = 2.0 ** -24 * Ao.abs() + 1e-11 * Ao.abs().amax(dim=(2, 3, 4), keepdim=True)
    assert torch.all(err_a <= bound_a + 1e-300)
    assert float((Xg.cpu().to(DT) - X[el]).abs().max()) <= 1e-6
    So, To = LN.probe_defects(At[el], F[el], pat, Dinv[el], V.permute(1, 0, 2, 3)[el])
    for Gg, Go, what in ((Sg, So, "s"), (Tg, To, "t")):
        scale = Go.abs().reshape(n, -1).amax(1).clamp_min(1e-30)
        e = ((Gg.cpu().to(DT) - Go).abs().reshape(n, -1).amax(1) / scale).max()
        print(f"  {what}: worst element-relative error {float(e):.2e}", flush=True)
        assert float(e) <= 1e-5, what
    ctx.close()


def oracle_batch(name, gamma=0.03, K=3, seed=11):
    pr = case(name)
    orc, At, pat, F, X, Dinv = oracle_system(pr, gamma)
    E, m, Np = pr.mesh.n_elem, pr.m, pr.mesh.np_
    V = torch.randn(E, K, m, Np, generator=torch.Generator().manual_seed(seed), dtype=DT)
    S, T = LN.probe_defects(At, F, pat, Dinv, V)
    # everything the GPU sees is FP32: round the inputs once and use the rounded values on both sides
    r32 = lambda t: t.to(torch.float32).to(DT)
    return pr, orc, r32(X), r32(At), line_rows(orc, r32(At)), r32(S), r32(T)


# ------------------------------------------------------------------ loss and gradients
@pytest.mark.parametrize("name", ["tgv2p3", "ns2d_p2"])
def test_loss_and_gradients_match_oracle(name):
    print(f"[gpu] learned loss/grad {name}", flush=True)
    pr, orc, X, At, Arows, S, T = oracle_batch(name)
    n, K = X.shape[0], S.shape[1]
    dim, p, m = pr.mesh.dim, pr.mesh.p, pr.m
    h = 48
    net = Net(dim, p, m, hidden=h, seed=2, stream=stream())
    P = random_params(X.shape[1], h, net.n_out, seed=6)
    net.ldg_net_set_params(flat_params(P).cuda())
    dev = [t.float().cuda().contiguous() for t in (X, Arows, S, T)]
    for prec, bf16, tl, tg in ((LDG_F32, False, 1e-5, 1e-4), (LDG_BF16, True, 1e-2, 5e-2)):
        grad = torch.empty(net.ldg_net_num_params(), device="cuda")
        loss = net.ldg_net_loss_grad(*dev, n, K, prec=prec, grad=grad)
        Lo, go, _ = LN.loss_and_grad(P, X, At, S, T, bf16=bf16)
        print(f"  prec {prec}: loss {loss:.6e} oracle {float(Lo):.6e}", flush=True)
        assert abs(loss - float(Lo)) <= tl * abs(float(Lo))
        gg = LN.unflatten(grad.cpu().to(DT), X.shape[1], h, net.n_out)
        for k in go:
            e = float((gg[k] - go[k]).abs().max()) / max(float(go[k].abs().max()), 1e-30)
            print(f"    d{k}: relative error {e:.2e}", flush=True)
            assert e <= tg, k
    net.close()


def test_loss_gradients_large_batch_tiles():
    """A batch spanning several 64-row tiles with a ragged tail (replicated samples), FP32 mode."""
    print("[gpu] learned loss/grad large batch", flush=True)
    pr, orc, X, At, Arows, S, T = oracle_batch("tgv2p3")
    idx = torch.as_tensor(np.random.default_rng(3).integers(0, X.shape[0], size=203))
    X, At, Arows, S, T = X[idx], At[idx], Arows[idx], S[idx], T[idx]
    n, K = X.shape[0], S.shape[1]
    net = Net(3, 3, 5, hidden=256, seed=2, stream=stream())
    P = random_params(X.shape[1], 256, net.n_out, seed=9)
    net.ldg_net_set_params(flat_params(P).cuda())
    grad = torch.empty(net.ldg_net_num_params(), device="cuda")
    loss = net.ldg_net_loss_grad(*[t.float().cuda().contiguous() for t in (X, Arows, S, T)], n, K, prec=LDG_F32,
                                 grad=grad)
    Lo, go, _ = LN.loss_and_grad(P, X, At, S, T)
    assert abs(loss - float(Lo)) <= 1e-5 * abs(float(Lo))
    gg = LN.unflatten(grad.cpu().to(DT), X.shape[1], 256, net.n_out)
    for k in go:
        e = float((gg[k] - go[k]).abs().max()) / max(float(go[k].abs().max()), 1e-30)
        assert e <= 1e-4, (k, e)
    net.close()


def test_adam_steps_follow_the_update_rule():
    print("[gpu] learned adam", flush=True)
    pr, orc, X, At, Arows, S, T = oracle_batch("ns2d_p2")
    n, K = X.shape[0], S.shape[1]
    net = Net(2, 2, 4, hidden=16, seed=4, stream=stream())
    P = random_params(X.shape[1], 16, net.n_out, seed=1)
    w0 = flat_params(P)
    net.ldg_net_set_params(w0.cuda())
    dev = [t.float().cuda().contiguous() for t in (X, Arows, S, T)]
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8
    w = w0.to(DT)
    m1 = torch.zeros_like(w)
    m2 = torch.zeros_like(w)
    for step in (1, 2):
        grad = torch.empty(net.ldg_net_num_params(), device="cuda")
        net.ldg_net_loss_grad(*dev, n, K, prec=LDG_F32, grad=grad)
        net.ldg_net_adam_step(lr)
        g = grad.cpu().to(DT)
        m1 = b1 * m1 + (1 - b1) * g
        m2 = b2 * m2 + (1 - b2) * g * g
        w = w - lr * (m1 / (1 - b1 ** step)) / (torch.sqrt(m2 / (1 - b2 ** step)) + eps)
        wg = torch.empty(net.ldg_net_num_params(), device="cuda")
        net.ldg_net_get_params(wg)
        err = float((wg.cpu().to(DT) - w).abs().max())
        print(f"  step {step}: max deviation {err:.2e} (lr {lr})", flush=True)
        assert err <= 1e-6 * lr + 2e-7 * float(w.abs().max())
    net.close()


# ------------------------------------------------------------------ corrected preconditioner
@pytest.mark.parametrize("name", ["tgv2p3", "ns2d_p2"])
def test_corrected_apply_matches_oracle(name):
    print(f"[gpu] learned apply {name}", flush=True)
    pr = case(name)
    gamma = 0.03
    orc, At, pat, F, X, Dinv = oracle_system(pr, gamma)
    E, m, Np = pr.mesh.n_elem, pr.m, pr.mesh.np_
    h = 64
    net = Net(pr.mesh.dim, pr.mesh.p, m, hidden=h, seed=5, stream=stream())
    P = random_params(X.shape[1], h, net.n_out, seed=12)
    for k in ("W3", "b3"):
        P[k] = (0.3 * P[k]).to(torch.float32).to(DT)
    net.ldg_net_set_params(flat_params(P).cuda())
    ctx = gpu_of(pr)
    ctx.ldg_learned_attach(net, LDG_F32)
    U = torch.as_tensor(pr.U0, device="cuda").contiguous()
    ctx.ldg_jacobian_assemble(U, 1.0, gamma, 0)
    assert ctx.ldg_learned_active() == 1
    r = torch.randn(E, m, Np, generator=torch.Generator().manual_seed(13), dtype=DT)
    z = torch.empty(r.shape, dtype=DT, device="cuda")
    ctx.ldg_precond_apply(r.cuda(), z)
    Yo, _ = LN.mlp_forward(P, X)
    zo = LN.corrected_apply(F, pat, At, LN.correction_blocks(Yo, Dinv), r)
    z0 = solver.bilu0_apply(F, pat, r)
    err = float((z.cpu() - zo).abs().max())
    corr = float((zo - z0).abs().max())
    bound = 1e-10 * float(zo.abs().max()) + 1e-4 * corr
    print(f"  max err {err:.2e}, correction size {corr:.2e}, bound {bound:.2e}", flush=True)
    assert corr > 1e-3 * float(z0.abs().max())  # the correction is not negligible
    assert err <= bound
    ctx.close()
    net.close()


def test_zero_output_and_nonfinite_fallback():
    """A fresh network (zero output layer) reproduces plain ILU(0) exactly; NaN output falls back."""
    print("[gpu] learned zero / fallback", flush=True)
    pr = case("tgv2p3")
    gamma = 0.03
    E, m, Np = pr.mesh.n_elem, pr.m, pr.mesh.np_
    U = torch.as_tensor(pr.U0, device="cuda").contiguous()
    r = torch.randn(E, m, Np, generator=torch.Generator().manual_seed(2), dtype=DT).cuda()
    ref_ctx = gpu_of(pr)
    ref_ctx.ldg_jacobian_assemble(U, 1.0, gamma, 1)
    z_ref = torch.empty_like(r)
    ref_ctx.ldg_precond_apply(r, z_ref)
    net = Net(3, 3, 5, hidden=256, seed=7, stream=stream())
    ctx = gpu_of(pr)
    ctx.ldg_learned_attach(net, LDG_BF16)
    ctx.ldg_jacobian_assemble(U, 1.0, gamma, 1)
    assert ctx.ldg_learned_active() == 1
    z = torch.empty_like(r)
    ctx.ldg_precond_apply(r, z)
    assert torch.equal(z, z_ref)
    # NaN in the output bias: the assembly falls back to ILU(0) and the Newton step reports it
    w = torch.empty(net.ldg_net_num_params(), device="cuda")
    net.ldg_net_get_params(w)
    w[-1] = float("nan")
    net.ldg_net_set_params(w)
    ctx.ldg_jacobian_assemble(U, 1.0, gamma, 1)
    assert ctx.ldg_learned_active() == 0
    ctx.ldg_precond_apply(r, z)
    assert torch.equal(z, z_ref)
    Un = U.clone()
    rep = ctx.ldg_newton_step(Un, U, 1.0, gamma, storage_prec=1, use_learned=1)
    assert rep["fallback_used"] == 1 and rep["converged"] == 1
    ctx.close()
    ref_ctx.close()
    net.close()


def test_harmful_correction_is_rejected_by_the_outcome():
    """A finite but harmful correction (a large constant output bias) makes the corrected solve
    miss the tolerance within the iterations that plain BILU(0) needs; the Newton step then
    repeats the solve with the plain factors, reports the fallback, and gives the plain result."""
    print("[gpu] learned harmful correction fallback", flush=True)
    pr = case("tgv2p3")
    gamma = 0.03
    U = torch.as_tensor(pr.U0, device="cuda").contiguous()
    ref = gpu_of(pr)
    U_ref = U.clone()
    rep0 = ref.ldg_newton_step(U_ref, U, 1.0, gamma, storage_prec=1, max_iters=600, rtol=1e-8)
    n_plain = rep0["gmres_iters"]
    net = Net(3, 3, 5, hidden=64, seed=3, stream=stream())
    w = torch.zeros(net.ldg_net_num_params(), device="cuda")
    w[-net.n_out:] = 50.0
    net.ldg_net_set_params(w)
    ctx = gpu_of(pr)
    ctx.ldg_learned_attach(net, LDG_F32)
    U_l = U.clone()
    rep = ctx.ldg_newton_step(U_l, U, 1.0, gamma, storage_prec=1, use_learned=1, max_iters=n_plain, rtol=1e-8)
    torch.cuda.synchronize()
    print(f"  plain {n_plain} iterations; with the harmful correction: {rep}", flush=True)
    assert rep["fallback_used"] == 1 and rep["converged"] == 1
    assert rep["lin_relres"] <= 1e-8
    err = float((U_l - U_ref).abs().max())
    assert err <= 1e-12 * float((U_ref - U).abs().max())
    assert ctx.ldg_learned_active() == 0
    ctx.close()
    ref.close()
    net.close()


# ------------------------------------------------------------------ what the trained network gains
def test_learned_gain_over_ilu0():
    """Train on solver-generated samples (12^3, p = 3 Navier-Stokes runs, seeds 0-7), then compare
    one BDF2 Newton step with and without the correction on held-out seeds 1000-1003.

    The gain has no oracle (the paper has no learned part): the Newton residual measures the
    error, so both solves must reach the 1e-8 linear tolerance and give the same Newton
    residual, and the corrected preconditioner must need fewer GMRES iterations in total.
    """
    from paper_1204_1533_amd import learned
    print("[gpu] learned gain 12^3", flush=True)
    data = learned.generate(list(range(8)), n=12, steps=4, n_elem=256, n_probe=4, log=False)
    net = Net(3, 3, 5, hidden=256, seed=1, stream=stream())
    hist = learned.train(net, data, iters=1500, batch=256, lr=1e-3, log=False)
    first, last = hist[0], float(np.mean(hist[-100:]))
    print(f"  training loss {first:.4f} -> {last:.4f}", flush=True)
    assert last < 0.2 * first
    rows = learned.evaluate(net, [1000, 1001, 1002, 1003], n=12, log=False)
    tot = {"ilu0": 0, "learned": 0}
    for r in rows:
        a, b = r["ilu0"], r["learned"]
        print(f"  seed {r['seed']} (Re {r['re']:.0f}, M {r['mach']:.2f}): GMRES {a['gmres_iters']} -> "
              f"{b['gmres_iters']}, ||G|| after {a['newton_res_after']:.6e} / {b['newton_res_after']:.6e}", flush=True)
        assert a["lin_relres"] <= 1e-8 and b["lin_relres"] <= 1e-8
        assert b["fallback_used"] == 0
        assert abs(a["newton_res_after"] - b["newton_res_after"]) <= 1e-6 * a["newton_res_after"]
        tot["ilu0"] += a["gmres_iters"]
        tot["learned"] += b["gmres_iters"]
    print(f"  total GMRES iterations: ILU(0) {tot['ilu0']}, learned {tot['learned']}", flush=True)
    assert tot["learned"] < tot["ilu0"]
    net.close()
