"""Pins for the oracle's learned preconditioner correction (network, loss, Adam, corrected apply)."""
import numpy as np
import pytest
import torch

from oracle import learned as LN
from oracle import solver
from tests.gpu_cases import oracle_of, small_ns_2d

DT = torch.float64


def small_system(p=1, n=2, seed=0):
    pr = small_ns_2d(p=p, n=n, seed=seed)
    d = oracle_of(pr)
    U = torch.as_tensor(pr.U0).reshape(d.E, d.m, d.Np)
    K11, K12, K21 = d.jacobian(U)
    At = solver.precond_matrix(d, K11, K12, K21, gamma=0.05, alpha=1.0)
    pat = solver.line_pattern(d)
    F = solver.bilu0(At, pat)
    G = -0.05 * d.residual(U)
    return d, At, pat, F, G


def random_params(n_in, n_hidden, n_out, seed, scale=0.3):
    g = torch.Generator().manual_seed(seed)
    return {k: scale * torch.randn(shp, generator=g, dtype=DT) for k, shp in LN.param_shapes(n_in, n_hidden, n_out)}


# ------------------------------------------------------------------ bfloat16 rounding
def test_bf16_round_known_values():
    x = torch.tensor([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -8 + 2 ** -20, -2.5, 1.0 / 3.0, 0.0, -0.0])
    want = torch.tensor([1.0, 1.0, 1 + 2 ** -6, 1 + 2 ** -7, -2.5, 0.333984375, 0.0, -0.0], dtype=DT)
    got = LN.bf16_round(x)
    assert torch.equal(got, want)
    assert torch.isnan(LN.bf16_round(torch.tensor([float("nan")])))[0]
    # unit roundoff of an 8-bit significand: relative error at most 2^-8
    y = torch.randn(10000, dtype=DT) * 10
    assert float(((LN.bf16_round(y) - y).abs() / y.abs()).max()) <= 2 ** -8


# ------------------------------------------------------------------ features
def test_features_layout_and_scale_invariance():
    d, At, pat, F, G = small_system()
    X, Dinv, sig = LN.features(At, G)
    E, Np, m = d.E, d.Np, d.m
    assert X.shape == (E, Np * m * m + Np * m)
    # block part: node-major D_b / sigma, max-norm one per element
    for e in range(E):
        for b in range(Np):
            blk = X[e, b * m * m:(b + 1) * m * m].reshape(m, m)
            assert torch.allclose(blk * sig[e], At[e, b, :, b, :], rtol=1e-15, atol=0)
            assert torch.allclose(Dinv[e, b] @ At[e, b, :, b, :], torch.eye(m, dtype=DT), atol=1e-12)
    assert torch.allclose(X[:, :Np * m * m].abs().amax(1), torch.ones(E, dtype=DT))
    gpart = X[:, Np * m * m:]
    assert torch.allclose(gpart.abs().amax(1), torch.ones(E, dtype=DT))
    g = torch.as_tensor(G).reshape(E, m, Np)
    assert torch.allclose(gpart.reshape(E, Np, m).permute(0, 2, 1) * g.abs().reshape(E, -1).amax(1)[:, None, None], g,
                          rtol=1e-14, atol=0)
    # scaling A~ by 3 and G by 1e-4 leaves the features unchanged and scales D^{-1} by 1/3
    X2, Dinv2, _ = LN.features(3.0 * At, 1e-4 * torch.as_tensor(G))
    assert torch.allclose(X2, X, rtol=1e-14, atol=1e-15)
    assert torch.allclose(Dinv2 * 3.0, Dinv, rtol=1e-13, atol=0)
    # a zero residual gives zero residual features
    X3, _, _ = LN.features(At, torch.zeros_like(torch.as_tensor(G)))
    assert torch.all(X3[:, Np * m * m:] == 0)


# ------------------------------------------------------------------ gradient vs finite differences
@pytest.mark.parametrize("bf16", [False])
def test_mlp_loss_gradient_matches_central_differences(bf16):
    d, At, pat, F, G = small_system()
    X, Dinv, _ = LN.features(At, G)
    n_in, n_out, H = X.shape[1], d.Np * d.m * d.m, 6
    P = random_params(n_in, H, n_out, seed=1)
    V = torch.randn(d.E, 2, d.m, d.Np, generator=torch.Generator().manual_seed(2), dtype=DT)
    S, T = LN.probe_defects(At, F, pat, Dinv, V)
    L0, grads, _ = LN.loss_and_grad(P, X, At, S, T, bf16=bf16)
    rng = np.random.default_rng(3)
    for k, shp in LN.param_shapes(n_in, H, n_out):
        flat = P[k].reshape(-1)
        for idx in rng.choice(flat.numel(), size=min(12, flat.numel()), replace=False):
            h = 1e-6 * max(1.0, abs(float(flat[idx])))
            Pp = {kk: v.clone() for kk, v in P.items()}
            Pm = {kk: v.clone() for kk, v in P.items()}
            Pp[k].reshape(-1)[idx] += h
            Pm[k].reshape(-1)[idx] -= h
            Lp = LN.loss_and_grad(Pp, X, At, S, T)[0]
            Lm = LN.loss_and_grad(Pm, X, At, S, T)[0]
            fd = float(Lp - Lm) / (2 * h)
            an = float(grads[k].reshape(-1)[idx])
            assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * float(L0)), (k, idx, fd, an)


def test_output_gradient_matches_central_differences():
    """dL/dY of the correction loss alone, against central differences in Y."""
    d, At, pat, F, G = small_system()
    _, Dinv, _ = LN.features(At, G)
    V = torch.randn(d.E, 3, d.m, d.Np, generator=torch.Generator().manual_seed(5), dtype=DT)
    S, T = LN.probe_defects(At, F, pat, Dinv, V)
    Y = 0.2 * torch.randn(d.E, d.Np * d.m * d.m, generator=torch.Generator().manual_seed(6), dtype=DT)
    L, dY = LN.correction_loss(Y, At, S, T)
    for idx in np.random.default_rng(7).choice(Y.numel(), 20, replace=False):
        h = 1e-6
        Yp, Ym = Y.clone(), Y.clone()
        Yp.reshape(-1)[idx] += h
        Ym.reshape(-1)[idx] -= h
        fd = float(LN.correction_loss(Yp, At, S, T)[0] - LN.correction_loss(Ym, At, S, T)[0]) / (2 * h)
        assert abs(fd - float(dY.reshape(-1)[idx])) <= 1e-6 * max(abs(fd), 1e-3 * float(L))


# ------------------------------------------------------------------ special cases of the correction
def test_zero_output_is_plain_ilu_and_loss_is_defect_norm():
    d, At, pat, F, G = small_system()
    _, Dinv, _ = LN.features(At, G)
    E, Np, m = d.E, d.Np, d.m
    C = LN.correction_blocks(torch.zeros(E, Np * m * m, dtype=DT), Dinv)
    r = torch.randn(E, m, Np, generator=torch.Generator().manual_seed(1), dtype=DT)
    assert torch.equal(LN.corrected_apply(F, pat, At, C, r), solver.bilu0_apply(F, pat, r))
    V = torch.randn(E, 2, m, Np, generator=torch.Generator().manual_seed(2), dtype=DT)
    S, T = LN.probe_defects(At, F, pat, Dinv, V)
    L, _ = LN.correction_loss(torch.zeros(E, Np * m * m, dtype=DT), At, S, T)
    assert abs(float(L) - float((S ** 2).sum()) / (E * 2)) <= 1e-15 * float(L)
    # ILU(0) on this 2-D p=1 pattern drops fill, so the defect is not zero
    assert float(L) > 1e-8


def test_identity_output_is_one_block_jacobi_sweep():
    """Y_b = I gives C_b = D_b^{-1}: z = z0 + D^{-1}(r - A~ z0), one block-Jacobi sweep from z0."""
    d, At, pat, F, G = small_system(p=2)
    _, Dinv, _ = LN.features(At, G)
    E, Np, m = d.E, d.Np, d.m
    Y = torch.eye(m, dtype=DT).repeat(E, Np, 1, 1).reshape(E, -1)
    C = LN.correction_blocks(Y, Dinv)
    r = torch.randn(E, m, Np, generator=torch.Generator().manual_seed(3), dtype=DT)
    z = LN.corrected_apply(F, pat, At, C, r)
    z0 = solver.bilu0_apply(F, pat, r)
    for e in range(E):
        A = At[e].reshape(Np * m, Np * m)
        res = (r[e].T.reshape(-1) - A @ z0[e].T.reshape(-1)).reshape(Np, m)
        for b in range(Np):
            step = torch.linalg.solve(At[e, b, :, b, :], res[b])
            assert torch.allclose(z[e, :, b], z0[e, :, b] + step, rtol=1e-12, atol=1e-13)


def test_corrected_apply_is_linear_in_r():
    d, At, pat, F, G = small_system()
    X, Dinv, _ = LN.features(At, G)
    P = random_params(X.shape[1], 5, d.Np * d.m * d.m, seed=4)
    Y, _ = LN.mlp_forward(P, X)
    C = LN.correction_blocks(Y, Dinv)
    g = torch.Generator().manual_seed(9)
    r1 = torch.randn(d.E, d.m, d.Np, generator=g, dtype=DT)
    r2 = torch.randn(d.E, d.m, d.Np, generator=g, dtype=DT)
    lhs = LN.corrected_apply(F, pat, At, C, 2.0 * r1 - 0.5 * r2)
    rhs = 2.0 * LN.corrected_apply(F, pat, At, C, r1) - 0.5 * LN.corrected_apply(F, pat, At, C, r2)
    assert torch.allclose(lhs, rhs, rtol=1e-12, atol=1e-12)


# ------------------------------------------------------------------ Adam and training
def test_adam_first_step_closed_form():
    """From zero moments, step 1 moves each weight by lr g / (|g| + eps)."""
    w = torch.randn(50, dtype=DT)
    g = torch.randn(50, dtype=DT)
    w1, m1, m2 = LN.adam_step(w, g, torch.zeros(50, dtype=DT), torch.zeros(50, dtype=DT), 1, lr=1e-2)
    assert torch.allclose(w1, w - 1e-2 * g / (g.abs() + 1e-8), rtol=0, atol=1e-15)
    assert torch.allclose(m1, 0.1 * g) and torch.allclose(m2, 0.001 * g * g)


def test_training_lowers_the_loss_on_a_fixed_batch():
    d, At, pat, F, G = small_system(p=2)
    X, Dinv, _ = LN.features(At, G)
    n_in, n_out, H = X.shape[1], d.Np * d.m * d.m, 16
    P = random_params(n_in, H, n_out, seed=5, scale=0.1)
    P["W3"].zero_()
    P["b3"].zero_()
    V = torch.randn(d.E, 2, d.m, d.Np, generator=torch.Generator().manual_seed(6), dtype=DT)
    S, T = LN.probe_defects(At, F, pat, Dinv, V)
    L0 = float(LN.loss_and_grad(P, X, At, S, T)[0])
    m1 = {k: torch.zeros_like(v) for k, v in P.items()}
    m2 = {k: torch.zeros_like(v) for k, v in P.items()}
    for step in range(1, 201):
        L, g, _ = LN.loss_and_grad(P, X, At, S, T)
        for k in P:
            P[k], m1[k], m2[k] = LN.adam_step(P[k], g[k], m1[k], m2[k], step, lr=3e-3)
    assert float(L) < 0.5 * L0


def test_bf16_emulated_gradient_is_the_exact_gradient_within_rounding():
    """The BF16-emulated backward rounds features, weights, hidden activations and activation
    gradients to bfloat16 (relative error at most 2^-9 each).  Its gradients must therefore agree
    with central differences of the exact FP64 loss to within a few such roundings per factor of
    each product (bound 4e-2 of the block's largest entry), while a wrong operand, sign or
    transposition would be off by O(1)."""
    d, At, pat, F, G = small_system()
    X, Dinv, _ = LN.features(At, G)
    n_in, n_out, H = X.shape[1], d.Np * d.m * d.m, 6
    P = random_params(n_in, H, n_out, seed=11)
    V = torch.randn(d.E, 2, d.m, d.Np, generator=torch.Generator().manual_seed(12), dtype=DT)
    S, T = LN.probe_defects(At, F, pat, Dinv, V)
    _, g16, _ = LN.loss_and_grad(P, X, At, S, T, bf16=True)
    rng = np.random.default_rng(13)
    for k, shp in LN.param_shapes(n_in, H, n_out):
        flat = P[k].reshape(-1)
        gk = g16[k].reshape(-1)
        idxs = rng.choice(flat.numel(), size=min(16, flat.numel()), replace=False)
        fds = []
        for idx in idxs:
            h = 1e-6 * max(1.0, abs(float(flat[idx])))
            Pp = {kk: v.clone() for kk, v in P.items()}
            Pm = {kk: v.clone() for kk, v in P.items()}
            Pp[k].reshape(-1)[idx] += h
            Pm[k].reshape(-1)[idx] -= h
            fds.append(float(LN.loss_and_grad(Pp, X, At, S, T)[0] - LN.loss_and_grad(Pm, X, At, S, T)[0]) / (2 * h))
        fds = np.array(fds)
        an = gk[torch.as_tensor(idxs)].numpy()
        scale = max(float(np.abs(fds).max()), 1e-12)
        assert np.abs(an - fds).max() <= 4e-2 * scale, (k, np.abs(an - fds).max(), scale)
