"""Learned per-element preconditioner correction (oracle).

TEST INFRASTRUCTURE ONLY: part of the plain FP64 CPU oracle.

This part is not in the paper; it adds a correction to the element-local
line-pattern preconditioner of Section 4.2 (A~_e, factorised by block
ILU(0)).  Definitions, with Np nodes and m components per element:

* D_b  = the m x m diagonal block of A~_e at node b.
* Features of an element (length Np m^2 + Np m): the D_b divided by
  sigma_e = max |entries of all D_b|, node-major ((b m + i) m + j), followed
  by the element's Newton residual G divided by its max-norm, node-major
  (b m + i); an all-zero residual gives zero features.
* Network: two tanh hidden layers, H1 = tanh(X W1 + b1), H2 = tanh(H1 W2 + b2),
  Y = H2 W3 + b3 with Y read as Np blocks Y_b of size m x m.
* Correction: C_b = Y_b D_b^{-1}.  With z0 = ILU(0)^{-1} r and the element
  defect s = r - A~_e z0, the corrected preconditioner is z = z0 + C s.  C is
  fixed once per Jacobian, so z is linear in r.
* Loss over samples e and probes v_k:  s_k = v_k - A~_e ILU_e^{-1} v_k,
  t_k = D^{-1} s_k (node-wise), rho_k = s_k - A~_e (Y t_k) (node-wise Y),
  L = 1/(n K) sum_e sum_k ||rho_k||^2 / ||v_k||^2.
* Adam (Kingma and Ba) with bias correction.

BF16 emulation rounds to the nearest even bfloat16 (8-bit significand)
wherever the GPU path stores a BF16 operand: the features, the weights and
the hidden activations fed to the next layer.
"""
from __future__ import annotations

import numpy as np
import torch

from .solver import bilu0_apply

DT = torch.float64


# --------------------------------------------------------------------------- bfloat16
def bf16_round(x) -> torch.Tensor:
    """Round to the nearest bfloat16 (ties to even), via float32 bit patterns."""
    t = torch.as_tensor(x, dtype=DT)
    f = t.to(torch.float32).contiguous().numpy().view(np.uint32).astype(np.uint64)
    nan = np.isnan(t.to(torch.float32).numpy())
    lsb = (f >> np.uint64(16)) & np.uint64(1)
    r = ((f + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    r = (r & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    out = torch.from_numpy(r.view(np.float32).copy()).to(DT)
    out[torch.from_numpy(nan)] = float("nan")
    return out.reshape(t.shape)


# --------------------------------------------------------------------------- features
def diag_blocks(At: torch.Tensor) -> torch.Tensor:
    """D[e, b] = A~_e[b, :, b, :] from the dense [E, Np, m, Np, m] form."""
    Np = At.shape[1]
    return torch.stack([At[:, b, :, b, :] for b in range(Np)], 1)


def features(At: torch.Tensor, G: torch.Tensor):
    """Network inputs X [E, Np m^2 + Np m], D^{-1} [E, Np, m, m] and the scales."""
    E, Np, m = At.shape[0], At.shape[1], At.shape[2]
    Db = diag_blocks(At)
    sig = Db.abs().reshape(E, -1).amax(1)
    sig = torch.where(sig > 0, sig, torch.ones_like(sig))
    g = torch.as_tensor(G, dtype=DT).reshape(E, m, Np).permute(0, 2, 1).reshape(E, Np * m)
    rn = g.abs().amax(1)
    gfeat = torch.where(rn[:, None] > 0, g / torch.where(rn > 0, rn, torch.ones_like(rn))[:, None],
                        torch.zeros_like(g))
    X = torch.cat([(Db / sig[:, None, None, None]).reshape(E, Np * m * m), gfeat], 1)
    return X, torch.linalg.inv(Db), sig


# --------------------------------------------------------------------------- network
def param_shapes(n_in: int, n_hidden: int, n_out: int):
    return [("W1", (n_in, n_hidden)), ("b1", (n_hidden,)), ("W2", (n_hidden, n_hidden)), ("b2", (n_hidden,)),
            ("W3", (n_hidden, n_out)), ("b3", (n_out,))]


def unflatten(flat, n_in, n_hidden, n_out):
    flat = torch.as_tensor(flat, dtype=DT).reshape(-1)
    out, o = {}, 0
    for k, shp in param_shapes(n_in, n_hidden, n_out):
        n = int(np.prod(shp))
        out[k] = flat[o:o + n].reshape(shp)
        o += n
    assert o == flat.numel()
    return out


def flatten(P):
    return torch.cat([P[k].reshape(-1) for k in ("W1", "b1", "W2", "b2", "W3", "b3")])


def mlp_forward(P, X, bf16=False):
    """Y and the cache for the backward pass; bf16 emulates the GPU's BF16 operands."""
    rnd = bf16_round if bf16 else (lambda a: a)
    X = torch.as_tensor(X, dtype=DT)
    Xr = rnd(X)
    W1, W2, W3 = rnd(P["W1"]), rnd(P["W2"]), rnd(P["W3"])
    H1 = torch.tanh(Xr @ W1 + P["b1"])
    H1r = rnd(H1)
    H2 = torch.tanh(H1r @ W2 + P["b2"])
    H2r = rnd(H2)
    Y = H2r @ W3 + P["b3"]
    return Y, dict(Xr=Xr, H1=H1, H1r=H1r, H2=H2, H2r=H2r, W1=W1, W2=W2, W3=W3, bf16=bf16)


def mlp_backward(cache, dY):
    """Gradients of sum(dY * Y) with respect to every parameter (chain rule, layer by layer)."""
    rnd = bf16_round if cache["bf16"] else (lambda a: a)
    dYr = rnd(dY)
    g = {"W3": cache["H2r"].T @ dYr, "b3": dY.sum(0)}
    dA2 = (dYr @ cache["W3"].T) * (1.0 - cache["H2"] ** 2)
    dA2r = rnd(dA2)
    g["W2"] = cache["H1r"].T @ dA2r
    g["b2"] = dA2.sum(0)
    dA1 = (dA2r @ cache["W2"].T) * (1.0 - cache["H1"] ** 2)
    g["W1"] = cache["Xr"].T @ rnd(dA1)
    g["b1"] = dA1.sum(0)
    return g


# --------------------------------------------------------------------------- loss
def probe_defects(Ae, F, pat, Dinv, V):
    """s = v - A~ ILU^{-1} v and t = D^{-1} s for probes V [n, K, m, Np], scaled by 1/||v||.

    Ae: dense [n, Np, m, Np, m]; F: ILU(0) factors of Ae.  Returns s, t as
    [n, K, Np, m] (node-major).
    """
    n, K = V.shape[0], V.shape[1]
    Np, m = Ae.shape[1], Ae.shape[2]
    Ad = Ae.reshape(n, Np * m, Np * m)
    S = torch.zeros(n, K, Np, m, dtype=DT)
    T = torch.zeros(n, K, Np, m, dtype=DT)
    for k in range(K):
        v = V[:, k]
        z0 = bilu0_apply(F, pat, v)  # [n, m, Np]
        vn = v.permute(0, 2, 1).reshape(n, Np * m)
        zn = z0.permute(0, 2, 1).reshape(n, Np * m, 1)
        s = (vn - (Ad @ zn)[..., 0]) / torch.linalg.norm(vn, dim=1, keepdim=True)
        S[:, k] = s.reshape(n, Np, m)
        T[:, k] = (Dinv @ S[:, k, :, :, None])[..., 0]
    return S, T


def correction_loss(Y, Ae, S, T):
    """Loss and dL/dY for outputs Y [n, Np m^2]; Ae dense [n, Np, m, Np, m]."""
    n, K, Np, m = S.shape
    Ad = Ae.reshape(n, Np * m, Np * m)
    Yb = Y.reshape(n, Np, m, m)
    L = torch.zeros((), dtype=DT)
    dY = torch.zeros(n, Np, m, m, dtype=DT)
    for k in range(K):
        c = (Yb @ T[:, k, :, :, None])[..., 0].reshape(n, Np * m, 1)
        rho = S[:, k].reshape(n, Np * m) - (Ad @ c)[..., 0]
        L = L + (rho ** 2).sum()
        g = -2.0 * (Ad.transpose(1, 2) @ rho[..., None])[..., 0].reshape(n, Np, m)
        dY += g[..., :, None] * T[:, k, :, None, :]
    scale = 1.0 / (n * K)
    return L * scale, (dY * scale).reshape(n, Np * m * m)


def loss_and_grad(P, X, Ae, S, T, bf16=False):
    Y, cache = mlp_forward(P, X, bf16)
    L, dY = correction_loss(Y, Ae, S, T)
    return L, mlp_backward(cache, dY), Y


def adam_step(w, g, m1, m2, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam update; returns (w, m1, m2)."""
    m1 = b1 * m1 + (1 - b1) * g
    m2 = b2 * m2 + (1 - b2) * g * g
    mh = m1 / (1 - b1 ** step)
    vh = m2 / (1 - b2 ** step)
    return w - lr * mh / (torch.sqrt(vh) + eps), m1, m2


# --------------------------------------------------------------------------- corrected preconditioner
def correction_blocks(Y, Dinv):
    """C_b = Y_b D_b^{-1}; Y [E, Np m^2], Dinv [E, Np, m, m]."""
    E, Np, m = Dinv.shape[0], Dinv.shape[1], Dinv.shape[2]
    return Y.reshape(E, Np, m, m) @ Dinv


def corrected_apply(F, pat, At, C, r):
    """z = z0 + C (r - A~ z0), z0 = ILU(0)^{-1} r; r and z as [E, m, Np]."""
    E, Np, m = At.shape[0], At.shape[1], At.shape[2]
    z0 = bilu0_apply(F, pat, r)
    Ad = At.reshape(E, Np * m, Np * m)
    zn = z0.permute(0, 2, 1).reshape(E, Np * m, 1)
    s = r.reshape(E, m, Np).permute(0, 2, 1).reshape(E, Np * m) - (Ad @ zn)[..., 0]
    cs = (C @ s.reshape(E, Np, m, 1))[..., 0]
    return z0 + cs.permute(0, 2, 1)
