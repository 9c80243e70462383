"""Split matrix-vector product, line-pattern preconditioner, GMRES, Newton, RK4 (oracle).

TEST INFRASTRUCTURE ONLY: part of the plain FP64 CPU oracle.

* Newton system (Section 4.2, eqs. dirkeqn, fulldiscprimal): with
  A = K11 + K12 K21, each Newton step solves (alpha I - gamma A) dU = -G.  For a
  BDF2 step G(U) = U - (4U^n - U^{n-1})/3 - gamma F(U), gamma = 2 dt / 3 and
  alpha = 1; a steady solve uses alpha = 0, gamma = 1.
* Split product (eq. matvecsplit): (alpha I - gamma A) p =
  alpha p - gamma (K11 p + K12 (K21 p)); K21 p is the discrete gradient of p
  with homogeneous boundary data, so A is never formed.
* Preconditioner (Section 4.2): A~ equals A on the element-local line pattern
  (the node-blocks on the D lines through each node) and is zero elsewhere; the
  K12 K21 product is taken over intra-element nodes only.  It is factorised by
  block ILU(0) in natural node order (the paper factorises with a sparse
  direct LU and names ILU as an improvement); a dense per-element LU is the
  exact-block reference.
* GMRES (Saad and Schultz) with right preconditioning, x0 = 0, restart m,
  modified Gram-Schmidt, Givens rotations; stop when ||b - A x|| <= rtol ||b||.
* Classical four-stage Runge-Kutta and the three-stage DIRK with Newton
  stage solves (Section 4.1).
* The coupled (U, Q) system of Section 4.1 (needed when C22 != 0): for a
  linear problem its matrix, formed by forward differentiation, and a dense
  solve.
"""
from __future__ import annotations

import math

import numpy as np
import torch
from torch.func import jacfwd

from .linedg import LineDG, DT


# --------------------------------------------------------------------------- products
def blocks_apply(d: LineDG, K: torch.Tensor, cols: np.ndarray, x: torch.Tensor, width: int) -> torch.Tensor:
    """y[e, :, a] = sum_slot K[e, a, slot] @ x_col(slot); x given as [E, width, Np]."""
    E, Np = d.E, d.Np
    xf = x.reshape(E, width, Np).permute(0, 2, 1).reshape(E * Np, width)
    c = torch.as_tensor(cols)
    valid = (c >= 0)
    xs = xf[torch.where(valid, c, torch.zeros_like(c))]  # [E, Np, nslot, width]
    xs = xs * valid[..., None].to(DT)
    y = torch.einsum("eascw,easw->eca", K, xs)
    return y


def split_matvec(d: LineDG, K11, K12, x, gamma, alpha=1.0, cols11=None, cols12=None):
    """(alpha I - gamma (K11 + K12 K21)) x with K21 x = D(x) at g_D = 0."""
    if cols11 is None:
        cols11 = d.column_nodes("K11")
    if cols12 is None:
        cols12 = d.column_nodes("K12")
    x = torch.as_tensor(x, dtype=DT).reshape(d.E, d.m, d.Np)
    w = d.gradient(x, homogeneous=True)  # [E, m, D, Np]
    y11 = blocks_apply(d, K11, cols11, x, d.m)
    y12 = blocks_apply(d, K12, cols12, w.reshape(d.E, d.m * d.D, d.Np), d.m * d.D)
    return alpha * x - gamma * (y11 + y12)


# --------------------------------------------------------------------------- preconditioner
def line_pattern(d: LineDG) -> np.ndarray:
    """pat[a, b] = True when node b lies on one of the D lines through node a."""
    co = d.node_coords()
    diff = (co[:, None, :] != co[None, :, :]).sum(-1)
    return diff <= 1


def precond_matrix(d: LineDG, K11, K12, K21, gamma, alpha=1.0) -> torch.Tensor:
    """Dense per-element A~_e = alpha I - gamma (K11_ee + K12_ee K21_ee) on the line pattern.

    Returns [E, Np, m, Np, m] (zero outside the pattern).
    """
    E, Np, m, D = K11.shape[0], d.Np, d.m, d.D
    c11 = d.column_nodes("K11")
    c12 = d.column_nodes("K12")
    c21 = d.column_nodes("K21")
    own = (np.arange(E) * Np)[:, None, None]
    A11 = torch.zeros(E, Np, m, Np, m, dtype=DT)
    A12 = torch.zeros(E, Np, m, Np, m * D, dtype=DT)
    A21 = torch.zeros(E, Np, m * D, Np, m, dtype=DT)
    eye_m = torch.eye(m, dtype=DT)
    for e in range(E):
        for a in range(Np):
            for s in range(c11.shape[2]):
                g = c11[e, a, s] - own[e, 0, 0]
                if c11[e, a, s] >= 0 and 0 <= g < Np and c11[e, a, s] // Np == e:
                    A11[e, a, :, g, :] += K11[e, a, s]
            for s in range(c12.shape[2]):
                g = c12[e, a, s] - own[e, 0, 0]
                if c12[e, a, s] >= 0 and c12[e, a, s] // Np == e:
                    A12[e, a, :, g, :] += K12[e, a, s]
            for s in range(c21.shape[2]):
                g = c21[e, a, s] - own[e, 0, 0]
                if c21[e, a, s] >= 0 and c21[e, a, s] // Np == e:
                    # rows (c, d) of Q, column component c: weight w_d
                    blk = torch.zeros(m * D, m, dtype=DT)
                    for c in range(m):
                        for dd in range(D):
                            blk[c * D + dd, c] = K21[e, a, s, dd]
                    A21[e, a, :, g, :] += blk
    prod = torch.einsum("eaibk,ebkcj->eaicj", A12, A21)
    A = -gamma * (A11 + prod)
    A = A + alpha * torch.einsum("ab,ij->aibj", torch.eye(Np, dtype=DT), eye_m)[None]
    pat = torch.as_tensor(line_pattern(d))
    return A * pat[None, :, None, :, None].to(DT)


def bilu0(Ae: torch.Tensor, pat: np.ndarray) -> torch.Tensor:
    """Block ILU(0) of A~ (natural order, pattern ``pat``); returns L\\U in place form.

    The strictly lower blocks hold L (unit block diagonal implied), the rest U.
    """
    F = Ae.clone()
    Np = F.shape[1]
    for i in range(1, Np):
        for k in range(i):
            if not pat[i, k]:
                continue
            F[:, i, :, k, :] = F[:, i, :, k, :] @ torch.linalg.inv(F[:, k, :, k, :])
            for j in range(k + 1, Np):
                if pat[i, j] and pat[k, j]:
                    F[:, i, :, j, :] -= F[:, i, :, k, :] @ F[:, k, :, j, :]
    return F


def bilu0_apply(F: torch.Tensor, pat: np.ndarray, r: torch.Tensor) -> torch.Tensor:
    """z = (LU)^{-1} r for every element; r given as [E, m, Np]."""
    E, Np, m = F.shape[0], F.shape[1], F.shape[2]
    rr = r.reshape(E, m, Np).permute(0, 2, 1)  # [E, Np, m]
    y = torch.zeros_like(rr)
    for i in range(Np):
        acc = rr[:, i].clone()
        for k in range(i):
            if pat[i, k]:
                acc -= (F[:, i, :, k, :] @ y[:, k, :, None])[..., 0]
        y[:, i] = acc
    z = torch.zeros_like(rr)
    for i in reversed(range(Np)):
        acc = y[:, i].clone()
        for j in range(i + 1, Np):
            if pat[i, j]:
                acc -= (F[:, i, :, j, :] @ z[:, j, :, None])[..., 0]
        z[:, i] = torch.linalg.solve(F[:, i, :, i, :], acc)
    return z.permute(0, 2, 1)


def dense_block_solve(Ae: torch.Tensor, r: torch.Tensor) -> torch.Tensor:
    """Exact per-element solve with A~_e (the exact-block reference)."""
    E, Np, m = Ae.shape[0], Ae.shape[1], Ae.shape[2]
    Ad = Ae.reshape(E, Np * m, Np * m)
    rr = r.reshape(E, m, Np).permute(0, 2, 1).reshape(E, Np * m, 1)
    z = torch.linalg.solve(Ad, rr).reshape(E, Np, m)
    return z.permute(0, 2, 1)


# --------------------------------------------------------------------------- GMRES
def gmres(matvec, precond, b: torch.Tensor, rtol=1e-8, restart=50, max_iters=1000, x0=None):
    """Right-preconditioned restarted GMRES with modified Gram-Schmidt.

    Returns (x, iterations, relative residual ||b - A x|| / ||b||).
    """
    shape = b.shape
    bf = b.reshape(-1)
    nb = float(torch.linalg.norm(bf))
    x = torch.zeros_like(bf) if x0 is None else x0.reshape(-1).clone()
    if nb == 0.0:
        return x.reshape(shape), 0, 0.0
    its = 0
    while True:
        r = bf - matvec(x.reshape(shape)).reshape(-1)
        beta = float(torch.linalg.norm(r))
        if beta <= rtol * nb or its >= max_iters:
            return x.reshape(shape), its, beta / nb
        V = [r / beta]
        Z = []
        H = np.zeros((restart + 1, restart))
        cs, sn = np.zeros(restart), np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        k_used = 0
        for k in range(restart):
            z = precond(V[k].reshape(shape)).reshape(-1)
            Z.append(z)
            w = matvec(z.reshape(shape)).reshape(-1)
            for j in range(k + 1):
                H[j, k] = float(torch.dot(w, V[j]))
                w = w - H[j, k] * V[j]
            H[k + 1, k] = float(torch.linalg.norm(w))
            V.append(w / H[k + 1, k] if H[k + 1, k] != 0 else w)
            for j in range(k):
                t = cs[j] * H[j, k] + sn[j] * H[j + 1, k]
                H[j + 1, k] = -sn[j] * H[j, k] + cs[j] * H[j + 1, k]
                H[j, k] = t
            den = math.hypot(H[k, k], H[k + 1, k])
            cs[k], sn[k] = H[k, k] / den, H[k + 1, k] / den
            H[k, k] = den
            H[k + 1, k] = 0.0
            g[k + 1] = -sn[k] * g[k]
            g[k] = cs[k] * g[k]
            its += 1
            k_used = k + 1
            if abs(g[k + 1]) <= rtol * nb or its >= max_iters:
                break
        y = np.linalg.solve(np.triu(H[:k_used, :k_used]), g[:k_used])
        for j in range(k_used):
            x = x + float(y[j]) * Z[j]


# --------------------------------------------------------------------------- Newton / RK4
class NewtonResult(dict):
    pass


def newton_step(d: LineDG, U, Ucomb, gamma, alpha=1.0, rtol=1e-8, restart=50, max_iters=2000,
                precond="bilu0"):
    """One Newton step on G(U) = alpha (U - Ucomb) - gamma R(U) (BDF2 form when alpha = 1).

    Solves (alpha I - gamma A) dU = -G(U) with GMRES(restart), the split product
    and the line-pattern preconditioner, then returns U + dU and statistics.
    """
    U = torch.as_tensor(U, dtype=DT).reshape(d.E, d.m, d.Np)
    Uc = torch.zeros_like(U) if Ucomb is None else torch.as_tensor(Ucomb, dtype=DT).reshape(U.shape)
    R0 = d.residual(U)
    G0 = alpha * (U - Uc) - gamma * R0
    K11, K12, K21 = d.jacobian(U)
    c11, c12 = d.column_nodes("K11"), d.column_nodes("K12")
    pat = line_pattern(d)
    At = precond_matrix(d, K11, K12, K21, gamma, alpha)
    if precond == "bilu0":
        F = bilu0(At, pat)
        pc = lambda r: bilu0_apply(F, pat, r)
    elif precond == "exact":
        pc = lambda r: dense_block_solve(At, r)
    else:
        pc = lambda r: r
    mv = lambda x: split_matvec(d, K11, K12, x, gamma, alpha, c11, c12)
    dU, its, rel = gmres(mv, pc, -G0, rtol=rtol, restart=restart, max_iters=max_iters)
    U1 = U + dU.reshape(U.shape)
    G1 = alpha * (U1 - Uc) - gamma * d.residual(U1)
    return NewtonResult(U=U1, iters=its, lin_relres=rel, G0=float(torch.linalg.norm(G0)),
                        G1=float(torch.linalg.norm(G1)), dU=dU.reshape(U.shape))


# Alexander's L-stable, three-stage, third-order DIRK (Section 4.1, eqs. dirk1, dirk2)
DIRK3_ALPHA = 0.435866521508459


def dirk3_tableau():
    """(A, b): a_ii = alpha, c_2 = tau_2 = (1 + alpha)/2, last row of A equal to b."""
    a = DIRK3_ALPHA
    tau2 = (1.0 + a) / 2.0
    b1 = -(6 * a * a - 16 * a + 1) / 4
    b2 = (6 * a * a - 20 * a + 5) / 4
    A = [[a, 0.0, 0.0], [tau2 - a, a, 0.0], [b1, b2, a]]
    return A, [b1, b2, a]


def dirk3_step(d: LineDG, U, dt, newton_tol=1e-12, max_newton=20, rtol=1e-12, restart=50):
    """One DIRK3 step: K_i = F(U_n + dt sum_j a_ij K_j), U_{n+1} = U_n + dt sum_j b_j K_j.

    Each stage solves Y_i - (U_n + dt sum_{j<i} a_ij K_j) - dt a_ii F(Y_i) = 0 by
    Newton's method (newton_step, a fresh Jacobian every iteration) until
    ||G|| <= newton_tol ||G(Y start)||, then K_i = F(Y_i).  Returns (U_{n+1}, stats).
    """
    A, b = dirk3_tableau()
    U = torch.as_tensor(U, dtype=DT).reshape(d.E, d.m, d.Np)
    K = []
    Y = U.clone()
    newton = []
    for i in range(3):
        Ucomb = U.clone()
        for j in range(i):
            Ucomb = Ucomb + dt * A[i][j] * K[j]
        gamma = dt * A[i][i]
        G0 = None
        for it in range(max_newton):
            res = newton_step(d, Y, Ucomb, gamma, rtol=rtol, restart=restart)
            if G0 is None:
                G0 = res["G0"]
            Y = res["U"]
            if res["G1"] <= newton_tol * G0:
                break
        newton.append(it + 1)
        K.append(d.residual(Y))
    U1 = U.clone()
    for j in range(3):
        U1 = U1 + dt * b[j] * K[j]
    return U1, {"newton": newton}


def rk4_step(d: LineDG, U, dt):
    """Classical RK4 for dU/dt = R(U) (Section 4.1)."""
    U = torch.as_tensor(U, dtype=DT)
    k1 = d.residual(U)
    k2 = d.residual(U + 0.5 * dt * k1)
    k3 = d.residual(U + 0.5 * dt * k2)
    k4 = d.residual(U + dt * k3)
    return U + dt / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)


# --------------------------------------------------------------------------- dense helpers (tiny meshes)
def dense_operator(d: LineDG, K11, K12, K21) -> np.ndarray:
    """Dense A = K11 + K12 K21 in the flattened [E, m, Np] ordering (tiny meshes only)."""
    E, Np, m, D = d.E, d.Np, d.m, d.D
    n = E * m * Np
    A = np.zeros((n, n))
    eye = torch.eye(n, dtype=DT)
    c11, c12 = d.column_nodes("K11"), d.column_nodes("K12")
    for j in range(n):
        A[:, j] = split_matvec(d, K11, K12, eye[j], gamma=-1.0, alpha=0.0, cols11=c11,
                               cols12=c12).reshape(-1).numpy()
    return A


def sparse_blocks(d: LineDG, K11, K12, K21):
    """scipy.sparse K11 [n x n], K12 [n x nq], K21 [nq x n] in the [E, m, Np] / [E, m, D, Np] orderings."""
    import scipy.sparse as sp
    E, Np, m, D = d.E, d.Np, d.m, d.D
    c11, c12, c21 = d.column_nodes("K11"), d.column_nodes("K12"), d.column_nodes("K21")

    def build(K, cols, rw, cw, fill):
        rows, colsi, vals = [], [], []
        e_idx = np.arange(E)[:, None, None]
        a_idx = np.arange(Np)[None, :, None]
        Kn = K.numpy()
        for s in range(cols.shape[2]):
            g = cols[:, :, s]
            ok = g >= 0
            ee, nd = np.divmod(np.where(ok, g, 0), Np)
            for r in range(rw):
                for c in range(cw):
                    v = fill(Kn, s, r, c)
                    rr = (np.arange(E)[:, None] * rw + r) * Np + np.arange(Np)[None, :]
                    cc = (ee * cw + c) * Np + nd
                    rows.append(rr[ok]); colsi.append(cc[ok]); vals.append(v[ok])
        return np.concatenate(rows), np.concatenate(colsi), np.concatenate(vals)

    n, nq = E * m * Np, E * m * D * Np
    r, c, v = build(K11, c11, m, m, lambda Kn, s, i, j: Kn[:, :, s, i, j])
    S11 = sp.csr_matrix((v, (r, c)), shape=(n, n))
    r, c, v = build(K12, c12, m, m * D, lambda Kn, s, i, j: Kn[:, :, s, i, j])
    S12 = sp.csr_matrix((v, (r, c)), shape=(n, nq))
    r, c, v = build(K21, c21, m * D, m,
                    lambda Kn, s, i, j: Kn[:, :, s, i % D] * (1.0 if i // D == j else 0.0))
    S21 = sp.csr_matrix((v, (r, c)), shape=(nq, n))
    return S11, S12, S21


def coupled_residuals(d: LineDG, U, Q):
    """The coupled system of Section 4.1 with Q an unknown: (R(U, Q), Q - G(U, Q))."""
    return d.residual(U, Q=Q), Q - d.gradient(U, Q=Q)


def coupled_steady_solve(d: LineDG):
    """Steady solve of the coupled (U, Q) system for a linear problem (Poisson), any C22.

    F(U, Q) = [-R(U, Q); Q - G(U, Q)] is affine in (U, Q); its matrix is formed by forward
    differentiation of F at zero (one column per unknown) and the system F = 0 is solved by a
    dense LU.  Returns (U [E, m, Np], Q [E, m, D, Np]).
    """
    E, m, D, Np = d.E, d.m, d.D, d.Np
    nu, nq = E * m * Np, E * m * D * Np

    def F(x):
        U = x[:nu].reshape(E, m, Np)
        Q = x[nu:].reshape(E, m, D, Np)
        R, RQ = coupled_residuals(d, U, Q)
        return torch.cat([-R.reshape(-1), RQ.reshape(-1)])

    x0 = torch.zeros(nu + nq, dtype=DT)
    F0 = F(x0)
    A = jacfwd(F)(x0)
    x = torch.linalg.solve(A, -F0)
    return x[:nu].reshape(E, m, Np), x[nu:].reshape(E, m, D, Np)


def steady_direct_solve(d: LineDG, U0=None):
    """Steady linear solve R(U) = 0 via the split system and a sparse direct solver.

    Solves [[K11, K12], [K21, -I]] [U; Q] = [-R(0) + K12 Q(0)..] in the form
    (K11 + K12 K21) dU = -R(U0) (exact for linear problems such as Poisson).
    """
    import scipy.sparse.linalg as spla
    U = torch.zeros(d.E, d.m, d.Np, dtype=DT) if U0 is None else torch.as_tensor(U0, dtype=DT)
    R0 = d.residual(U)
    K11, K12, K21 = d.jacobian(U)
    S11, S12, S21 = sparse_blocks(d, K11, K12, K21)
    A = (S11 + S12 @ S21).tocsc()
    dU = spla.spsolve(A, -R0.reshape(-1).numpy())
    return U + torch.as_tensor(dU).reshape(U.shape)
