"""Physical fluxes and numerical fluxes (oracle, torch fp64 on the CPU).

TEST INFRASTRUCTURE ONLY: part of the plain FP64 CPU oracle.

* Poisson (Section 5.1): m = 1, F = F^vis = -q, source f.
* Euler / Navier-Stokes (Section 5.2, eqs. ns1-ns3): conserved variables
  (rho, rho u_i, rho E), ideal gas p = (gamma-1)(rho E - rho|u|^2/2), viscous
  stress tau_ij = mu (du_i/dx_j + du_j/dx_i - 2/3 div u delta_ij) and heat flux
  q_j = -(mu/Pr) d/dx_j (E + p/rho - |u|^2/2).  The printed momentum equation
  differentiates by x_i and the printed stress uses du_k/dx_j: read as the
  usual d/dx_j (rho u_i u_j + p delta_ij) and du_k/dx_k.
* Roe's approximate Riemann solver (Section 5.2), no entropy fix:
  Fhat.n = 1/2 (F(uL) + F(uR)).n - 1/2 |A_roe| (uR - uL), where A_roe is the
  flux Jacobian at the Roe-averaged state and |A_roe| is evaluated by
  Sylvester's formula on its three distinct eigenvalues (Vn - c, Vn, Vn + c).
  For a non-unit normal, Fhat.n = |n| Fhat.nbar (Section 2.2).
* Shapes: a state is ``[..., m]``, a gradient ``[..., m, D]``, a flux
  ``[..., m, D]``, a normal ``[..., D]``.
"""
from __future__ import annotations

import torch
from torch.func import jacfwd, vmap

EQ_POISSON, EQ_EULER, EQ_NS = 0, 1, 2


class Physics:
    def __init__(self, equation: int, dim: int, gamma: float = 1.4, mu: float = 0.0,
                 prandtl: float = 0.72):
        self.eq = equation
        self.dim = dim
        self.gamma = gamma
        self.mu = mu
        self.prandtl = prandtl
        self.m = 1 if equation == EQ_POISSON else dim + 2
        self.has_inviscid = equation != EQ_POISSON
        self.has_viscous = equation == EQ_POISSON or (equation == EQ_NS and mu != 0.0)

    # ------------------------------------------------------------ inviscid
    def flux_inv(self, u: torch.Tensor) -> torch.Tensor:
        """Euler flux F[..., c, d]."""
        g, D = self.gamma, self.dim
        rho = u[..., 0]
        mom = u[..., 1:1 + D]
        rE = u[..., 1 + D]
        vel = mom / rho[..., None]
        p = (g - 1.0) * (rE - 0.5 * (mom * vel).sum(-1))
        rows = [mom]
        eye = torch.eye(D, dtype=u.dtype)
        rows += [mom[..., i, None] * vel + p[..., None] * eye[i] for i in range(D)]
        rows += [vel * (rE + p)[..., None]]
        return torch.stack(rows, dim=-2)

    def flux_inv_n(self, u: torch.Tensor, n: torch.Tensor) -> torch.Tensor:
        return (self.flux_inv(u) * n[..., None, :]).sum(-1)

    # ------------------------------------------------------------ viscous
    def flux_vis(self, u: torch.Tensor, q: torch.Tensor) -> torch.Tensor:
        """Viscous flux F^vis[..., c, d] (sign: u_t + div(F^inv + F^vis) = S)."""
        if self.eq == EQ_POISSON:
            return -q
        g, D, mu = self.gamma, self.dim, self.mu
        rho = u[..., 0]
        vel = u[..., 1:1 + D] / rho[..., None]
        Esp = u[..., 1 + D] / rho
        drho = q[..., 0, :]                                       # [..., D]
        dvel = (q[..., 1:1 + D, :] - vel[..., :, None] * drho[..., None, :]) / rho[..., None, None]
        dE = (q[..., 1 + D, :] - Esp[..., None] * drho) / rho[..., None]
        # h = E + p/rho - |u|^2/2 = gamma (E - |u|^2/2)
        dh = g * (dE - (vel[..., :, None] * dvel).sum(-2))
        div = torch.diagonal(dvel, dim1=-2, dim2=-1).sum(-1)
        eye = torch.eye(D, dtype=u.dtype)
        tau = mu * (dvel + dvel.transpose(-1, -2) - (2.0 / 3.0) * div[..., None, None] * eye)
        heat = -(mu / self.prandtl) * dh
        zero = torch.zeros_like(drho)
        rows = [zero] + [-tau[..., i, :] for i in range(D)]
        rows += [-(vel[..., :, None] * tau).sum(-2) + heat]
        return torch.stack(rows, dim=-2)

    def flux_total(self, u, q):
        F = torch.zeros(u.shape + (self.dim,), dtype=u.dtype)
        if self.has_inviscid:
            F = F + self.flux_inv(u)
        if self.has_viscous:
            F = F + self.flux_vis(u, q)
        return F

    # ------------------------------------------------------------ Roe
    def roe_state(self, uR, uL):
        """Conserved state whose Euler flux Jacobian is the Roe matrix.

        The Euler flux Jacobian depends on the state only through the velocity
        and the total enthalpy H, so the Roe averages (sqrt(rho) weighted
        velocity and H) and the geometric-mean density define it.
        """
        g, D = self.gamma, self.dim

        def prim(u):
            rho = u[..., 0]
            vel = u[..., 1:1 + D] / rho[..., None]
            p = (g - 1.0) * (u[..., 1 + D] - 0.5 * rho * (vel * vel).sum(-1))
            H = (u[..., 1 + D] + p) / rho
            return rho, vel, H

        rR, vR, HR = prim(uR)
        rL, vL, HL = prim(uL)
        sR, sL = torch.sqrt(rR), torch.sqrt(rL)
        vel = (sL[..., None] * vL + sR[..., None] * vR) / (sL + sR)[..., None]
        H = (sL * HL + sR * HR) / (sL + sR)
        rho = sL * sR
        Esp = (H + 0.5 * (g - 1.0) * (vel * vel).sum(-1)) / g
        return torch.cat([rho[..., None], rho[..., None] * vel, (rho * Esp)[..., None]], dim=-1)

    def roe_matrix(self, uR, uL, nbar):
        """A_roe(nbar) = d(F(w).nbar)/dw at the Roe-average state w."""
        w = self.roe_state(uR, uL)
        batch = w.shape[:-1]
        wf = w.reshape(-1, self.m)
        nf = nbar.expand(batch + (self.dim,)).reshape(-1, self.dim)
        A = vmap(jacfwd(lambda ww, nn: self.flux_inv_n(ww, nn)))(wf, nf)
        return A.reshape(batch + (self.m, self.m)), w

    def roe_abs_matrix(self, uR, uL, nbar):
        """|A_roe| by Sylvester's formula with eigenvalues Vn - c, Vn, Vn + c."""
        A, w = self.roe_matrix(uR, uL, nbar)
        g, D = self.gamma, self.dim
        vel = w[..., 1:1 + D] / w[..., 0:1]
        H = (w[..., 1 + D] + (g - 1.0) * (w[..., 1 + D] - 0.5 * w[..., 0] * (vel * vel).sum(-1))) / w[..., 0]
        c = torch.sqrt((g - 1.0) * (H - 0.5 * (vel * vel).sum(-1)))
        vn = (vel * nbar).sum(-1)
        lams = [vn - c, vn, vn + c]
        eye = torch.eye(self.m, dtype=A.dtype).expand(A.shape)
        absA = torch.zeros_like(A)
        for k in range(3):
            term = torch.abs(lams[k])[..., None, None] * eye
            for j in range(3):
                if j == k:
                    continue
                term = term @ (A - lams[j][..., None, None] * eye) / (lams[k] - lams[j])[..., None, None]
            absA = absA + term
        return absA, A

    def roe_flux(self, uR, uL, n):
        """Fhat . n (uR on the side n points to, uL on the other; n non-unit)."""
        nn = torch.sqrt((n * n).sum(-1))
        nbar = n / nn[..., None]
        absA, _ = self.roe_abs_matrix(uR, uL, nbar)
        avg = 0.5 * (self.flux_inv_n(uL, nbar) + self.flux_inv_n(uR, nbar))
        diss = 0.5 * (absA @ (uR - uL)[..., None])[..., 0]
        return nn[..., None] * (avg - diss)
