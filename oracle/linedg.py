"""Line-DG semi-discretisation: residual, LDG gradient and Jacobians (oracle).

TEST INFRASTRUCTURE ONLY: part of the plain FP64 CPU oracle (torch on CPU).

What is computed, and where the paper defines it:

* geometry (Section 2.2): the isoparametric map x(X) = sum x_ijk phi_i phi_j phi_k,
  G = grad_X x, J = det G, and the non-unit normals a_n = J G^{-T} N_n
  (eq. contraflux); along a direction-n line, G is evaluated exactly at the Gauss
  points; the face normals are n^+ = a_n(xi_n = 1), n^- = -a_n(xi_n = 0);
* the 1-D Galerkin problem on every line (eqs. galerkinscheme2, reqn):
  M r = b with b_i = phi_i(1) Fhat(n^+) + phi_i(0) Fhat(n^-) - int f~ phi_i',
  f~ = F . a_n, integrated with ceil((3p+1)/2) Gauss points, solved with the
  Cholesky factor of M; R = -(1/J) sum_n r^(n) + S (eq. semidisc);
* the auxiliary equation (eqs. splitdisc2, numfluxu1, semidisc2-2):
  d^(n) from the same 1-D procedure applied to u (x) a_n with face values
  uhat (x) n, and q = (1/J) sum_n d^(n);
* LDG fluxes with C12 = n S/2 (Section 3): Fhat^vis from the outside when the
  face switch is +1 and from the inside when it is -1, uhat the other way
  round; interior penalty C11 |n| (u_in - u_out); Dirichlet faces use
  Fhat = F(u_in, q_in).n + C11_D |n| (u_in - g_D), uhat = g_D (eqs.
  dirichlet1/2); inviscid Dirichlet faces take Roe(g_D, u_in) (the
  characteristic far-field condition);
* Neumann faces (eqs. neumann1/2): Fhat . n = |n| g_N, uhat = u_in - C22 (F(u_in, q_in) . nbar - g_N);
* C22 (eqs. ldgflux1/2): uhat gains C22 [[F . nbar]] = C22 (F(u_out, q_out) - F(u_in, q_in)) . nbar
  on interior faces (nbar the unit outward normal), so the auxiliary equation
  couples q across faces: the coupled system of Section 4.1 with unknowns
  (U, Q), residuals R(U, Q) and Q - G(U, Q); C22 = 0 (the default) gives the
  reduced system where Q = D(U) is eliminated element by element;
* slip walls: Roe(u_m, u_in) with the mirror state u_m (normal momentum
  reflected), no viscous flux through the wall, uhat = u_in;
  boundary kinds come from face_nbr = -(kind + 1): 0 Dirichlet, 1 Neumann,
  2 slip wall;
* Jacobians K11 = dR/dU, K12 = dR/dQ, K21 = dD/dU (Section 4.1), obtained by
  forward-mode differentiation of each line's right-hand side.

Line-block storage (identical slot numbering on both sides of the parity
tests).  For a row node with reference coordinates (i_0, .., i_{D-1}):
  slots 0..p            : nodes (t, i_1, ..) of its direction-0 line (self at t = i_0)
  slots p+1+(n-1)p + t' : nodes of its direction-n line (n >= 1) other than itself,
                          t' = t (t < i_n) or t - 1 (t > i_n)
  then neighbour slots: K11 has 2D (face 2n+s), K12 has D (the side whose
  switch is +1), K21 has D (the side whose switch is -1).
"""
from __future__ import annotations

import numpy as np
import torch
from torch.func import jacfwd, vmap

from .basis import LineOps
from .physics import Physics, EQ_POISSON

DT = torch.float64


def _t(x):
    if isinstance(x, torch.Tensor):
        return x.to(DT)
    return torch.as_tensor(np.asarray(x), dtype=DT)


class LineDG:
    """The discrete operator for one mesh and one equation set."""

    def __init__(self, dim, p, xyz, face_nbr, nbr_node, switch_plus, physics: Physics,
                 c11_interior=0.0, c11_dirichlet=10.0, source=None, gD=None, nodes="gll", gN=None, c22=0.0):
        self.D = dim
        self.p = p
        self.n1 = p + 1
        self.Np = self.n1 ** dim
        self.NL = self.n1 ** (dim - 1)
        self.ph = physics
        self.m = physics.m
        self.ops = LineOps(p, nodes)
        self.ng = self.ops.ng
        self.I = _t(self.ops.I)
        self.Dg = _t(self.ops.Dg)
        self.wg = _t(self.ops.wg)
        self.Mchol = _t(self.ops.Mchol)
        self.Dn = _t(self.ops.Dn)
        self.xyz = _t(xyz)
        self.E = self.xyz.shape[0]
        self.face_nbr = torch.as_tensor(np.asarray(face_nbr), dtype=torch.int64)
        self.nbr_node = torch.as_tensor(np.asarray(nbr_node), dtype=torch.int64)
        self.switch_plus = torch.as_tensor(np.asarray(switch_plus), dtype=torch.int64)
        self.c11_int = float(c11_interior)
        self.c11_dir = float(c11_dirichlet)
        self.source = None if source is None else _t(source)
        self.gD = None if gD is None else _t(gD)
        self.gN = None if gN is None else _t(gN)
        self.c22 = float(c22)
        self.nslot_line = dim * p + 1
        self.nslot11 = self.nslot_line + 2 * dim
        self.nslot12 = self.nslot_line + dim
        self.nslot21 = self.nslot_line + dim

    # ------------------------------------------------------------------ layout
    def _axis(self, n):
        return 2 + (self.D - 1 - n)

    def to_lines(self, X, n):
        """[Ne, C, Np] -> [Ne, NL, N1, C] (lines of direction n)."""
        Ne, C = X.shape[0], X.shape[1]
        Y = X.reshape((Ne, C) + (self.n1,) * self.D).movedim(self._axis(n), -1)
        return Y.reshape(Ne, C, self.NL, self.n1).permute(0, 2, 3, 1)

    def from_lines(self, Y, n):
        """Inverse of :meth:`to_lines`."""
        Ne, C = Y.shape[0], Y.shape[3]
        Z = Y.permute(0, 3, 1, 2).reshape((Ne, C) + (self.n1,) * self.D)
        Z = Z.movedim(-1, self._axis(n))
        return Z.reshape(Ne, C, self.Np)

    def node_coords(self):
        """coords[node, d] = reference index of the node along direction d."""
        idx = np.arange(self.Np)
        return np.stack([(idx // self.n1 ** d) % self.n1 for d in range(self.D)], axis=1)

    # ------------------------------------------------------------------ geometry
    def nodal_G(self, elems):
        """G[e, node, a, b] = d x_a / d X_b at the nodes."""
        x = self.xyz[elems]
        cols = []
        for b in range(self.D):
            xl = self.to_lines(x, b)
            cols.append(self.from_lines(torch.einsum("ij,eljc->elic", self.Dn, xl), b))
        return torch.stack(cols, dim=-1).permute(0, 2, 1, 3)  # [Ne, Np, a, b]

    def metric_on_lines(self, elems, n, E1, D1, Gn=None):
        """a_n = J G^{-T} N_n at points along direction-n lines.

        ``E1[q, i]`` / ``D1[q, i]`` hold the basis values / derivatives at the
        points along the line; the other reference coordinates are nodes.
        Returns [Ne, NL, npts, D].
        """
        x = self.xyz[elems]
        if Gn is None:
            Gn = self.nodal_G(elems)
        cols = []
        for b in range(self.D):
            if b == n:
                cols.append(torch.einsum("gi,elic->elgc", D1, self.to_lines(x, n)))
            else:
                gb = Gn[:, :, :, b].permute(0, 2, 1)  # [Ne, a, Np]
                cols.append(torch.einsum("gi,elic->elgc", E1, self.to_lines(gb, n)))
        G = torch.stack(cols, dim=-1)  # [Ne, NL, npts, a, b]
        Jdet = torch.linalg.det(G)
        Ginv = torch.linalg.inv(G)
        return Jdet[..., None] * Ginv[..., n, :]

    def geometry(self, elems):
        Gn = self.nodal_G(elems)
        J = torch.linalg.det(Gn)  # [Ne, Np]
        eye = torch.eye(self.n1, dtype=DT)
        ends_v = eye[[0, self.p]]
        ends_d = self.Dn[[0, self.p]]
        ag, n0, n1 = [], [], []
        for n in range(self.D):
            ag.append(self.metric_on_lines(elems, n, self.I, self.Dg, Gn))
            an = self.metric_on_lines(elems, n, ends_v, ends_d, Gn)
            n0.append(-an[:, :, 0])
            n1.append(an[:, :, 1])
        return dict(J=J, ag=ag, n0=n0, n1=n1)

    # ------------------------------------------------------------------ faces
    def _outside(self, V, elems, n, s):
        """Values of nodal field V[E, C, Np] at the coinciding neighbour nodes.

        Returns ([Ne, NL, C] values, [Ne] boundary flag); boundary rows are 0.
        """
        f = 2 * n + s
        nb = self.face_nbr[elems, f]
        nodes = self.nbr_node[elems, f]
        bnd = nb < 0
        nbc = torch.where(bnd, torch.zeros_like(nb), nb)
        ndc = torch.where(nodes < 0, torch.zeros_like(nodes), nodes)
        vals = V[nbc[:, None], :, ndc]  # [Ne, NL, C]
        vals = torch.where(bnd[:, None, None], torch.zeros_like(vals), vals)
        return vals, bnd

    def _gD_face(self, elems, n, s):
        if self.gD is None:
            return torch.zeros(len(elems), self.NL, self.m, dtype=DT)
        return self.gD[elems, 2 * n + s].permute(0, 2, 1)  # [Ne, NL, m]

    def _gN_face(self, elems, n, s):
        if self.gN is None:
            return torch.zeros(len(elems), self.NL, self.m, dtype=DT)
        return self.gN[elems, 2 * n + s].permute(0, 2, 1)  # [Ne, NL, m]

    def _kind(self, elems, n, s):
        """Boundary kind of face 2n+s per element: -1 interior, 0 Dirichlet, 1 Neumann, 2 slip wall."""
        nb = self.face_nbr[elems, 2 * n + s]
        return torch.where(nb >= 0, torch.full_like(nb, -1), -nb - 1)

    # ------------------------------------------------------------------ line problems
    def _mass_solve(self, b):
        """Solve M r = b along axis -3 (b: [..., N1, a, b'])."""
        sh = b.shape
        bb = b.reshape(sh[:-3] + (self.n1, -1))
        r = torch.cholesky_solve(bb, self.Mchol)
        return r.reshape(sh)

    def grad_line_rhs(self, u_line, uh0, uh1, ag, n0, n1):
        """Right-hand side b[.., i, c, d] of the line problem for d^(n)."""
        ug = torch.einsum("gi,...ic->...gc", self.I, u_line)
        vol = torch.einsum("g,gi,...gc,...gd->...icd", self.wg, self.Dg, ug, ag)
        e0 = torch.zeros(self.n1, dtype=DT)
        e0[0] = 1.0
        ep = torch.zeros(self.n1, dtype=DT)
        ep[self.p] = 1.0
        face = (e0[:, None, None] * (uh0[..., :, None] * n0[..., None, :])[..., None, :, :]
                + ep[:, None, None] * (uh1[..., :, None] * n1[..., None, :])[..., None, :, :])
        return face - vol

    def _uhat(self, u_in, u_out, S, kind, gD):
        """LDG trace: inside if S = +1, outside if S = -1; g_D on Dirichlet faces; the inside
        value on Neumann faces (C22 = 0) and slip walls."""
        sel = torch.where((S > 0)[..., None], u_in, u_out)
        sel = torch.where((kind > 0)[..., None], u_in, sel)
        return torch.where((kind == 0)[..., None], gD, sel)

    def gradient(self, U, elems=None, homogeneous=False, geo=None, Q=None):
        """Q = D(U) for the given elements: [Ne, m, D, Np] (eqs. semidisc2-2).

        With C22 != 0 the trace uhat involves the normal viscous flux of both
        sides, so the gradient field ``Q`` [E, m, D, Np] entering it must be
        given: the result is then G(U, Q) of the coupled system.
        """
        if elems is None:
            elems = torch.arange(self.E)
        elems = torch.as_tensor(elems, dtype=torch.int64)
        U = _t(U)
        if self.c22 != 0.0 and Q is None:
            raise ValueError("C22 != 0: the gradient needs the current Q")
        if geo is None:
            geo = self.geometry(elems)
        Ne = len(elems)
        acc = torch.zeros(Ne, self.m, self.D, self.Np, dtype=DT)
        for n in range(self.D):
            ul = self.to_lines(U[elems], n)  # [Ne, NL, N1, m]
            Sp = self.switch_plus[elems, n][:, None].expand(Ne, self.NL)
            if self.c22 != 0.0:
                Qa = _t(Q)
                ql = self.to_lines(Qa[elems].reshape(Ne, self.m * self.D, self.Np), n).reshape(
                    Ne, self.NL, self.n1, self.m, self.D)
            uh = []
            for s in (0, 1):
                uo, bnd = self._outside(U, elems, n, s)
                gD = torch.zeros_like(uo) if homogeneous else self._gD_face(elems, n, s)
                S = Sp if s == 1 else -Sp
                uin = ul[:, :, self.p if s == 1 else 0]
                kind = self._kind(elems, n, s)[:, None].expand(Ne, self.NL)
                u_hat = self._uhat(uin, uo, S, kind, gD)
                if self.c22 != 0.0:
                    # C22 [[F . nbar]]: interior faces take the jump of the normal viscous flux,
                    # Neumann faces its difference from g_N; Dirichlet faces and slip walls none
                    nrm = geo["n1"][n] if s == 1 else geo["n0"][n]  # outward, [Ne, NL, D]
                    nbar = nrm / torch.sqrt((nrm * nrm).sum(-1, keepdim=True))
                    qin = ql[:, :, self.p if s == 1 else 0]
                    qo = self._outside(Qa.reshape(self.E, self.m * self.D, self.Np), elems, n, s)[0].reshape(
                        Ne, self.NL, self.m, self.D)
                    Fin = (self.ph.flux_vis(uin, qin) * nbar[..., None, :]).sum(-1)
                    Fout = (self.ph.flux_vis(uo, qo) * nbar[..., None, :]).sum(-1)
                    gN = torch.zeros_like(uo) if homogeneous else self._gN_face(elems, n, s)
                    jump = torch.where((kind == 1)[..., None], Fin - gN, Fin - Fout)
                    jump = torch.where(((kind == 0) | (kind == 2))[..., None], torch.zeros_like(jump), jump)
                    u_hat = u_hat + self.c22 * jump
                uh.append(u_hat)
            b = self.grad_line_rhs(ul, uh[0], uh[1], geo["ag"][n], geo["n0"][n], geo["n1"][n])
            d = self._mass_solve(b)  # [Ne, NL, N1, m, D]
            acc += self.from_lines(d.reshape(Ne, self.NL, self.n1, self.m * self.D), n).reshape(
                Ne, self.m, self.D, self.Np)
        return acc / geo["J"][:, None, None, :]

    @staticmethod
    def mirror(u, nrm):
        """The wall's mirror state: normal momentum reversed, density and energy kept."""
        nb = nrm / torch.sqrt((nrm * nrm).sum(-1, keepdim=True))
        D = nrm.shape[-1]
        mom = u[..., 1:1 + D]
        mn = (mom * nb).sum(-1, keepdim=True)
        return torch.cat([u[..., :1], mom - 2.0 * mn * nb, u[..., 1 + D:]], dim=-1)

    def face_flux(self, u_in, q_in, u_out, q_out, nrm, S, kind, gD, gN):
        """Numerical flux Fhat . n at one face point (shapes [..., m]); kind -1 interior,
        0 Dirichlet, 1 Neumann, 2 slip wall."""
        ph = self.ph
        nn = torch.sqrt((nrm * nrm).sum(-1))[..., None]
        out = torch.zeros_like(u_in)
        dirichlet, slip = (kind == 0)[..., None], (kind == 2)[..., None]
        if ph.has_inviscid:
            uR = torch.where(dirichlet, gD, torch.where(slip, self.mirror(u_in, nrm), u_out))
            out = out + ph.roe_flux(uR, u_in, nrm)
        if ph.has_viscous:
            Fin = (ph.flux_vis(u_in, q_in) * nrm[..., None, :]).sum(-1)
            Fout = (ph.flux_vis(u_out, q_out) * nrm[..., None, :]).sum(-1)
            interior = torch.where((S > 0)[..., None], Fout, Fin) + self.c11_int * nn * (u_in - u_out)
            dirich = Fin + self.c11_dir * nn * (u_in - gD)
            vis = torch.where(dirichlet, dirich, interior)
            out = out + torch.where(slip, torch.zeros_like(vis), vis)
        return torch.where((kind == 1)[..., None], nn * gN, out)

    def resid_line_rhs(self, u_line, q_line, uo0, qo0, uo1, qo1, ag, n0, n1, S1, k0, k1, gD0, gD1, gN0, gN1):
        """Right-hand side b[.., i, c] of the line problem for r^(n) (eq. galerkinscheme2)."""
        ug = torch.einsum("gi,...ic->...gc", self.I, u_line)
        qg = torch.einsum("gi,...icd->...gcd", self.I, q_line)
        Fg = self.ph.flux_total(ug, qg)
        ft = (Fg * ag[..., None, :]).sum(-1)  # [..., ng, m]
        vol = torch.einsum("g,gi,...gc->...ic", self.wg, self.Dg, ft)
        F1 = self.face_flux(u_line[..., self.p, :], q_line[..., self.p, :, :], uo1, qo1, n1, S1, k1, gD1, gN1)
        F0 = self.face_flux(u_line[..., 0, :], q_line[..., 0, :, :], uo0, qo0, n0, -S1, k0, gD0, gN0)
        e0 = torch.zeros(self.n1, dtype=DT)
        e0[0] = 1.0
        ep = torch.zeros(self.n1, dtype=DT)
        ep[self.p] = 1.0
        face = e0[:, None] * F0[..., None, :] + ep[:, None] * F1[..., None, :]
        return face - vol

    def _line_inputs(self, U, Q, elems, n, qidx):
        """Per-line inputs of direction n for elements ``elems``.

        ``Q`` holds rows for the elements listed in ``qidx`` (global -> row).
        """
        Ne = len(elems)
        m, D = self.m, self.D
        ul = self.to_lines(U[elems], n)
        ql = self.to_lines(Q[qidx[elems]].reshape(Ne, m * D, self.Np), n).reshape(Ne, self.NL, self.n1, m, D)
        outs = []
        for s in (0, 1):
            uo, bnd = self._outside(U, elems, n, s)
            f = 2 * n + s
            nb = self.face_nbr[elems, f]
            nodes = self.nbr_node[elems, f]
            rows = qidx[torch.where(nb < 0, torch.zeros_like(nb), nb)]
            ndc = torch.where(nodes < 0, torch.zeros_like(nodes), nodes)
            qo = Q[rows[:, None], :, :, ndc]  # [Ne, NL, m, D]
            qo = torch.where((nb < 0)[:, None, None, None], torch.zeros_like(qo), qo)
            gD = self._gD_face(elems, n, s)
            gN = self._gN_face(elems, n, s)
            kind = self._kind(elems, n, s)[:, None].expand(Ne, self.NL)
            outs.append((uo, qo, kind, gD, gN))
        S1 = self.switch_plus[elems, n][:, None].expand(Ne, self.NL)
        return ul, ql, outs, S1

    def _with_neighbours(self, elems):
        nb = self.face_nbr[elems].reshape(-1)
        nb = nb[nb >= 0]
        allel = torch.unique(torch.cat([elems, nb]))
        qidx = torch.full((self.E,), -1, dtype=torch.int64)
        qidx[allel] = torch.arange(len(allel))
        return allel, qidx

    def residual(self, U, elems=None, return_abs=False, Q=None):
        """R = -(1/J) sum_n r^(n) + S for the given elements: [Ne, m, Np].

        ``Q`` [E, m, D, Np], when given, is used as the gradient (the coupled system's
        unknown); otherwise Q = D(U) (the reduced system, C22 = 0)."""
        if elems is None:
            elems = torch.arange(self.E)
        elems = torch.as_tensor(elems, dtype=torch.int64)
        U = _t(U)
        allel, qidx = self._with_neighbours(elems)
        if Q is not None:
            Q = _t(Q)[allel]
        elif self.ph.has_viscous:
            if self.c22 != 0.0:
                raise ValueError("C22 != 0: Q is an unknown of the coupled system and must be given")
            Q = self.gradient(U, allel)
        else:
            Q = torch.zeros(len(allel), self.m, self.D, self.Np, dtype=DT)
        geo = self.geometry(elems)
        Ne = len(elems)
        acc = torch.zeros(Ne, self.m, self.Np, dtype=DT)
        acc_abs = torch.zeros(Ne, self.m, self.Np, dtype=DT)
        for n in range(self.D):
            ul, ql, outs, S1 = self._line_inputs(U, Q, elems, n, qidx)
            (uo0, qo0, b0, g0, h0), (uo1, qo1, b1, g1, h1) = outs
            b = self.resid_line_rhs(ul, ql, uo0, qo0, uo1, qo1, geo["ag"][n], geo["n0"][n], geo["n1"][n],
                                    S1, b0, b1, g0, g1, h0, h1)
            r = torch.cholesky_solve(b, self.Mchol)  # [Ne, NL, N1, m]
            rn = self.from_lines(r, n)
            acc += rn
            acc_abs += rn.abs()
        R = -acc / geo["J"][:, None, :]
        if self.source is not None:
            R = R + self.source[elems]
        if return_abs:
            mag = acc_abs / geo["J"][:, None, :].abs()
            if self.source is not None:
                mag = mag + self.source[elems].abs()
            return R, mag
        return R

    # ------------------------------------------------------------------ Jacobians
    def _slot_tables(self):
        """slot[row_node, n, t] = line slot of column position t on the row's direction-n line."""
        co = self.node_coords()
        tab = np.empty((self.Np, self.D, self.n1), dtype=np.int64)
        for a in range(self.Np):
            for n in range(self.D):
                for t in range(self.n1):
                    if n == 0:
                        tab[a, n, t] = t
                    elif t == co[a, n]:
                        tab[a, n, t] = co[a, 0]
                    else:
                        tab[a, n, t] = self.n1 + (n - 1) * self.p + (t if t < co[a, n] else t - 1)
        return tab

    def jacobian(self, U, elems=None, chunk=64):
        """Line-block K11 [Ne,Np,nslot11,m,m], K12 [Ne,Np,nslot12,m,m*D], K21 [Ne,Np,nslot21,D].

        K12 columns are ordered (c', d) like Q[m][D].  K21 is diagonal in the
        component index, so only its per-direction weight is stored.
        """
        if elems is None:
            elems = torch.arange(self.E)
        elems = torch.as_tensor(elems, dtype=torch.int64)
        U = _t(U)
        out11, out12, out21 = [], [], []
        for c0 in range(0, len(elems), chunk):
            k11, k12, k21 = self._jacobian_chunk(U, elems[c0:c0 + chunk])
            out11.append(k11)
            out12.append(k12)
            out21.append(k21)
        return torch.cat(out11), torch.cat(out12), torch.cat(out21)

    def _jacobian_chunk(self, U, elems):
        m, D, p, n1, NL = self.m, self.D, self.p, self.n1, self.NL
        Ne = len(elems)
        allel, qidx = self._with_neighbours(elems)
        if self.ph.has_viscous:
            Q = self.gradient(U, allel)
        else:
            Q = torch.zeros(len(allel), m, D, self.Np, dtype=DT)
        geo = self.geometry(elems)
        J = geo["J"]
        K11 = torch.zeros(Ne, self.Np, self.nslot11, m, m, dtype=DT)
        K12 = torch.zeros(Ne, self.Np, self.nslot12, m, m * D, dtype=DT)
        K21 = torch.zeros(Ne, self.Np, self.nslot21, D, dtype=DT)
        slot = torch.as_tensor(self._slot_tables())
        ar_e = torch.arange(Ne)
        for n in range(D):
            ul, ql, outs, S1 = self._line_inputs(U, Q, elems, n, qidx)
            (uo0, qo0, b0, g0, h0), (uo1, qo1, b1, g1, h1) = outs
            flat = lambda t: t.reshape((Ne * NL,) + t.shape[2:])
            args = [flat(x) for x in (ul, ql, uo0, qo0, uo1, qo1, geo["ag"][n], geo["n0"][n], geo["n1"][n],
                                      S1, b0, b1, g0, g1, h0, h1)]
            jf = vmap(jacfwd(self.resid_line_rhs, argnums=(0, 1, 2, 3, 4, 5)))
            jb = jf(*args)
            # solve with M along the row-position axis (axis 1 after the batch)
            def msolve(x):
                sh = x.shape
                return torch.cholesky_solve(x.reshape(sh[0], n1, -1), self.Mchol).reshape(sh)
            d_ul, d_ql, d_uo0, d_qo0, d_uo1, d_qo1 = [msolve(x).reshape((Ne, NL) + x.shape[1:]) for x in jb]
            # row node indices of each (line, position)
            rownode = self.to_lines(torch.arange(self.Np, dtype=DT)[None, None, :].expand(1, 1, self.Np), n)
            rownode = rownode[0, :, :, 0].long()  # [NL, N1]
            Jrow = J[:, rownode]  # [Ne, NL, N1]
            sc = (-1.0 / Jrow)[..., None, None]
            Sp = self.switch_plus[elems, n]
            for l in range(NL):
                for i in range(n1):
                    a = int(rownode[l, i])
                    for t in range(n1):
                        sl = int(slot[a, n, t])
                        K11[:, a, sl] += sc[:, l, i] * d_ul[:, l, i, :, t, :]
                        K12[:, a, sl] += sc[:, l, i] * d_ql[:, l, i, :, t, :, :].reshape(Ne, m, m * D)
                    base = self.nslot_line
                    for s, (duo, dqo, kd) in enumerate(((d_uo0, d_qo0, b0), (d_uo1, d_qo1, b1))):
                        keep = (kd[:, l] < 0).to(DT)[:, None, None]
                        K11[:, a, base + 2 * n + s] += keep * sc[:, l, i] * duo[:, l, i]
                        # K12 neighbour slot: the side whose switch is +1
                        side_plus = torch.where(Sp > 0, 1, 0)
                        mask = (side_plus == s).to(DT)[:, None, None] * keep
                        K12[:, a, base + n] += mask * sc[:, l, i] * dqo[:, l, i].reshape(Ne, m, m * D)
            # K21 weights: gradient operator is linear and component-diagonal
            K21 += self._k21_direction(elems, n, geo, slot, rownode)
        return K11, K12, K21

    def _k21_direction(self, elems, n, geo, slot, rownode):
        """Direction-n contribution to the K21 weights w[e, row, slot, d]."""
        D, p, n1, NL = self.D, self.p, self.n1, self.NL
        Ne = len(elems)
        W = torch.zeros(Ne, self.Np, self.nslot21, D, dtype=DT)
        Sp = self.switch_plus[elems, n]
        # derivative of the scalar line problem with unit data per column position
        ag, n0, n1v = geo["ag"][n], geo["n0"][n], geo["n1"][n]
        J = geo["J"]
        eye = torch.eye(n1, dtype=DT)
        k0 = self._kind(elems, n, 0)[:, None, None]
        k1 = self._kind(elems, n, 1)[:, None, None]
        for t in range(n1):
            ul = eye[t][None, None, :, None].expand(Ne, NL, n1, 1)
            zero = torch.zeros(Ne, NL, 1, dtype=DT)
            uin0, uin1 = ul[:, :, 0], ul[:, :, p]
            # uhat: inside where the face switch is +1 on interior faces and on Neumann / slip
            # faces (g_D, which does not depend on U, on Dirichlet faces)
            uh1 = torch.where(((Sp > 0)[:, None, None] & (k1 < 0)) | (k1 > 0), uin1, zero)
            uh0 = torch.where(((Sp < 0)[:, None, None] & (k0 < 0)) | (k0 > 0), uin0, zero)
            b = self.grad_line_rhs(ul, uh0, uh1, ag, n0, n1v)
            d = self._mass_solve(b)[..., 0, :]  # [Ne, NL, N1, D]
            for l in range(NL):
                for i in range(n1):
                    a = int(rownode[l, i])
                    W[:, a, int(slot[a, n, t])] += d[:, l, i] / J[:, a, None]
        # neighbour slot: the side whose switch is -1 takes uhat from outside
        for s in (0, 1):
            one = torch.ones(Ne, NL, 1, dtype=DT)
            zero = torch.zeros(Ne, NL, 1, dtype=DT)
            if s == 1:
                uh1 = torch.where((Sp < 0)[:, None, None], one, zero)
                uh0 = zero
            else:
                uh0 = torch.where((Sp > 0)[:, None, None], one, zero)
                uh1 = zero
            ul = torch.zeros(Ne, NL, n1, 1, dtype=DT)
            b = self.grad_line_rhs(ul, uh0, uh1, ag, n0, n1v)
            d = self._mass_solve(b)[..., 0, :]
            bnd = self.face_nbr[elems, 2 * n + s] < 0
            keep = (~bnd).to(DT)[:, None]
            for l in range(NL):
                for i in range(n1):
                    a = int(rownode[l, i])
                    W[:, a, self.nslot_line + n] += keep * d[:, l, i] / J[:, a, None]
        return W

    def k21(self, elems=None):
        """Weights of the linear gradient operator K21 = dD/dU: [Ne, Np, nslot21, D]."""
        if elems is None:
            elems = torch.arange(self.E)
        elems = torch.as_tensor(elems, dtype=torch.int64)
        geo = self.geometry(elems)
        slot = torch.as_tensor(self._slot_tables())
        W = torch.zeros(len(elems), self.Np, self.nslot21, self.D, dtype=DT)
        for n in range(self.D):
            rownode = self.to_lines(torch.arange(self.Np, dtype=DT)[None, None, :].expand(1, 1, self.Np), n)
            W += self._k21_direction(elems, n, geo, slot, rownode[0, :, :, 0].long())
        return W

    # ------------------------------------------------------------------ column maps
    def column_nodes(self, kind="K11"):
        """cols[e, a, slot] = global node index (e' * Np + node') of each slot, -1 if none."""
        co = self.node_coords()
        E, Np, D, p, n1 = self.E, self.Np, self.D, self.p, self.n1
        nsl = {"K11": self.nslot11, "K12": self.nslot12, "K21": self.nslot21}[kind]
        cols = np.full((E, Np, nsl), -1, dtype=np.int64)
        stride = [n1 ** d for d in range(D)]
        fn = self.face_nbr.numpy()
        nn = self.nbr_node.numpy()
        sp = self.switch_plus.numpy()
        tab = self._slot_tables()
        for a in range(Np):
            for n in range(D):
                for t in range(n1):
                    col = a + (t - co[a, n]) * stride[n]
                    cols[:, a, tab[a, n, t]] = np.arange(E) * Np + col
            for n in range(D):
                others = [d for d in range(D) if d != n]
                l = 0
                for d in reversed(others):
                    l = l * n1 + co[a, d]
                for s in (0, 1):
                    nb = fn[:, 2 * n + s]
                    node = nn[:, 2 * n + s, l]
                    g = np.where(nb >= 0, nb * Np + node, -1)
                    if kind == "K11":
                        cols[:, a, self.nslot_line + 2 * n + s] = g
                    elif kind == "K12":
                        side = np.where(sp[:, n] > 0, 1, 0)
                        cols[:, a, self.nslot_line + n] = np.where(side == s, g, cols[:, a, self.nslot_line + n])
                    else:
                        side = np.where(sp[:, n] < 0, 1, 0)
                        cols[:, a, self.nslot_line + n] = np.where(side == s, g, cols[:, a, self.nslot_line + n])
        return cols
