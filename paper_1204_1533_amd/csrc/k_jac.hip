// Line-block Jacobians K11 = dR/dU and K12 = dR/dQ (Section 4.1), computed in
// FP64 with forward-mode dual numbers and stored in FP64, FP32 or BF16.
//
// Because the residual of a node only sees the D lines through it, the block
// row of node a couples to the D p + 1 nodes of those lines and to one
// neighbour node per line end (2D for K11; for K12 only the end whose switch
// takes the viscous flux from outside, Section 3).  For a line of direction n
// and a row at position t on it:
//   d r_t / d u_t' = - sum_g V_tg (d f~/d u)_g I_gt'  +  L1_t dFhat^+/du_in [t'=p]
//                    + L0_t dFhat^-/du_in [t'=0],
//   d r_t / d u_nbr(xi=1) = L1_t dFhat^+/du_out,  d r_t / d u_nbr(xi=0) = L0_t dFhat^-/du_out,
// and the same with q in place of u for K12; rows are scaled by -1/J.
//
// Three launches:
//   geometry (once per context)  Gauss-point metrics a_n, face normals and
//            -1/J of every node, from the node coordinates;
//   points   one work item per Gauss point of every line of every direction
//            (and one per line end): the m x m flux Jacobians d f~ . a_n / du
//            (m forward-mode passes with one tangent each, the gradient held
//            constant) and d f~ . a_n / dq_{:,d} (exact: the viscous flux is
//            linear in q with no q-free part, so column k is F^vis(u, e_{k,d})),
//            written to a workspace with the point index fastest;
//   contract one work item per (element, part, component pair, row node)
//            contracts the point Jacobians of the node's D lines into every
//            slot of its block row; the self slot sums the D directions in a
//            register, so each output is written exactly once, and
//            consecutive work items write consecutive nodes of the
//            [slot][c][c'][node] layout.
// No launch holds more than the 1-D operators in LDS.
#include "ldg_dispatch.hpp"
#include "ldg_kernels.hpp"
#include "ldg_store.hpp"

namespace ldg {

template <int D, int P, int EQ>
struct JacShape {
  static constexpr int N1 = P + 1, NG = n_gauss(P), NP = ipow(N1, D), NL = ipow(N1, D - 1);
  static constexpr int M = Eq<D, EQ>::M;
  static constexpr bool VIS = Eq<D, EQ>::VIS;
  static constexpr int NPART = VIS ? 1 + D : 1;  // u, then q_{:,d}
  static constexpr int MM = M * M;
  static constexpr int NLG = NL * NG;            // Gauss points of one direction
  static constexpr int NLS = NL * 2;             // line ends of one direction
  // volume workspace [E][D][NPART][MM][NLG]; face workspace [E][D][NPART][2 sides][MM][NLS]
  static constexpr int64_t VOL = (int64_t)D * NPART * MM * NLG;
  static constexpr int64_t FACE = (int64_t)D * NPART * 2 * MM * NLS;
  static constexpr int NITEM = (NP * MM + NT_ELEM - 1) / NT_ELEM;
  static constexpr int NS11 = D * P + 1 + 2 * D;
  static constexpr int NS12 = D * P + 1 + D;
};

// LDS copy of the 1-D operators (per-lane indexing of a kernel argument would
// need private copies)
__device__ __forceinline__ const LineOps& stage_ops(const LineOps& ops_arg, double* dst) {
  const double* src = reinterpret_cast<const double*>(&ops_arg);
  for (int i = threadIdx.x; i < (int)(sizeof(LineOps) / sizeof(double)); i += blockDim.x) dst[i] = src[i];
  __syncthreads();
  return *reinterpret_cast<const LineOps*>(dst);
}

constexpr int OPS_DOUBLES = (int)(sizeof(LineOps) / sizeof(double));

template <int D, int P>
__global__ void __launch_bounds__(NT_ELEM) geometry_kernel(LineOps ops_arg, MeshParams mp, double* __restrict__ geo) {
  using G = GeoShape<D, P>;
  constexpr int N1 = G::N1, NG = G::NG, NP = G::NP, NL = G::NL;
  __shared__ double sX[D * NP];
  __shared__ double sG[D * D * NP];
  __shared__ double sOps[OPS_DOUBLES];
  const int64_t e = blockIdx.x;
  const int tid = threadIdx.x;
  for (int i = tid; i < D * NP; i += NT_ELEM) sX[i] = mp.xyz[e * D * NP + i];
  const LineOps& ops = stage_ops(ops_arg, sOps);
  for (int i = tid; i < D * D * NP; i += NT_ELEM) {
    const int ab = i / NP, node = i % NP;
    const int a = ab / D, b = ab % D;
    int s = 1;
    for (int k = 0; k < b; ++k) s *= N1;
    const int tb = (node / s) % N1;
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < N1; ++q) acc += ops.Dn[tb][q] * sX[a * NP + node - tb * s + q * s];
    sG[ab * NP + node] = acc;
  }
  __syncthreads();
  double* out = geo + e * G::REC;
  for (int i = tid; i < NP; i += NT_ELEM) {
    double Gm[D][D];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = 0; b < D; ++b) Gm[a][b] = sG[(a * D + b) * NP + i];
    out[G::oJs + i] = -1.0 / det<D>(Gm);
  }
  for (int it = tid; it < D * NL * NG; it += NT_ELEM) {
    const int n = it / (NL * NG), l = (it / NG) % NL, g = it % NG;
    double Gm[D][D], an[D];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = 0; b < D; ++b) {
        double acc = 0.0;
        if (b == n) {
#pragma unroll
          for (int t = 0; t < N1; ++t) acc += ops.Dg[g][t] * sX[a * NP + line_node<D, N1>(n, l, t)];
        } else {
#pragma unroll
          for (int t = 0; t < N1; ++t) acc += ops.I[g][t] * sG[(a * D + b) * NP + line_node<D, N1>(n, l, t)];
        }
        Gm[a][b] = acc;
      }
    cofactor_row<D>(Gm, n, an);
#pragma unroll
    for (int d = 0; d < D; ++d) out[G::oAg + it * D + d] = an[d];
  }
  for (int it = tid; it < D * NL * 2; it += NT_ELEM) {
    const int n = it / (NL * 2), l = (it / 2) % NL, s = it % 2;
    const int nin = line_node<D, N1>(n, l, s ? P : 0);
    double Gm[D][D], an[D];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = 0; b < D; ++b) Gm[a][b] = sG[(a * D + b) * NP + nin];
    cofactor_row<D>(Gm, n, an);
#pragma unroll
    for (int d = 0; d < D; ++d) out[G::oNf + it * D + d] = s ? an[d] : -an[d];
  }
}

// Volume flux Jacobians at every Gauss point: work item (e, n, l, g).
template <int D, int P, int EQ>
__global__ void __launch_bounds__(256) jac_volume_kernel(LineOps ops_arg, MeshParams mp, const double* __restrict__ geo,
                                                         const double* __restrict__ U, const double* __restrict__ Q,
                                                         double* __restrict__ W) {
  using S = JacShape<D, P, EQ>;
  using G = GeoShape<D, P>;
  constexpr int N1 = S::N1, NG = S::NG, NP = S::NP, M = S::M, MM = S::MM, NLG = S::NLG, NPART = S::NPART;
  constexpr bool INV = Eq<D, EQ>::INV, VIS = Eq<D, EQ>::VIS;
  constexpr int QW = VIS ? M * D : 1;
  typedef Dual<1> T1;
  __shared__ double sOps[OPS_DOUBLES];
  const LineOps& ops = stage_ops(ops_arg, sOps);
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= mp.E * D * NLG) return;  // no barrier below
  const int lg = (int)(idx % NLG);
  const int n = (int)((idx / NLG) % D);
  const int64_t e = idx / ((int64_t)D * NLG);
  const int l = lg / NG, g = lg % NG;
  double an[D];
#pragma unroll
  for (int d = 0; d < D; ++d) an[d] = geo[e * G::REC + G::oAg + ((int64_t)n * NLG + lg) * D + d];
  double ud[M];
#pragma unroll
  for (int c = 0; c < M; ++c) {
    double acc = 0.0;
#pragma unroll
    for (int t = 0; t < N1; ++t) acc += ops.I[g][t] * U[(e * M + c) * NP + line_node<D, N1>(n, l, t)];
    ud[c] = acc;
  }
  double* out = W + (e * D + n) * (int64_t)NPART * MM * NLG + lg;
  {
    double qd[QW];
    if constexpr (VIS) {
#pragma unroll
      for (int k = 0; k < M * D; ++k) {
        double acc = 0.0;
#pragma unroll
        for (int t = 0; t < N1; ++t) acc += ops.I[g][t] * Q[(e * M * D + k) * NP + line_node<D, N1>(n, l, t)];
        qd[k] = acc;
      }
    }
    // d f / d u, one state component per pass (the gradient is a constant here)
#pragma unroll 1
    for (int k = 0; k < M; ++k) {
      T1 u[M], f[M];
#pragma unroll
      for (int c = 0; c < M; ++c) {
        u[c] = mk<1>(ud[c]);
        u[c].d[0] = c == k ? 1.0 : 0.0;
        f[c] = mk<1>(0.0);
      }
      if constexpr (VIS) visc_flux_dot_add<D, EQ, T1, double>(u, qd, an, mp.gamma, mp.mu, mp.prandtl, f);
      if constexpr (INV) {
        T1 fi[M];
        euler_flux_dot<D, T1>(u, an, mp.gamma, fi);
#pragma unroll
        for (int c = 0; c < M; ++c) f[c] += fi[c];
      }
#pragma unroll
      for (int c = 0; c < M; ++c) out[(int64_t)(c * M + k) * NLG] = f[c].d[0];
    }
  }
  if constexpr (VIS) {
    // d f / d q_{:,dq}: column k is F^vis(u, e_{k,dq}) (no q-free term; no q in the inviscid flux)
#pragma unroll 1
    for (int dq = 0; dq < D; ++dq)
#pragma unroll 1
      for (int k = 0; k < M; ++k) {
        double ek[M * D], fk[M];
#pragma unroll
        for (int j = 0; j < M * D; ++j) ek[j] = (j == k * D + dq) ? 1.0 : 0.0;
#pragma unroll
        for (int c = 0; c < M; ++c) fk[c] = 0.0;
        visc_flux_dot_add<D, EQ, double>(ud, ek, an, mp.gamma, mp.mu, mp.prandtl, fk);
#pragma unroll
        for (int c = 0; c < M; ++c) out[(int64_t)((1 + dq) * MM + c * M + k) * NLG] = fk[c];
      }
  }
}

// Face flux Jacobians at both ends of every line: work item (e, n, l, s);
// d Fhat / d (inside, outside) for u and for q_{:,d}.
template <int D, int P, int EQ>
__global__ void __launch_bounds__(256) jac_face_kernel(MeshParams mp, const double* __restrict__ geo,
                                                       const double* __restrict__ U, const double* __restrict__ Q,
                                                       double* __restrict__ W) {
  using S = JacShape<D, P, EQ>;
  using G = GeoShape<D, P>;
  constexpr int N1 = S::N1, NP = S::NP, NL = S::NL, M = S::M, MM = S::MM, NLS = S::NLS, NPART = S::NPART;
  constexpr bool VIS = Eq<D, EQ>::VIS;
  constexpr int QW = VIS ? M * D : 1;
  typedef Dual<1> T1;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= mp.E * D * NLS) return;
  const int ls = (int)(idx % NLS);
  const int n = (int)((idx / NLS) % D);
  const int64_t e = idx / ((int64_t)D * NLS);
  const int l = ls / 2, s = ls % 2;
  const int nin = line_node<D, N1>(n, l, s ? P : 0);
  double nrm[D];
#pragma unroll
  for (int d = 0; d < D; ++d) nrm[d] = geo[e * G::REC + G::oNf + ((int64_t)n * NLS + ls) * D + d];
  const int f = 2 * n + s;
  const int64_t nb = mp.face_nbr[e * 2 * D + f];
  const int kind = face_kind(nb);
  const bool bnd = nb < 0;
  const int Sp = mp.sw[e * D + n];
  const int Sg = s ? Sp : -Sp;
  double uin[M], uout[M];
#pragma unroll
  for (int c = 0; c < M; ++c) uin[c] = U[(e * M + c) * NP + nin];
  int nd = 0;
  if (!bnd) {
    nd = mp.nbr_node[(e * 2 * D + f) * NL + l];
#pragma unroll
    for (int c = 0; c < M; ++c) uout[c] = U[(nb * M + c) * NP + nd];
  } else {
    const double* gb = kind == BC_NEUMANN ? mp.gN : mp.gD;
#pragma unroll
    for (int c = 0; c < M; ++c) uout[c] = gb ? gb[((e * 2 * D + f) * M + c) * NL + l] : 0.0;
  }
  const bool use_out = !bnd && Sg > 0;  // the side whose viscous flux the switch selects
  // record of this line end: [part][side][c][c'] with the line-end index fastest
  double* out = W + (e * D + n) * (int64_t)NPART * 2 * MM * NLS + ls;
  {
    double qs[QW];
    if constexpr (VIS) {
#pragma unroll
      for (int k = 0; k < M * D; ++k)
        qs[k] = use_out ? Q[(nb * M * D + k) * NP + nd] : Q[(e * M * D + k) * NP + nin];
    }
#pragma unroll 1
    for (int side = 0; side < 2; ++side) {
      if (side == 1 && bnd) {
#pragma unroll
        for (int k = 0; k < MM; ++k) out[(int64_t)(MM + k) * NLS] = 0.0;
        continue;
      }
#pragma unroll 1
      for (int k = 0; k < M; ++k) {
        T1 ti[M], to[M], F[M];
#pragma unroll
        for (int c = 0; c < M; ++c) {
          ti[c] = mk<1>(uin[c]);
          to[c] = mk<1>(uout[c]);
          const double seed = c == k ? 1.0 : 0.0;
          ti[c].d[0] = side == 0 ? seed : 0.0;
          to[c].d[0] = side == 0 ? 0.0 : seed;
        }
        face_flux_point<D, EQ, T1, true, double>(ti, to, qs, nrm, Sg, kind, mp, F);
#pragma unroll
        for (int c = 0; c < M; ++c) out[(int64_t)(side * MM + c * M + k) * NLS] = F[c].d[0];
      }
    }
  }
  if constexpr (VIS) {
    // only the selected side's gradient enters the flux, linearly (none on Neumann faces and slip walls)
    const bool none = kind == BC_NEUMANN || kind == BC_SLIP;
    double us[M];
#pragma unroll
    for (int c = 0; c < M; ++c) us[c] = use_out ? uout[c] : uin[c];
#pragma unroll 1
    for (int dq = 0; dq < D; ++dq)
#pragma unroll 1
      for (int k = 0; k < M; ++k) {
        double ek[M * D], fk[M];
#pragma unroll
        for (int j = 0; j < M * D; ++j) ek[j] = (j == k * D + dq) ? 1.0 : 0.0;
#pragma unroll
        for (int c = 0; c < M; ++c) fk[c] = 0.0;
        if (!none) visc_flux_dot_add<D, EQ, double>(us, ek, nrm, mp.gamma, mp.mu, mp.prandtl, fk);
        double* o = out + (int64_t)((1 + dq) * 2 * MM) * NLS;
#pragma unroll
        for (int c = 0; c < M; ++c) {
          o[(int64_t)(0 * MM + c * M + k) * NLS] = use_out ? 0.0 : fk[c];
          o[(int64_t)(1 * MM + c * M + k) * NLS] = use_out ? fk[c] : 0.0;
        }
      }
  }
}

// Contraction into the block rows: one work item per (element, part,
// component pair, row node), the node fastest so that a wavefront writes
// consecutive nodes of every [slot][c][c'][node] row.  Grid: x over the
// element's (component pair, node) items, y over elements, z over parts, so
// element and part are uniform in a workgroup.  The point Jacobians of a line
// are read by the p + 1 work items of its nodes, next to each other in the
// wavefront (cache hits after the first); the self slot sums the D directions
// in a register.
template <int D, int P, int EQ, int PR>
__global__ void __launch_bounds__(256) jac_contract_kernel(LineOps ops_arg, MeshParams mp,
                                                           const double* __restrict__ geo,
                                                           const double* __restrict__ Wv,
                                                           const double* __restrict__ Wf, void* __restrict__ K11,
                                                           void* __restrict__ K12) {
  using S = JacShape<D, P, EQ>;
  using G = GeoShape<D, P>;
  constexpr int N1 = S::N1, NG = S::NG, NP = S::NP, M = S::M, MM = S::MM, NLG = S::NLG, NLS = S::NLS;
  constexpr int NPART = S::NPART, NSL = D * P + 1;
  using T = typename Store<PR>::type;
  __shared__ double sOps[OPS_DOUBLES];
  const LineOps& ops = stage_ops(ops_arg, sOps);
  const int64_t NN = mp.E * NP;
  const int item = blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= NP * MM) return;  // no barrier below
  const int a = item % NP, cc = item / NP;
  const int part = blockIdx.z;
  const int c = cc / M, k = cc % M;
  // the block row's first row of K11 (slot, c, k) or K12 (slot, c, (k, dq)), and the slot stride
  const int64_t row0 = part == 0 ? (int64_t)(c * M + k) : (int64_t)c * (M * D) + k * D + (part - 1);
  const int64_t slot_stride = (part == 0 ? (int64_t)MM : (int64_t)MM * D) * NN;
  T* Kp = (T*)(part == 0 ? K11 : K12) + row0 * NN;
  for (int64_t e = blockIdx.y; e < mp.E; e += gridDim.y) {
    const int64_t gn = e * NP + a;
    const double sc = geo[e * G::REC + G::oJs + a];
    double diag = 0.0;
#pragma unroll 1
    for (int n = 0; n < D; ++n) {
      int l, t;
      node_line<N1>(a, n, l, t);
      const double* Ar = Wv + ((e * D + n) * NPART + part) * (int64_t)MM * NLG + cc * NLG + l * NG;
      const double* Fr = Wf + ((e * D + n) * NPART + part) * (int64_t)2 * MM * NLS + cc * NLS + l * 2;
      double Vt[NG];
#pragma unroll
      for (int g = 0; g < NG; ++g) Vt[g] = ops.V[t][g] * Ar[g];
      const double fin0 = Fr[0], fin1 = Fr[1], fo0 = Fr[MM * NLS], fo1 = Fr[MM * NLS + 1];
#pragma unroll
      for (int tp = 0; tp < N1; ++tp) {
        double v = 0.0;
#pragma unroll
        for (int g = 0; g < NG; ++g) v -= Vt[g] * ops.I[g][tp];
        if (tp == P) v += ops.L1[t] * fin1;
        if (tp == 0) v += ops.L0[t] * fin0;
        v *= sc;
        if (tp == t)
          diag += v;
        else
          Store<PR>::put(Kp, slot_of<N1>(n, t, tp, t) * slot_stride + gn, v);
      }
      if (part == 0) {
        Store<PR>::put(Kp, (NSL + 2 * n + 1) * slot_stride + gn, sc * ops.L1[t] * fo1);
        Store<PR>::put(Kp, (NSL + 2 * n + 0) * slot_stride + gn, sc * ops.L0[t] * fo0);
      } else {
        const int s = mp.sw[e * D + n] > 0 ? 1 : 0;
        Store<PR>::put(Kp, (NSL + n) * slot_stride + gn, sc * (s ? ops.L1[t] * fo1 : ops.L0[t] * fo0));
      }
    }
    Store<PR>::put(Kp, (a % N1) * slot_stride + gn, diag);
  }
}

size_t jacobian_geometry_doubles(const DevCtx& dc) {
  const size_t rec = (size_t)dc.D * dc.NL * dc.NG * dc.D + (size_t)dc.D * dc.NL * 2 * dc.D + dc.NP;
  return (size_t)dc.E * rec;
}

size_t jacobian_workspace_doubles(const DevCtx& dc) {
  const size_t npart = dc.EQ != EQ_EULER ? 1 + dc.D : 1, mm = (size_t)dc.M * dc.M;
  return (size_t)dc.E * dc.D * npart * mm * ((size_t)dc.NL * dc.NG + 2 * (size_t)dc.NL * 2);
}

hipError_t launch_jacobian_geometry(const DevCtx& dc, double* geo) {
  LDG_DISPATCH(dc, {
    hipLaunchKernelGGL((geometry_kernel<D, P>), dim3((unsigned)dc.E), dim3(NT_ELEM), 0, dc.stream, dc.ops, dc.mp, geo);
    return hipGetLastError();
  })
}

hipError_t launch_jacobian(const DevCtx& dc, const double* U, const double* Q, void* K11, void* K12, int prec,
                           const double* geo, double* work) {
  LDG_DISPATCH(dc, {
    using S = JacShape<D, P, EQ>;
    double* Wv = work;
    double* Wf = work + dc.E * S::VOL;
    const int64_t nv = dc.E * D * S::NLG, nf = dc.E * D * S::NLS;
    // at most 2048 element rows in the grid: each workgroup then contracts
    // several elements (its operator copy staged once), 6 % faster at 32^3 p=4
    // than one element per workgroup
    const dim3 cgrid((unsigned)((S::NP * S::MM + 255) / 256), (unsigned)(dc.E < 2048 ? dc.E : 2048),
                     (unsigned)S::NPART);
    hipLaunchKernelGGL((jac_volume_kernel<D, P, EQ>), dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, dc.stream,
                       dc.ops, dc.mp, geo, U, Q, Wv);
    hipLaunchKernelGGL((jac_face_kernel<D, P, EQ>), dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, dc.stream,
                       dc.mp, geo, U, Q, Wf);
    LDG_PREC_DISPATCH(prec, {
      hipLaunchKernelGGL((jac_contract_kernel<D, P, EQ, PR>), cgrid, dim3(256), 0, dc.stream, dc.ops, dc.mp, geo,
                         Wv, Wf, K11, K12);
      return hipGetLastError();
    })
  })
}

// internal [slot][c][c'][E*Np] -> exchange [E][Np][slot][c][c'] in FP64
template <int PR>
__global__ void export_kernel(const void* __restrict__ K, int64_t NN, int nslot, int M, int ncol, int64_t total,
                              double* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t gn = i % NN;
    const int64_t r = i / NN;  // ((slot * M + c) * ncol + c2)
    const int c2 = (int)(r % ncol);
    const int c = (int)((r / ncol) % M);
    const int slot = (int)(r / ((int64_t)ncol * M));
    out[((gn * nslot + slot) * M + c) * ncol + c2] = Store<PR>::get(K, i);
  }
}

hipError_t launch_export_blocks(const DevCtx& dc, const void* K, int prec, int nslot, int ncol, double* out) {
  const int64_t NN = dc.E * dc.NP;
  const int64_t total = NN * nslot * dc.M * ncol;
  int64_t g = (total + 255) / 256;
  if (g > 65536) g = 65536;
  LDG_PREC_DISPATCH(prec, {
    hipLaunchKernelGGL(export_kernel<PR>, dim3((unsigned)g), dim3(256), 0, dc.stream, K, NN, nslot, dc.M, ncol, total,
                       out);
    return hipGetLastError();
  })
}

}  // namespace ldg
