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
// One workgroup per element.  For each part (u, then q_{:,d} for d < D) and
// each direction, the m x m flux Jacobians at all Gauss points and line ends
// are formed in LDS; then one thread per (row node, component pair) contracts
// them into every slot of its block row.  The self slot sums the D directions
// in LDS, so each output is written exactly once, and consecutive threads
// write consecutive nodes of the [slot][c][c'][node] layout.
// Flux Jacobians: d/du by m forward-mode passes with one tangent each (the
// gradient held constant); d/dq exactly, since the viscous flux is linear in q
// with no q-free part (column k of dF/dq_{:,d} is F^vis(u, e_{k,d})) and the
// inviscid and penalty terms do not involve q.  The 1-D operators are copied
// to LDS because every lane indexes them by its own line position.
#include "ldg_dispatch.hpp"
#include "ldg_kernels.hpp"
#include "ldg_store.hpp"

namespace ldg {

template <int D, int P, int EQ>
struct JacLayout {
  static constexpr int N1 = P + 1, NG = n_gauss(P), NP = ipow(N1, D), NL = ipow(N1, D - 1);
  static constexpr int M = Eq<D, EQ>::M;
  static constexpr bool VIS = Eq<D, EQ>::VIS;
  static constexpr int QW = VIS ? M * D : 0;
  static constexpr int oU = 0;
  static constexpr int oQ = oU + M * NP;
  static constexpr int oX = oQ + QW * NP;
  static constexpr int oG = oX + D * NP;
  static constexpr int oJ = oG + D * D * NP;
  static constexpr int oA = oJ + NP;
  static constexpr int oFi = oA + NL * NG * M * M;
  static constexpr int oFo = oFi + NL * 2 * M * M;
  static constexpr int oOps = oFo + NL * 2 * M * M;  // copy of the 1-D operators
  static constexpr int oDiag = oOps + (int)(sizeof(LineOps) / sizeof(double));
  static constexpr int NITEM_ = (NP * M * M + NT_ELEM - 1) / NT_ELEM;
  static constexpr int ndoubles = oDiag + NITEM_ * NT_ELEM;  // per-thread self-slot sums
  static constexpr size_t bytes = sizeof(double) * ndoubles;
  static constexpr int NITEM = (NP * M * M + NT_ELEM - 1) / NT_ELEM;
  static constexpr int NS11 = D * P + 1 + 2 * D;
  static constexpr int NS12 = D * P + 1 + D;
};

template <int D, int N1>
__device__ __forceinline__ int line_slot(int n, int t, int tp) {
  // slot of column position tp on the row's direction-n line (row at position t), tp != t for n > 0
  return n == 0 ? tp : N1 + (n - 1) * (N1 - 1) + (tp < t ? tp : tp - 1);
}

// Parts [PART0, PART1) of the derivative passes: launched as two kernels, the
// state part (K11, with tangents) and the gradient parts (K12, plain doubles),
// so that each gets its own register allocation.
template <int D, int P, int EQ, int PR, int PART0, int PART1>
__global__ void __launch_bounds__(NT_ELEM) jac_kernel(LineOps ops_arg, MeshParams mp, const double* __restrict__ U,
                                                      const double* __restrict__ Q, void* __restrict__ K11,
                                                      void* __restrict__ K12) {
  using L = JacLayout<D, P, EQ>;
  constexpr int N1 = L::N1, NG = L::NG, NP = L::NP, NL = L::NL, M = L::M, QW = L::QW;
  constexpr bool INV = Eq<D, EQ>::INV, VIS = Eq<D, EQ>::VIS;
  constexpr int NSL = D * P + 1;
  typedef Dual<1> T1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* sm = reinterpret_cast<double*>(smem_raw);
  double* sU = sm + L::oU;
  double* sQ = sm + L::oQ;
  double* sX = sm + L::oX;
  double* sG = sm + L::oG;
  double* sJ = sm + L::oJ;
  double* sA = sm + L::oA;
  double* sFi = sm + L::oFi;
  double* sFo = sm + L::oFo;

  const int64_t e = blockIdx.x;
  const int tid = threadIdx.x;
  const int64_t NN = mp.E * NP;
  for (int i = tid; i < M * NP; i += NT_ELEM) sU[i] = U[e * M * NP + i];
  if constexpr (VIS)
    for (int i = tid; i < QW * NP; i += NT_ELEM) sQ[i] = Q[e * QW * NP + i];
  for (int i = tid; i < D * NP; i += NT_ELEM) sX[i] = mp.xyz[e * D * NP + i];
  // the 1-D operators are indexed by per-lane positions; from LDS that is a
  // plain load, from the kernel argument it would need private copies
  {
    const double* src = reinterpret_cast<const double*>(&ops_arg);
    for (int i = tid; i < (int)(sizeof(LineOps) / sizeof(double)); i += NT_ELEM) sm[L::oOps + i] = src[i];
  }
  const LineOps& ops = *reinterpret_cast<const LineOps*>(sm + L::oOps);
  __syncthreads();
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
  for (int i = tid; i < NP; i += NT_ELEM) {
    double G[D][D];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = 0; b < D; ++b) G[a][b] = sG[(a * D + b) * NP + i];
    sJ[i] = -1.0 / det<D>(G);  // row scaling -1/J
  }
  __syncthreads();

  constexpr int NPART = VIS ? 1 + D : 1;
  for (int part = PART0; part < (PART1 < NPART ? PART1 : NPART); ++part) {
    // self-slot sums over the D directions, one LDS entry per (item, thread):
    // kept out of registers, which the flux evaluations need
    double* diag = sm + L::oDiag;
#pragma unroll
    for (int q = 0; q < L::NITEM; ++q) diag[q * NT_ELEM + tid] = 0.0;
    const int dq = part - 1;  // derivative direction of q for part > 0
    for (int n = 0; n < D; ++n) {
      // ---- volume flux Jacobians at the Gauss points of every direction-n line
      for (int it = tid; it < NL * NG; it += NT_ELEM) {
        const int l = it / NG, g = it % NG;
        double G[D][D], an[D];
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
            G[a][b] = acc;
          }
        cofactor_row<D>(G, n, an);
        if (part == 0) {
          // the gradient enters the state derivatives as a constant
          double qd[VIS ? M * D : 1];
          if constexpr (VIS) {
#pragma unroll
            for (int k = 0; k < M * D; ++k) {
              double acc = 0.0;
#pragma unroll
              for (int t = 0; t < N1; ++t) acc += ops.I[g][t] * sQ[k * NP + line_node<D, N1>(n, l, t)];
              qd[k] = acc;
            }
          }
          // d f / d u, one state component per pass (single-tangent duals);
          // the gradient is a constant here
          double ud[M];
#pragma unroll
          for (int c = 0; c < M; ++c) {
            double acc = 0.0;
#pragma unroll
            for (int t = 0; t < N1; ++t) acc += ops.I[g][t] * sU[c * NP + line_node<D, N1>(n, l, t)];
            ud[c] = acc;
          }
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
            for (int c = 0; c < M; ++c) sA[((l * NG + g) * M + c) * M + k] = f[c].d[0];
          }
        } else if constexpr (VIS) {
          // d f / d q_{:,dq}: F^vis is linear in q with no q-free term, so
          // column k is F^vis(u, e_{k,dq}); the inviscid flux has no q
          double ud[M];
#pragma unroll
          for (int c = 0; c < M; ++c) {
            double acc = 0.0;
#pragma unroll
            for (int t = 0; t < N1; ++t) acc += ops.I[g][t] * sU[c * NP + line_node<D, N1>(n, l, t)];
            ud[c] = acc;
          }
#pragma unroll 1
          for (int k = 0; k < M; ++k) {
            double ek[M * D], fk[M];
#pragma unroll
            for (int j = 0; j < M * D; ++j) ek[j] = (j == k * D + dq) ? 1.0 : 0.0;
#pragma unroll
            for (int c = 0; c < M; ++c) fk[c] = 0.0;
            visc_flux_dot_add<D, EQ, double>(ud, ek, an, mp.gamma, mp.mu, mp.prandtl, fk);
#pragma unroll
            for (int c = 0; c < M; ++c) sA[((l * NG + g) * M + c) * M + k] = fk[c];
          }
        }
      }
      // ---- face flux Jacobians at both ends of every direction-n line
      for (int it = tid; it < NL * 2; it += NT_ELEM) {
        const int l = it / 2, s = it % 2;
        const int nin = line_node<D, N1>(n, l, s ? P : 0);
        double G[D][D], an[D], nrm[D];
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
          for (int b = 0; b < D; ++b) G[a][b] = sG[(a * D + b) * NP + nin];
        cofactor_row<D>(G, n, an);
#pragma unroll
        for (int d = 0; d < D; ++d) nrm[d] = s ? an[d] : -an[d];
        const int f = 2 * n + s;
        const int64_t nb = mp.face_nbr[e * 2 * D + f];
        const int kind = face_kind(nb);
        const bool bnd = nb < 0;
        const int Sp = mp.sw[e * D + n];
        const int S = s ? Sp : -Sp;
        double uin[M], uout[M], qin[M * D > 0 ? M * D : 1], qout[M * D > 0 ? M * D : 1];
#pragma unroll
        for (int c = 0; c < M; ++c) uin[c] = sU[c * NP + nin];
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
        if constexpr (VIS) {
          if (part == 0) {  // the gradient derivatives do not involve q itself
#pragma unroll
            for (int k = 0; k < M * D; ++k) {
              qin[k] = sQ[k * NP + nin];
              qout[k] = (!bnd && S > 0) ? Q[(nb * QW + k) * NP + nd] : qin[k];
            }
          }
        }
        // derivative with respect to the inside (side 0) and outside (side 1) variable
        const bool use_out = !bnd && S > 0;  // the side whose viscous flux the switch selects
        for (int side = 0; side < 2; ++side) {
          double* dst = (side == 0 ? sFi : sFo) + ((l * 2 + s) * M) * M;
          if (side == 1 && bnd) {
#pragma unroll
            for (int k = 0; k < M * M; ++k) dst[k] = 0.0;
            continue;
          }
          if (part == 0) {
            double qs[VIS ? M * D : 1];
#pragma unroll
            for (int k = 0; k < (VIS ? M * D : 1); ++k) qs[k] = VIS ? (use_out ? qout[k] : qin[k]) : 0.0;
            // one state component of this side per pass
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
              face_flux_point<D, EQ, T1, true, double>(ti, to, qs, nrm, S, kind, mp, F);
#pragma unroll
              for (int c = 0; c < M; ++c) dst[c * M + k] = F[c].d[0];
            }
          } else if constexpr (VIS) {
            // only the selected side's gradient enters the flux, linearly (and none on
            // Neumann faces and slip walls)
            if ((side == 1) != use_out || kind == BC_NEUMANN || kind == BC_SLIP) {
#pragma unroll
              for (int k = 0; k < M * M; ++k) dst[k] = 0.0;
              continue;
            }
            double us[M];
#pragma unroll
            for (int c = 0; c < M; ++c) us[c] = use_out ? uout[c] : uin[c];
#pragma unroll 1
            for (int k = 0; k < M; ++k) {
              double ek[M * D], fk[M];
#pragma unroll
              for (int j = 0; j < M * D; ++j) ek[j] = (j == k * D + dq) ? 1.0 : 0.0;
#pragma unroll
              for (int c = 0; c < M; ++c) fk[c] = 0.0;
              visc_flux_dot_add<D, EQ, double>(us, ek, nrm, mp.gamma, mp.mu, mp.prandtl, fk);
#pragma unroll
              for (int c = 0; c < M; ++c) dst[c * M + k] = fk[c];
            }
          }
        }
      }
      __syncthreads();
      // ---- contraction into the block rows
#pragma unroll 1
      for (int q = 0; q < L::NITEM; ++q) {
        const int item = tid + q * NT_ELEM;
        if (item < NP * M * M) {
          const int a = item % NP, cc = item / NP;
          const int c = cc / M, k = cc % M;
          int l, t;
          node_line<N1>(a, n, l, t);
          const double sc = sJ[a];
          const int64_t gn = e * NP + a;
          const int Sp = mp.sw[e * D + n];
#pragma unroll
          for (int tp = 0; tp < N1; ++tp) {
            double v = 0.0;
#pragma unroll
            for (int g = 0; g < NG; ++g) v -= ops.V[t][g] * ops.I[g][tp] * sA[((l * NG + g) * M + c) * M + k];
            if (tp == P) v += ops.L1[t] * sFi[((l * 2 + 1) * M + c) * M + k];
            if (tp == 0) v += ops.L0[t] * sFi[((l * 2 + 0) * M + c) * M + k];
            v *= sc;
            if (tp == t) {
              diag[q * NT_ELEM + tid] += v;
            } else {
              const int slot = line_slot<D, N1>(n, t, tp);
              if (part == 0)
                Store<PR>::put(K11, ((int64_t)(slot * M + c) * M + k) * NN + gn, v);
              else
                Store<PR>::put(K12, ((int64_t)(slot * M + c) * (M * D) + k * D + dq) * NN + gn, v);
            }
          }
          if (part == 0) {
            const double v1 = sc * ops.L1[t] * sFo[((l * 2 + 1) * M + c) * M + k];
            const double v0 = sc * ops.L0[t] * sFo[((l * 2 + 0) * M + c) * M + k];
            Store<PR>::put(K11, ((int64_t)((NSL + 2 * n + 1) * M + c) * M + k) * NN + gn, v1);
            Store<PR>::put(K11, ((int64_t)((NSL + 2 * n + 0) * M + c) * M + k) * NN + gn, v0);
          } else {
            const int s = Sp > 0 ? 1 : 0;
            const double v = sc * (s ? ops.L1[t] : ops.L0[t]) * sFo[((l * 2 + s) * M + c) * M + k];
            Store<PR>::put(K12, ((int64_t)((NSL + n) * M + c) * (M * D) + k * D + dq) * NN + gn, v);
          }
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < L::NITEM; ++q) {
      const int item = tid + q * NT_ELEM;
      if (item < NP * M * M) {
        const int a = item % NP, cc = item / NP;
        const int c = cc / M, k = cc % M;
        const int slot = a % N1;
        const int64_t gn = e * NP + a;
        if (part == 0)
          Store<PR>::put(K11, ((int64_t)(slot * M + c) * M + k) * NN + gn, diag[q * NT_ELEM + tid]);
        else
          Store<PR>::put(K12, ((int64_t)(slot * M + c) * (M * D) + k * D + dq) * NN + gn, diag[q * NT_ELEM + tid]);
      }
    }
  }
}

hipError_t launch_jacobian(const DevCtx& dc, const double* U, const double* Q, void* K11, void* K12, int prec) {
  LDG_DISPATCH(dc, {
    using L = JacLayout<D, P, EQ>;
    static_assert(L::bytes <= LDS_PER_CU, "assembly workspace must fit one CU's LDS");
    LDG_PREC_DISPATCH(prec, {
      auto k11 = jac_kernel<D, P, EQ, PR, 0, 1>;
      auto k12 = jac_kernel<D, P, EQ, PR, 1, 1 + D>;
      if (L::bytes > 65536) {
        hipError_t err =
            hipFuncSetAttribute((const void*)k11, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L::bytes);
        if (err == hipSuccess)
          err = hipFuncSetAttribute((const void*)k12, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L::bytes);
        if (err != hipSuccess) return err;
      }
      hipLaunchKernelGGL(k11, dim3((unsigned)dc.E), dim3(NT_ELEM), L::bytes, dc.stream, dc.ops, dc.mp, U, Q, K11, K12);
      if constexpr (Eq<D, EQ>::VIS)
        hipLaunchKernelGGL(k12, dim3((unsigned)dc.E), dim3(NT_ELEM), L::bytes, dc.stream, dc.ops, dc.mp, U, Q, K11,
                           K12);
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
