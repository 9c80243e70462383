// Residual R = F(U) and LDG gradient Q = D(U) of the line-DG scheme.
//
// One workgroup owns EPB elements.  Each element's nodal state is staged in
// LDS, the geometry (Gauss-point metrics a_n = J G^{-T} N_n of eq. contraflux,
// exact for the Q_p map, line-end normals and 1/J) is read from the record
// computed once per context; every reference line of every direction is then
// processed from LDS:
//   * Gauss phase (one work item per line and Gauss point): interpolate the
//     state to the point and form the contravariant flux F . a_n;
//   * face phase (one work item per line end): the point flux at the face
//     node with the coinciding node of the neighbour (Riemann + LDG switch,
//     Section 3), or the boundary flux of the face's kind (Dirichlet,
//     Neumann, slip wall);
//   * projection (one work item per node and component): the 1-D Galerkin
//     solution r_i = L1_i Fhat^+ + L0_i Fhat^- - sum_g V_ig f~_g of eq.
//     galerkinscheme2 with the mass solve folded into L0, L1, V, summed over
//     the D lines through the node and scaled by -1/J (eq. semidisc).
// The only global reads besides the element's own contiguous block are one
// neighbour node per line end.
#include <type_traits>

#include "ldg_dispatch.hpp"
#include "ldg_kernels.hpp"

namespace ldg {

template <class T> struct IO;
template <> struct IO<double> {
  static __device__ __forceinline__ double load(const double* a, const double*, int64_t i) { return a[i]; }
};
template <> struct IO<Dual<1>> {
  static __device__ __forceinline__ Dual<1> load(const double* a, const double* t, int64_t i) {
    Dual<1> r;
    r.v = a[i];
    r.d[0] = t[i];
    return r;
  }
};
__device__ __forceinline__ double tangent_or_value(double x) { return x; }
__device__ __forceinline__ double tangent_or_value(const Dual<1>& x) { return x.d[0]; }

// Geometry (Gauss-point metrics a_n, line-end normals, -1/J) comes from the
// per-element record computed once per context from the node coordinates
// (GeoShape, geometry_kernel).

// --------------------------------------------------------------------------- residual
// Same organisation as the gradient kernel below: directions one after
// another, each thread owns fixed (element, component, node) outputs and
// accumulates the D line contributions in registers.
template <int D, int P, int EQ, class T>
struct ResidLayout {
  static constexpr int N1 = P + 1, NG = n_gauss(P), NP = ipow(N1, D), NL = ipow(N1, D - 1);
  static constexpr int M = Eq<D, EQ>::M;
  static constexpr bool VIS = Eq<D, EQ>::VIS;
  static constexpr int EPB = elems_per_block(NP, M);
  static constexpr int QW = VIS ? M * D : 0;
  // byte offsets (T arrays first, then doubles; all multiples of 16)
  static constexpr size_t oU = 0;
  static constexpr size_t oQ = oU + sizeof(T) * EPB * M * NP;
  static constexpr int NW = M + QW;  // state and gradient components interpolated to a Gauss point
  static constexpr size_t oF = oQ + sizeof(T) * EPB * QW * NP;
  static constexpr size_t oH = oF + sizeof(T) * EPB * NL * NG * M;
  // The dual-number (tangent) variant stages the Gauss-point interpolants and
  // metrics of a direction in LDS in a phase of their own; the FP64 residual
  // interpolates inside its Gauss phase (fewer barriers; measured faster for
  // FP64 and slower for the dual numbers, whose registers it then exhausts).
  static constexpr bool STAGE = !std::is_same<T, double>::value;
  static constexpr size_t oW = oH + sizeof(T) * EPB * NL * 2 * M;
  static constexpr size_t oJ = oW + (STAGE ? sizeof(T) * EPB * NL * NG * NW : 0);
  static constexpr size_t oA = oJ + sizeof(double) * EPB * NP;
  static constexpr size_t bytes = oA + (STAGE ? sizeof(double) * EPB * NL * NG * D : 0);
  static constexpr int NITEM = (EPB * M * NP + NT_ELEM - 1) / NT_ELEM;
};

template <int D, int P, int EQ, class T>
__global__ void __launch_bounds__(NT_ELEM) resid_kernel(LineOps ops, MeshParams mp, const double* __restrict__ U,
                                                        const double* __restrict__ Ut, const double* __restrict__ Q,
                                                        const double* __restrict__ Qt, double* __restrict__ R) {
  using L = ResidLayout<D, P, EQ, T>;
  using GR = GeoShape<D, P>;
  constexpr int N1 = L::N1, NG = L::NG, NP = L::NP, NL = L::NL, M = L::M, EPB = L::EPB, QW = L::QW;
  constexpr bool INV = Eq<D, EQ>::INV, VIS = Eq<D, EQ>::VIS;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sU = reinterpret_cast<T*>(smem_raw + L::oU);
  T* sQ = reinterpret_cast<T*>(smem_raw + L::oQ);
  T* sF = reinterpret_cast<T*>(smem_raw + L::oF);
  T* sH = reinterpret_cast<T*>(smem_raw + L::oH);
  double* sJ = reinterpret_cast<double*>(smem_raw + L::oJ);
  T* sWg = reinterpret_cast<T*>(smem_raw + L::oW);
  double* sAg = reinterpret_cast<double*>(smem_raw + L::oA);
  constexpr int NW = L::NW;

  const int64_t e0 = xcd_block(blockIdx.x, gridDim.x) * EPB;
  const int ne = (int)min((int64_t)EPB, mp.E - e0);
  const int tid = threadIdx.x;

  for (int i = tid; i < ne * M * NP; i += NT_ELEM) sU[i] = IO<T>::load(U, Ut, e0 * M * NP + i);
  if constexpr (VIS)
    for (int i = tid; i < ne * QW * NP; i += NT_ELEM) sQ[i] = IO<T>::load(Q, Qt, e0 * QW * NP + i);
  // -1/J of the nodes from the geometry record
  for (int i = tid; i < ne * NP; i += NT_ELEM) sJ[i] = mp.geo[(e0 + i / NP) * GR::REC + GR::oJs + i % NP];
  __syncthreads();
  T acc[L::NITEM];
#pragma unroll
  for (int q = 0; q < L::NITEM; ++q) acc[q] = cst<T>(0.0);

#pragma unroll
  for (int n = 0; n < D; ++n) {
    if constexpr (L::STAGE) {
      // interpolation phase: state, gradient and non-unit normal a_n at every Gauss point
      for (int i = tid; i < ne * NL * NG * NW; i += NT_ELEM) {
        const int k = i % NW, pt = i / NW;
        const int e = pt / (NL * NG), l = (pt / NG) % NL, g = pt % NG;
        const T* src = k < M ? sU + (e * M + k) * NP : sQ + (e * QW + (k - M)) * NP;
        T a = cst<T>(0.0);
#pragma unroll
        for (int t = 0; t < N1; ++t) a += ops.I[g][t] * src[line_node<D, N1>(n, l, t)];
        sWg[i] = a;
      }
      for (int i = tid; i < ne * NL * NG; i += NT_ELEM) {
        const int e = i / (NL * NG), lg = i % (NL * NG);
#pragma unroll
        for (int d = 0; d < D; ++d) sAg[i * D + d] = mp.geo[(e0 + e) * GR::REC + GR::oAg + (n * NL * NG + lg) * D + d];
      }
      __syncthreads();
      // Gauss phase: contravariant flux F . a_n at every Gauss point of the direction-n lines
      for (int i = tid; i < ne * NL * NG; i += NT_ELEM) {
        double an[D];
#pragma unroll
        for (int d = 0; d < D; ++d) an[d] = sAg[i * D + d];
        const T* w = sWg + i * NW;
        T ug[M];
#pragma unroll
        for (int c = 0; c < M; ++c) ug[c] = w[c];
        T f[M];
#pragma unroll
        for (int c = 0; c < M; ++c) f[c] = cst<T>(0.0);
        if constexpr (INV) euler_flux_dot<D, T>(ug, an, mp.gamma, f);
        if constexpr (VIS) {
          T qg[M * D];
#pragma unroll
          for (int c = 0; c < M * D; ++c) qg[c] = w[M + c];
          visc_flux_dot_add<D, EQ, T>(ug, qg, an, mp.gamma, mp.mu, mp.prandtl, f);
        }
#pragma unroll
        for (int c = 0; c < M; ++c) sF[i * M + c] = f[c];
      }
    } else {
      // Gauss phase: state and gradient interpolated to the point, the non-unit
      // normal a_n from the geometry record, and the contravariant flux F . a_n
      for (int i = tid; i < ne * NL * NG; i += NT_ELEM) {
        const int e = i / (NL * NG), l = (i / NG) % NL, g = i % NG;
        double an[D];
#pragma unroll
        for (int d = 0; d < D; ++d)
          an[d] = mp.geo[(e0 + e) * GR::REC + GR::oAg + (n * NL * NG + l * NG + g) * D + d];
        T ug[M];
#pragma unroll
        for (int c = 0; c < M; ++c) {
          T a = cst<T>(0.0);
#pragma unroll
          for (int t = 0; t < N1; ++t) a += ops.I[g][t] * sU[(e * M + c) * NP + line_node<D, N1>(n, l, t)];
          ug[c] = a;
        }
        T f[M];
#pragma unroll
        for (int c = 0; c < M; ++c) f[c] = cst<T>(0.0);
        if constexpr (INV) euler_flux_dot<D, T>(ug, an, mp.gamma, f);
        if constexpr (VIS) {
          T qg[M * D];
#pragma unroll
          for (int k = 0; k < M * D; ++k) {
            T a = cst<T>(0.0);
#pragma unroll
            for (int t = 0; t < N1; ++t) a += ops.I[g][t] * sQ[(e * QW + k) * NP + line_node<D, N1>(n, l, t)];
            qg[k] = a;
          }
          visc_flux_dot_add<D, EQ, T>(ug, qg, an, mp.gamma, mp.mu, mp.prandtl, f);
        }
#pragma unroll
        for (int c = 0; c < M; ++c) sF[i * M + c] = f[c];
      }
    }
    // face phase: point fluxes at both ends of every direction-n line
    for (int i = tid; i < ne * NL * 2; i += NT_ELEM) {
      const int e = i / (NL * 2), l = (i / 2) % NL, s = i % 2;
      const int64_t eg = e0 + e;
      const int nin = line_node<D, N1>(n, l, s ? P : 0);
      double nrm[D];  // outward non-unit normal of the line end
#pragma unroll
      for (int d = 0; d < D; ++d) nrm[d] = mp.geo[eg * GR::REC + GR::oNf + (n * NL * 2 + l * 2 + s) * D + d];
      const int f = 2 * n + s;
      const int64_t nb = mp.face_nbr[eg * 2 * D + f];
      const int kind = face_kind(nb);
      T uin[M], uout[M];
#pragma unroll
      for (int c = 0; c < M; ++c) uin[c] = sU[(e * M + c) * NP + nin];
      int nd = 0;
      if (kind == BC_INTERIOR) {
        nd = mp.nbr_node[(eg * 2 * D + f) * NL + l];
#pragma unroll
        for (int c = 0; c < M; ++c) uout[c] = IO<T>::load(U, Ut, (nb * M + c) * NP + nd);
      } else {
        // boundary data of the face's kind (unused on slip walls)
        const double* gb = kind == BC_NEUMANN ? mp.gN : mp.gD;
#pragma unroll
        for (int c = 0; c < M; ++c) uout[c] = cst<T>(gb ? gb[((eg * 2 * D + f) * M + c) * NL + l] : 0.0);
      }
      T F[M];
      if constexpr (VIS) {
        const int Sp = mp.sw[eg * D + n];
        const int S = s ? Sp : -Sp;
        T qsel[M * D];
        if (kind == BC_INTERIOR && S > 0) {
#pragma unroll
          for (int c = 0; c < M * D; ++c) qsel[c] = IO<T>::load(Q, Qt, (nb * QW + c) * NP + nd);
        } else {
#pragma unroll
          for (int c = 0; c < M * D; ++c) qsel[c] = sQ[(e * QW + c) * NP + nin];
        }
        face_flux_point<D, EQ, T>(uin, uout, qsel, nrm, S, kind, mp, F);
      } else {
        face_flux_point<D, EQ, T>(uin, uout, uin, nrm, 1, kind, mp, F);
      }
#pragma unroll
      for (int c = 0; c < M; ++c) sH[i * M + c] = F[c];
    }
    __syncthreads();
    // projection of this direction's line problems onto the owned outputs
#pragma unroll
    for (int q = 0; q < L::NITEM; ++q) {
      const int i = tid + q * NT_ELEM;
      if (i < ne * M * NP) {
        const int e = i / (M * NP), r = i % (M * NP);
        const int c = r / NP, node = r % NP;
        int l, t;
        node_line<N1>(node, n, l, t);
        const T* h = sH + (e * NL + l) * 2 * M;
        T a = ops.L1[t] * h[M + c] + ops.L0[t] * h[c];
        const T* fl = sF + (e * NL + l) * NG * M;
#pragma unroll
        for (int g = 0; g < NG; ++g) a -= ops.V[t][g] * fl[g * M + c];
        acc[q] += a;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < L::NITEM; ++q) {
    const int i = tid + q * NT_ELEM;
    if (i < ne * M * NP) {
      const int e = i / (M * NP), node = i % NP;
      const int64_t gi = e0 * M * NP + i;
      double out = tangent_or_value(acc[q]) * sJ[e * NP + node];
      if constexpr (sizeof(T) == sizeof(double)) {
        if (mp.S) out += mp.S[gi];
      }
      R[gi] = out;
    }
  }
}

// --------------------------------------------------------------------------- gradient
// Directions are processed one after another with compile-time indexing; each
// thread owns fixed output entries (element, component, derivative, node) and
// accumulates the D line contributions in registers, so only one direction's
// Gauss-point and face data live in LDS at a time.
template <int D, int P, int EQ>
struct GradLayout {
  static constexpr int N1 = P + 1, NG = n_gauss(P), NP = ipow(N1, D), NL = ipow(N1, D - 1);
  static constexpr int M = Eq<D, EQ>::M;
  static constexpr int EPB = elems_per_block(NP, M);
  static constexpr int oU = 0;
  static constexpr int oJ = oU + EPB * M * NP;
  static constexpr int oUg = oJ + EPB * NP;
  static constexpr int oAg = oUg + EPB * NL * NG * M;
  static constexpr int oUh = oAg + EPB * NL * NG * D;
  static constexpr int oNh = oUh + EPB * NL * 2 * M;
  static constexpr int ndoubles = oNh + EPB * NL * 2 * D;
  static constexpr size_t bytes = 8 * (size_t)ndoubles;
  static constexpr int NOUT = EPB * M * D * NP;
  static constexpr int NITEM = (NOUT + NT_ELEM - 1) / NT_ELEM;
};

// C22: the trace carries the C22 jump of the normal viscous flux of Qc (the
// coupled system); instantiated only where that system is solved
template <int D, int P, int EQ, bool C22>
__global__ void __launch_bounds__(NT_ELEM) grad_kernel(LineOps ops, MeshParams mp, const double* __restrict__ U,
                                                       double* __restrict__ Q, int homogeneous,
                                                       const double* __restrict__ Qc) {
  using L = GradLayout<D, P, EQ>;
  using GR = GeoShape<D, P>;
  constexpr int N1 = L::N1, NG = L::NG, NP = L::NP, NL = L::NL, M = L::M, EPB = L::EPB;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* sm = reinterpret_cast<double*>(smem_raw);
  double* sU = sm + L::oU;
  double* sJ = sm + L::oJ;
  double* sUg = sm + L::oUg;
  double* sAg = sm + L::oAg;
  double* sUh = sm + L::oUh;
  double* sNh = sm + L::oNh;

  const int64_t e0 = xcd_block(blockIdx.x, gridDim.x) * EPB;
  const int ne = (int)min((int64_t)EPB, mp.E - e0);
  const int tid = threadIdx.x;
  for (int i = tid; i < ne * M * NP; i += NT_ELEM) sU[i] = U[e0 * M * NP + i];
  // 1/J of the nodes (the record holds -1/J)
  for (int i = tid; i < ne * NP; i += NT_ELEM) sJ[i] = -mp.geo[(e0 + i / NP) * GR::REC + GR::oJs + i % NP];
  __syncthreads();
  double acc[L::NITEM];
#pragma unroll
  for (int q = 0; q < L::NITEM; ++q) acc[q] = 0.0;
#pragma unroll
  for (int n = 0; n < D; ++n) {
    for (int i = tid; i < ne * NL * NG; i += NT_ELEM) {
      const int e = i / (NL * NG), l = (i / NG) % NL, g = i % NG;
#pragma unroll
      for (int d = 0; d < D; ++d)
        sAg[i * D + d] = mp.geo[(e0 + e) * GR::REC + GR::oAg + (n * NL * NG + l * NG + g) * D + d];
#pragma unroll
      for (int c = 0; c < M; ++c) {
        double a = 0.0;
#pragma unroll
        for (int t = 0; t < N1; ++t) a += ops.I[g][t] * sU[(e * M + c) * NP + line_node<D, N1>(n, l, t)];
        sUg[i * M + c] = a;
      }
    }
    for (int i = tid; i < ne * NL * 2; i += NT_ELEM) {
      const int e = i / (NL * 2), l = (i / 2) % NL, s = i % 2;
      const int64_t eg = e0 + e;
      const int nin = line_node<D, N1>(n, l, s ? P : 0);
#pragma unroll
      for (int d = 0; d < D; ++d) sNh[i * D + d] = mp.geo[eg * GR::REC + GR::oNf + (n * NL * 2 + l * 2 + s) * D + d];
      const int f = 2 * n + s;
      const int64_t nb = mp.face_nbr[eg * 2 * D + f];
      const int kind = face_kind(nb);
      const int Sp = mp.sw[eg * D + n];
      const int S = s ? Sp : -Sp;
      if (kind == BC_DIRICHLET) {
#pragma unroll
        for (int c = 0; c < M; ++c)
          sUh[i * M + c] = (homogeneous || !mp.gD) ? 0.0 : mp.gD[((eg * 2 * D + f) * M + c) * NL + l];
      } else if (kind != BC_INTERIOR || S > 0) {
        // the inside trace: switch +1, or a Neumann face / slip wall
#pragma unroll
        for (int c = 0; c < M; ++c) sUh[i * M + c] = sU[(e * M + c) * NP + nin];
      } else {
        const int nd = mp.nbr_node[(eg * 2 * D + f) * NL + l];
#pragma unroll
        for (int c = 0; c < M; ++c) sUh[i * M + c] = U[(nb * M + c) * NP + nd];
      }
      if constexpr (C22) {
        if (kind == BC_INTERIOR || kind == BC_NEUMANN) {
          // C22 [[F . nbar]] with the inside as the positive side: interior faces
          // (F_in - F_out) . nbar, Neumann faces F_in . nbar - g_N (nbar the unit outward normal)
          double nbar[D], nn = 0.0;
#pragma unroll
          for (int d = 0; d < D; ++d) nn += sNh[i * D + d] * sNh[i * D + d];
          nn = 1.0 / sqrt(nn);
#pragma unroll
          for (int d = 0; d < D; ++d) nbar[d] = sNh[i * D + d] * nn;
          double uin[M], qin[M * D], Fin[M], Fout[M];
#pragma unroll
          for (int c = 0; c < M; ++c) {
            uin[c] = sU[(e * M + c) * NP + nin];
            Fin[c] = 0.0;
            Fout[c] = 0.0;
          }
#pragma unroll
          for (int k = 0; k < M * D; ++k) qin[k] = Qc[(eg * M * D + k) * NP + nin];
          visc_flux_dot_add<D, EQ, double>(uin, qin, nbar, mp.gamma, mp.mu, mp.prandtl, Fin);
          if (kind == BC_INTERIOR) {
            const int nd = mp.nbr_node[(eg * 2 * D + f) * NL + l];
            double uout[M], qout[M * D];
#pragma unroll
            for (int c = 0; c < M; ++c) uout[c] = U[(nb * M + c) * NP + nd];
#pragma unroll
            for (int k = 0; k < M * D; ++k) qout[k] = Qc[(nb * M * D + k) * NP + nd];
            visc_flux_dot_add<D, EQ, double>(uout, qout, nbar, mp.gamma, mp.mu, mp.prandtl, Fout);
          } else if (!homogeneous && mp.gN) {
#pragma unroll
            for (int c = 0; c < M; ++c) Fout[c] = mp.gN[((eg * 2 * D + f) * M + c) * NL + l];
          }
#pragma unroll
          for (int c = 0; c < M; ++c) sUh[i * M + c] += mp.c22 * (Fin[c] - Fout[c]);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < L::NITEM; ++q) {
      const int i = tid + q * NT_ELEM;
      if (i < ne * M * D * NP) {
        const int e = i / (M * D * NP), r = i % (M * D * NP);
        const int c = r / (D * NP), d = (r / NP) % D, node = r % NP;
        int l, t;
        node_line<N1>(node, n, l, t);
        const int oh = (e * NL + l) * 2;
        double a = ops.L1[t] * sUh[(oh + 1) * M + c] * sNh[(oh + 1) * D + d] +
                   ops.L0[t] * sUh[oh * M + c] * sNh[oh * D + d];
        const int og = (e * NL + l) * NG;
#pragma unroll
        for (int g = 0; g < NG; ++g) a -= ops.V[t][g] * sUg[(og + g) * M + c] * sAg[(og + g) * D + d];
        acc[q] += a;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < L::NITEM; ++q) {
    const int i = tid + q * NT_ELEM;
    if (i < ne * M * D * NP) {
      const int e = i / (M * D * NP), node = i % NP;
      Q[e0 * M * D * NP + i] = acc[q] * sJ[e * NP + node];
    }
  }
}

template <class K>
static hipError_t launch_elem(K kernel, size_t bytes, int64_t E, int epb, hipStream_t s, LineOps ops, MeshParams mp,
                              const double* a, const double* b, const double* c, const double* d, double* out) {
  if (bytes > 65536) {
    hipError_t err = hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (err != hipSuccess) return err;
  }
  const int64_t grid = (E + epb - 1) / epb;
  hipLaunchKernelGGL(kernel, dim3((unsigned)grid), dim3(NT_ELEM), bytes, s, ops, mp, a, b, c, d, out);
  return hipGetLastError();
}

hipError_t launch_residual(const DevCtx& dc, const double* U, const double* Q, double* R) {
  LDG_DISPATCH(dc, {
    using L = ResidLayout<D, P, EQ, double>;
    static_assert(L::bytes <= LDS_PER_CU, "residual workspace must fit one CU's LDS");
    return launch_elem(resid_kernel<D, P, EQ, double>, L::bytes, dc.E, L::EPB, dc.stream, dc.ops, dc.mp, U, nullptr,
                       Q, nullptr, R);
  })
}

hipError_t launch_residual_tangent(const DevCtx& dc, const double* U, const double* V, const double* Q,
                                   const double* Qt, double* Rt) {
  LDG_DISPATCH(dc, {
    using L = ResidLayout<D, P, EQ, Dual<1>>;
    static_assert(L::bytes <= LDS_PER_CU, "tangent workspace must fit one CU's LDS");
    return launch_elem(resid_kernel<D, P, EQ, Dual<1>>, L::bytes, dc.E, L::EPB, dc.stream, dc.ops, dc.mp, U, V, Q,
                       Qt, Rt);
  })
}

hipError_t launch_gradient(const DevCtx& dc, const double* U, double* Q, bool homogeneous, const double* Qc) {
  LDG_DISPATCH(dc, {
    using L = GradLayout<D, P, EQ>;
    static_assert(L::bytes <= LDS_PER_CU, "gradient workspace must fit one CU's LDS");
    const bool c22 = dc.mp.c22 != 0.0 && Qc;
    if (c22 && EQ != EQ_POISSON) return hipErrorInvalidValue;
    auto kern = grad_kernel<D, P, EQ, false>;
    if constexpr (EQ == EQ_POISSON) {
      if (c22) kern = grad_kernel<D, P, EQ, true>;
    }
    if (L::bytes > 65536) {
      hipError_t err = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L::bytes);
      if (err != hipSuccess) return err;
    }
    const int64_t grid = (dc.E + L::EPB - 1) / L::EPB;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(NT_ELEM), L::bytes, dc.stream, dc.ops, dc.mp, U, Q,
                       homogeneous ? 1 : 0, c22 ? Qc : nullptr);
    return hipGetLastError();
  })
}

}  // namespace ldg
