// Residual R = F(U) and LDG gradient Q = D(U) of the line-DG scheme.
//
// One workgroup owns EPB elements.  Each element's nodal state, node
// coordinates and nodal mapping gradient are staged in LDS; every reference
// line of every direction is then processed from LDS:
//   * Gauss phase (one work item per line and Gauss point): interpolate the
//     state to the point, evaluate the mapping gradient there exactly (the
//     derivative along the line from the coordinates, the other columns
//     interpolated from nodal values), form the non-unit normal
//     a_n = J G^{-T} N_n (eq. contraflux) and the contravariant flux F . a_n;
//   * face phase (one work item per line end): the point flux at the face
//     node with the coinciding node of the neighbour (Riemann + LDG switch,
//     Section 3), or the Dirichlet flux (eqs. dirichlet1/2);
//   * projection (one work item per node and component): the 1-D Galerkin
//     solution r_i = L1_i Fhat^+ + L0_i Fhat^- - sum_g V_ig f~_g of eq.
//     galerkinscheme2 with the mass solve folded into L0, L1, V, summed over
//     the D lines through the node and scaled by -1/J (eq. semidisc).
// The only global reads besides the element's own contiguous block are one
// neighbour node per line end.
#include "ldg_kernels.hpp"
#include "ldg_dispatch.hpp"

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

template <int D, int N1>
__device__ __forceinline__ void nodal_G_item(const double* sX, double* sG, const LineOps& ops, int node, int a, int b,
                                             int NP) {
  int s = 1;
  for (int k = 0; k < b; ++k) s *= N1;
  const int tb = (node / s) % N1;
  const int base = node - tb * s;
  double acc = 0.0;
#pragma unroll
  for (int q = 0; q < N1; ++q) acc += ops.Dn[tb][q] * sX[a * NP + base + q * s];
  sG[(a * D + b) * NP + node] = acc;
}

// mapping gradient at Gauss point g of line (n, l): exact for the Q_p map
template <int D, int N1>
__device__ __forceinline__ void gauss_metric(const double* sX, const double* sG, const LineOps& ops, int n, int l,
                                             int g, int NP, double* an) {
  double G[D][D];
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
}

template <int D>
__device__ __forceinline__ void node_G(const double* sG, int node, int NP, double G[D][D]) {
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) G[a][b] = sG[(a * D + b) * NP + node];
}

// --------------------------------------------------------------------------- residual
template <int D, int P, int EQ, class T>
struct ResidLayout {
  static constexpr int N1 = P + 1, NG = n_gauss(P), NP = ipow(N1, D), NL = ipow(N1, D - 1);
  static constexpr int M = Eq<D, EQ>::M;
  static constexpr bool VIS = Eq<D, EQ>::VIS;
  static constexpr int EPB = elems_per_block(NP, M);
  static constexpr int QW = VIS ? M * D : 0;
  // byte offsets (T first, then doubles; all multiples of 16)
  static constexpr size_t oU = 0;
  static constexpr size_t oQ = oU + sizeof(T) * EPB * M * NP;
  static constexpr size_t oF = oQ + sizeof(T) * EPB * QW * NP;
  static constexpr size_t oH = oF + sizeof(T) * EPB * D * NL * NG * M;
  static constexpr size_t oX = oH + sizeof(T) * EPB * D * NL * 2 * M;
  static constexpr size_t oG = oX + sizeof(double) * EPB * D * NP;
  static constexpr size_t bytes = oG + sizeof(double) * EPB * D * D * NP;
};

template <int D, int P, int EQ, class T>
__global__ void __launch_bounds__(NT_ELEM) resid_kernel(LineOps ops, MeshParams mp, const double* __restrict__ U,
                                                        const double* __restrict__ Ut, const double* __restrict__ Q,
                                                        const double* __restrict__ Qt, double* __restrict__ R) {
  using L = ResidLayout<D, P, EQ, T>;
  constexpr int N1 = L::N1, NG = L::NG, NP = L::NP, NL = L::NL, M = L::M, EPB = L::EPB, QW = L::QW;
  constexpr bool INV = Eq<D, EQ>::INV, VIS = Eq<D, EQ>::VIS;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sU = reinterpret_cast<T*>(smem_raw + L::oU);
  T* sQ = reinterpret_cast<T*>(smem_raw + L::oQ);
  T* sF = reinterpret_cast<T*>(smem_raw + L::oF);
  T* sH = reinterpret_cast<T*>(smem_raw + L::oH);
  double* sX = reinterpret_cast<double*>(smem_raw + L::oX);
  double* sG = reinterpret_cast<double*>(smem_raw + L::oG);

  const int64_t e0 = (int64_t)blockIdx.x * EPB;
  const int ne = (int)min((int64_t)EPB, mp.E - e0);
  const int tid = threadIdx.x;

  for (int i = tid; i < ne * M * NP; i += NT_ELEM) sU[i] = IO<T>::load(U, Ut, e0 * M * NP + i);
  if constexpr (VIS)
    for (int i = tid; i < ne * QW * NP; i += NT_ELEM) sQ[i] = IO<T>::load(Q, Qt, e0 * QW * NP + i);
  for (int i = tid; i < ne * D * NP; i += NT_ELEM) sX[i] = mp.xyz[e0 * D * NP + i];
  __syncthreads();
  for (int i = tid; i < ne * D * D * NP; i += NT_ELEM) {
    const int e = i / (D * D * NP), r = i % (D * D * NP);
    const int ab = r / NP, node = r % NP;
    nodal_G_item<D, N1>(sX + e * D * NP, sG + e * D * D * NP, ops, node, ab / D, ab % D, NP);
  }
  __syncthreads();

  // Gauss phase: contravariant flux at every line Gauss point
  for (int i = tid; i < ne * D * NL * NG; i += NT_ELEM) {
    const int e = i / (D * NL * NG), r = i % (D * NL * NG);
    const int n = r / (NL * NG), l = (r / NG) % NL, g = r % NG;
    double an[D];
    gauss_metric<D, N1>(sX + e * D * NP, sG + e * D * D * NP, ops, n, l, g, NP, an);
    T ug[M];
#pragma unroll
    for (int c = 0; c < M; ++c) {
      T acc = cst<T>(0.0);
#pragma unroll
      for (int t = 0; t < N1; ++t) acc += ops.I[g][t] * sU[(e * M + c) * NP + line_node<D, N1>(n, l, t)];
      ug[c] = acc;
    }
    T f[M];
#pragma unroll
    for (int c = 0; c < M; ++c) f[c] = cst<T>(0.0);
    if constexpr (INV) euler_flux_dot<D, T>(ug, an, mp.gamma, f);
    if constexpr (VIS) {
      T qg[M * D];
#pragma unroll
      for (int c = 0; c < M * D; ++c) {
        T acc = cst<T>(0.0);
#pragma unroll
        for (int t = 0; t < N1; ++t) acc += ops.I[g][t] * sQ[(e * QW + c) * NP + line_node<D, N1>(n, l, t)];
        qg[c] = acc;
      }
      visc_flux_dot_add<D, EQ, T>(ug, qg, an, mp.gamma, mp.mu, mp.prandtl, f);
    }
#pragma unroll
    for (int c = 0; c < M; ++c) sF[(((e * D + n) * NL + l) * NG + g) * M + c] = f[c];
  }

  // face phase: point fluxes at both ends of every line
  for (int i = tid; i < ne * D * NL * 2; i += NT_ELEM) {
    const int e = i / (D * NL * 2), r = i % (D * NL * 2);
    const int n = r / (NL * 2), l = (r / 2) % NL, s = r % 2;
    const int64_t eg = e0 + e;
    const int nin = line_node<D, N1>(n, l, s ? P : 0);
    double G[D][D], an[D], nrm[D];
    node_G<D>(sG + e * D * D * NP, nin, NP, G);
    cofactor_row<D>(G, n, an);
#pragma unroll
    for (int d = 0; d < D; ++d) nrm[d] = s ? an[d] : -an[d];
    const int f = 2 * n + s;
    const int64_t nb = mp.face_nbr[eg * 2 * D + f];
    const bool bnd = nb < 0;
    T uin[M], uout[M];
#pragma unroll
    for (int c = 0; c < M; ++c) uin[c] = sU[(e * M + c) * NP + nin];
    int nd = 0;
    if (!bnd) {
      nd = mp.nbr_node[(eg * 2 * D + f) * NL + l];
#pragma unroll
      for (int c = 0; c < M; ++c) uout[c] = IO<T>::load(U, Ut, (nb * M + c) * NP + nd);
    } else {
#pragma unroll
      for (int c = 0; c < M; ++c) uout[c] = cst<T>(mp.gD ? mp.gD[((eg * 2 * D + f) * M + c) * NL + l] : 0.0);
    }
    T F[M];
    if constexpr (VIS) {
      T qin[M * D], qout[M * D];
#pragma unroll
      for (int c = 0; c < M * D; ++c) qin[c] = sQ[(e * QW + c) * NP + nin];
      const int Sp = mp.sw[eg * D + n];
      const int S = s ? Sp : -Sp;
      if (!bnd && S > 0) {
#pragma unroll
        for (int c = 0; c < M * D; ++c) qout[c] = IO<T>::load(Q, Qt, (nb * QW + c) * NP + nd);
      } else {
#pragma unroll
        for (int c = 0; c < M * D; ++c) qout[c] = qin[c];
      }
      face_flux_point<D, EQ, T>(uin, qin, uout, qout, nrm, S, bnd, mp, F);
    } else {
      face_flux_point<D, EQ, T>(uin, uin, uout, uout, nrm, 1, bnd, mp, F);
    }
#pragma unroll
    for (int c = 0; c < M; ++c) sH[(((e * D + n) * NL + l) * 2 + s) * M + c] = F[c];
  }
  __syncthreads();

  // projection, sum over directions, -1/J scaling
  for (int i = tid; i < ne * M * NP; i += NT_ELEM) {
    const int e = i / (M * NP), r = i % (M * NP);
    const int c = r / NP, node = r % NP;
    T acc = cst<T>(0.0);
#pragma unroll
    for (int n = 0; n < D; ++n) {
      int l, t;
      node_line<N1>(node, n, l, t);
      const T* h = sH + ((e * D + n) * NL + l) * 2 * M;
      acc += ops.L1[t] * h[M + c] + ops.L0[t] * h[c];
      const T* fl = sF + ((e * D + n) * NL + l) * NG * M;
#pragma unroll
      for (int g = 0; g < NG; ++g) acc -= ops.V[t][g] * fl[g * M + c];
    }
    double G[D][D];
    node_G<D>(sG + e * D * D * NP, node, NP, G);
    const double J = det<D>(G);
    const int64_t gi = e0 * M * NP + i;
    double out = -tangent_or_value(acc) / J;
    if constexpr (sizeof(T) == sizeof(double)) {
      if (mp.S) out += mp.S[gi];
    }
    R[gi] = out;
  }
}

// --------------------------------------------------------------------------- gradient
template <int D, int P, int EQ>
struct GradLayout {
  static constexpr int N1 = P + 1, NG = n_gauss(P), NP = ipow(N1, D), NL = ipow(N1, D - 1);
  static constexpr int M = Eq<D, EQ>::M;
  static constexpr int EPB = elems_per_block(NP, M);
  static constexpr size_t oU = 0;
  static constexpr size_t oUg = oU + 8 * EPB * M * NP;
  static constexpr size_t oAg = oUg + 8 * EPB * D * NL * NG * M;
  static constexpr size_t oUh = oAg + 8 * EPB * D * NL * NG * D;
  static constexpr size_t oNh = oUh + 8 * EPB * D * NL * 2 * M;
  static constexpr size_t oX = oNh + 8 * EPB * D * NL * 2 * D;
  static constexpr size_t oG = oX + 8 * EPB * D * NP;
  static constexpr size_t bytes = oG + 8 * EPB * D * D * NP;
};

template <int D, int P, int EQ>
__global__ void __launch_bounds__(NT_ELEM) grad_kernel(LineOps ops, MeshParams mp, const double* __restrict__ U,
                                                       double* __restrict__ Q, int homogeneous) {
  using L = GradLayout<D, P, EQ>;
  constexpr int N1 = L::N1, NG = L::NG, NP = L::NP, NL = L::NL, M = L::M, EPB = L::EPB;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* sU = reinterpret_cast<double*>(smem_raw + L::oU);
  double* sUg = reinterpret_cast<double*>(smem_raw + L::oUg);
  double* sAg = reinterpret_cast<double*>(smem_raw + L::oAg);
  double* sUh = reinterpret_cast<double*>(smem_raw + L::oUh);
  double* sNh = reinterpret_cast<double*>(smem_raw + L::oNh);
  double* sX = reinterpret_cast<double*>(smem_raw + L::oX);
  double* sG = reinterpret_cast<double*>(smem_raw + L::oG);

  const int64_t e0 = (int64_t)blockIdx.x * EPB;
  const int ne = (int)min((int64_t)EPB, mp.E - e0);
  const int tid = threadIdx.x;
  for (int i = tid; i < ne * M * NP; i += NT_ELEM) sU[i] = U[e0 * M * NP + i];
  for (int i = tid; i < ne * D * NP; i += NT_ELEM) sX[i] = mp.xyz[e0 * D * NP + i];
  __syncthreads();
  for (int i = tid; i < ne * D * D * NP; i += NT_ELEM) {
    const int e = i / (D * D * NP), r = i % (D * D * NP);
    const int ab = r / NP, node = r % NP;
    nodal_G_item<D, N1>(sX + e * D * NP, sG + e * D * D * NP, ops, node, ab / D, ab % D, NP);
  }
  __syncthreads();
  for (int i = tid; i < ne * D * NL * NG; i += NT_ELEM) {
    const int e = i / (D * NL * NG), r = i % (D * NL * NG);
    const int n = r / (NL * NG), l = (r / NG) % NL, g = r % NG;
    double an[D];
    gauss_metric<D, N1>(sX + e * D * NP, sG + e * D * D * NP, ops, n, l, g, NP, an);
    const int o = ((e * D + n) * NL + l) * NG + g;
#pragma unroll
    for (int d = 0; d < D; ++d) sAg[o * D + d] = an[d];
#pragma unroll
    for (int c = 0; c < M; ++c) {
      double acc = 0.0;
#pragma unroll
      for (int t = 0; t < N1; ++t) acc += ops.I[g][t] * sU[(e * M + c) * NP + line_node<D, N1>(n, l, t)];
      sUg[o * M + c] = acc;
    }
  }
  for (int i = tid; i < ne * D * NL * 2; i += NT_ELEM) {
    const int e = i / (D * NL * 2), r = i % (D * NL * 2);
    const int n = r / (NL * 2), l = (r / 2) % NL, s = r % 2;
    const int64_t eg = e0 + e;
    const int nin = line_node<D, N1>(n, l, s ? P : 0);
    double G[D][D], an[D];
    node_G<D>(sG + e * D * D * NP, nin, NP, G);
    cofactor_row<D>(G, n, an);
    const int o = ((e * D + n) * NL + l) * 2 + s;
#pragma unroll
    for (int d = 0; d < D; ++d) sNh[o * D + d] = s ? an[d] : -an[d];
    const int f = 2 * n + s;
    const int64_t nb = mp.face_nbr[eg * 2 * D + f];
    const int Sp = mp.sw[eg * D + n];
    const int S = s ? Sp : -Sp;
    if (nb < 0) {
#pragma unroll
      for (int c = 0; c < M; ++c)
        sUh[o * M + c] = (homogeneous || !mp.gD) ? 0.0 : mp.gD[((eg * 2 * D + f) * M + c) * NL + l];
    } else if (S > 0) {
#pragma unroll
      for (int c = 0; c < M; ++c) sUh[o * M + c] = sU[(e * M + c) * NP + nin];
    } else {
      const int nd = mp.nbr_node[(eg * 2 * D + f) * NL + l];
#pragma unroll
      for (int c = 0; c < M; ++c) sUh[o * M + c] = U[(nb * M + c) * NP + nd];
    }
  }
  __syncthreads();
  for (int i = tid; i < ne * M * D * NP; i += NT_ELEM) {
    const int e = i / (M * D * NP), r = i % (M * D * NP);
    const int c = r / (D * NP), d = (r / NP) % D, node = r % NP;
    double acc = 0.0;
#pragma unroll
    for (int n = 0; n < D; ++n) {
      int l, t;
      node_line<N1>(node, n, l, t);
      const int oh = ((e * D + n) * NL + l) * 2;
      acc += ops.L1[t] * sUh[(oh + 1) * M + c] * sNh[(oh + 1) * D + d] + ops.L0[t] * sUh[oh * M + c] * sNh[oh * D + d];
      const int og = ((e * D + n) * NL + l) * NG;
#pragma unroll
      for (int g = 0; g < NG; ++g) acc -= ops.V[t][g] * sUg[(og + g) * M + c] * sAg[(og + g) * D + d];
    }
    double G[D][D];
    node_G<D>(sG + e * D * D * NP, node, NP, G);
    Q[e0 * M * D * NP + i] = acc / det<D>(G);
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
    return launch_elem(resid_kernel<D, P, EQ, double>, L::bytes, dc.E, L::EPB, dc.stream, dc.ops, dc.mp, U, nullptr,
                       Q, nullptr, R);
  })
}

hipError_t launch_residual_tangent(const DevCtx& dc, const double* U, const double* V, const double* Q,
                                   const double* Qt, double* Rt) {
  LDG_DISPATCH(dc, {
    using L = ResidLayout<D, P, EQ, Dual<1>>;
    return launch_elem(resid_kernel<D, P, EQ, Dual<1>>, L::bytes, dc.E, L::EPB, dc.stream, dc.ops, dc.mp, U, V, Q,
                       Qt, Rt);
  })
}

hipError_t launch_gradient(const DevCtx& dc, const double* U, double* Q, bool homogeneous) {
  LDG_DISPATCH(dc, {
    using L = GradLayout<D, P, EQ>;
    auto kern = grad_kernel<D, P, EQ>;
    if (L::bytes > 65536) {
      hipError_t err = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L::bytes);
      if (err != hipSuccess) return err;
    }
    const int64_t grid = (dc.E + L::EPB - 1) / L::EPB;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(NT_ELEM), L::bytes, dc.stream, dc.ops, dc.mp, U, Q,
                       homogeneous ? 1 : 0);
    return hipGetLastError();
  })
}

}  // namespace ldg
