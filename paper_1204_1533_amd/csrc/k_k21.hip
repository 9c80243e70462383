// K21 = dD/dU as stored weights (Section 4.1: the gradient operator is linear,
// constant in time and the same for every solution component), for the
// split product's w = K21 x.
//
// Weights: for row node a and each of its K21 slots (the D p + 1 line slots,
// then one neighbour slot per direction), D weights, node-fastest
// [slot][d][E Np] so that consecutive nodes read consecutive memory.  For the
// direction-n line through a (position t) and a column on it at t',
//   W_n[t][t'][d] = -sum_g V_tg I_gt' a_n(x_g)_d + L1_t n^+_d [t'=p, inside]
//                   + L0_t n^-_d [t'=0, inside],
// "inside" when the trace at that end is taken from this element (switch +1
// on an interior face, or a Neumann face / slip wall); the self slot sums its
// D lines; the neighbour slot of direction n is the end whose trace comes from
// outside (switch -1), weight L_end[t] n_end / J.  All weights are divided by
// J of the row node.  They are computed once per context from the geometry.
//
// Apply: w[c][d][a] = sum_slots W[slot][d][a] x[c][column], one work item per
// node, the block's elements staged in LDS (x of the neighbour nodes from HBM).
#include "ldg_dispatch.hpp"
#include "ldg_kernels.hpp"

namespace ldg {

template <int D, int P>
struct K21Layout {
  static constexpr int N1 = P + 1, NG = n_gauss(P), NP = ipow(N1, D), NL = ipow(N1, D - 1);
  static constexpr int oX = 0;
  static constexpr int oG = oX + D * NP;
  static constexpr int oJ = oG + D * D * NP;
  static constexpr int oAg = oJ + NP;
  static constexpr int oN = oAg + D * NL * NG * D;
  static constexpr int oW = oN + D * NL * 2 * D;
  static constexpr int oOps = oW + D * NL * N1 * N1 * D;
  static constexpr int ndoubles = oOps + (int)(sizeof(LineOps) / sizeof(double));
  static constexpr size_t bytes = sizeof(double) * ndoubles;
  static constexpr int NS = D * P + 1 + D;
};

template <int D, int P>
__global__ void __launch_bounds__(NT_ELEM) k21_weights_kernel(LineOps ops_arg, MeshParams mp,
                                                              double* __restrict__ Wt) {
  using L = K21Layout<D, P>;
  constexpr int N1 = L::N1, NG = L::NG, NP = L::NP, NL = L::NL, NSL = D * P + 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* sm = reinterpret_cast<double*>(smem_raw);
  double* sX = sm + L::oX;
  double* sG = sm + L::oG;
  double* sJ = sm + L::oJ;
  double* sAg = sm + L::oAg;
  double* sN = sm + L::oN;
  double* sW = sm + L::oW;
  const int64_t e = blockIdx.x;
  const int tid = threadIdx.x;
  const int64_t NN = mp.E * NP;
  for (int i = tid; i < D * NP; i += NT_ELEM) sX[i] = mp.xyz[e * D * NP + i];
  {
    const double* src = reinterpret_cast<const double*>(&ops_arg);
    for (int i = tid; i < (int)(sizeof(LineOps) / sizeof(double)); i += NT_ELEM) sm[L::oOps + i] = src[i];
  }
  __syncthreads();
  const LineOps& ops = *reinterpret_cast<const LineOps*>(sm + L::oOps);
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
    sJ[i] = 1.0 / det<D>(G);
  }
  for (int it = tid; it < D * NL * NG; it += NT_ELEM) {
    const int n = it / (NL * NG), l = (it / NG) % NL, g = it % NG;
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
#pragma unroll
    for (int d = 0; d < D; ++d) sAg[it * D + d] = an[d];
  }
  for (int it = tid; it < D * NL * 2; it += NT_ELEM) {
    const int n = it / (NL * 2), l = (it / 2) % NL, s = it % 2;
    const int nin = line_node<D, N1>(n, l, s ? P : 0);
    double G[D][D], an[D];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = 0; b < D; ++b) G[a][b] = sG[(a * D + b) * NP + nin];
    cofactor_row<D>(G, n, an);
#pragma unroll
    for (int d = 0; d < D; ++d) sN[it * D + d] = s ? an[d] : -an[d];
  }
  __syncthreads();
  for (int it = tid; it < D * NL * N1 * N1 * D; it += NT_ELEM) {
    const int d = it % D;
    const int tp = (it / D) % N1;
    const int t = (it / (D * N1)) % N1;
    const int l = (it / (D * N1 * N1)) % NL;
    const int n = it / (D * N1 * N1 * NL);
    double v = 0.0;
#pragma unroll
    for (int g = 0; g < NG; ++g) v -= ops.V[t][g] * ops.I[g][tp] * sAg[((n * NL + l) * NG + g) * D + d];
    const int Sp = mp.sw[e * D + n];
    const int k1 = face_kind(mp.face_nbr[e * 2 * D + 2 * n + 1]), k0 = face_kind(mp.face_nbr[e * 2 * D + 2 * n]);
    if (tp == P && ((Sp > 0 && k1 == BC_INTERIOR) || k1 == BC_NEUMANN || k1 == BC_SLIP))
      v += ops.L1[t] * sN[((n * NL + l) * 2 + 1) * D + d];
    if (tp == 0 && ((Sp < 0 && k0 == BC_INTERIOR) || k0 == BC_NEUMANN || k0 == BC_SLIP))
      v += ops.L0[t] * sN[((n * NL + l) * 2 + 0) * D + d];
    sW[it] = v;
  }
  __syncthreads();
  // one work item per (node, slot): its D weights
  for (int it = tid; it < NP * L::NS; it += NT_ELEM) {
    const int a = it % NP, slot = it / NP;
    const int64_t gn = e * NP + a;
    double w[D];
#pragma unroll
    for (int d = 0; d < D; ++d) w[d] = 0.0;
    if (slot < NSL) {
      const int self = a % N1;
      if (slot == self) {
#pragma unroll
        for (int n = 0; n < D; ++n) {
          int l, t;
          node_line<N1>(a, n, l, t);
#pragma unroll
          for (int d = 0; d < D; ++d) w[d] += sW[(((n * NL + l) * N1 + t) * N1 + t) * D + d];
        }
      } else {
        const int b = slot_col<D, P>(a, slot);
        // the line shared by a and b: the one coordinate where they differ
        int n = 0;
        {
          int ra = a, rb = b;
          for (int k = 0; k < D; ++k) {
            if (ra % N1 != rb % N1) n = k;
            ra /= N1;
            rb /= N1;
          }
        }
        int l, t, lb, tb;
        node_line<N1>(a, n, l, t);
        node_line<N1>(b, n, lb, tb);
#pragma unroll
        for (int d = 0; d < D; ++d) w[d] = sW[(((n * NL + l) * N1 + t) * N1 + tb) * D + d];
      }
    } else {
      const int n = slot - NSL;
      const int Sp = mp.sw[e * D + n];
      const int s = Sp < 0 ? 1 : 0;  // the end whose trace comes from outside
      const int64_t nb = mp.face_nbr[e * 2 * D + 2 * n + s];
      int l, t;
      node_line<N1>(a, n, l, t);
      if (nb >= 0) {
#pragma unroll
        for (int d = 0; d < D; ++d) w[d] = (s ? ops.L1[t] : ops.L0[t]) * sN[((n * NL + l) * 2 + s) * D + d];
      }
    }
#pragma unroll
    for (int d = 0; d < D; ++d) Wt[((int64_t)slot * D + d) * NN + gn] = w[d] * sJ[a];
  }
}

// TW: the stored weights' type (FP64, or the FP32 copy used beside stored
// low-precision blocks); products accumulate in FP64 either way.
template <int D, int P, int EQ, class TW>
__global__ void __launch_bounds__(256) k21_apply_kernel(MeshParams mp, const TW* __restrict__ Wt,
                                                        const double* __restrict__ x, double* __restrict__ w) {
  constexpr int N1 = P + 1, NP = ipow(N1, D), NL = ipow(N1, D - 1), M = Eq<D, EQ>::M, NSL = D * P + 1;
  constexpr int EPB = NP >= 256 ? 1 : 256 / NP;
  static_assert(NP <= 256, "one work item per node of an element");
  __shared__ double sx[EPB * M * NP];
  const int64_t NN = mp.E * NP;
  const int64_t e0 = xcd_block(blockIdx.x, gridDim.x) * EPB;
  const int nel = (int)(mp.E - e0 < EPB ? mp.E - e0 : EPB);
  for (int i = threadIdx.x; i < nel * M * NP; i += 256) sx[i] = x[e0 * M * NP + i];
  __syncthreads();
  const int le = threadIdx.x / NP, a = threadIdx.x % NP;
  if (le >= nel) return;  // no barrier below
  const int64_t e = e0 + le;
  const int64_t gn = e * NP + a;
  const double* lx = sx + le * M * NP;
  double acc[M][D];
#pragma unroll
  for (int c = 0; c < M; ++c)
#pragma unroll
    for (int d = 0; d < D; ++d) acc[c][d] = 0.0;
#pragma unroll 1
  for (int s = 0; s < NSL + D; ++s) {
    double wt[D], xv[M];
#pragma unroll
    for (int d = 0; d < D; ++d) wt[d] = (double)Wt[((int64_t)s * D + d) * NN + gn];
    if (s < NSL) {
      const int b = slot_col<D, P>(a, s);
#pragma unroll
      for (int c = 0; c < M; ++c) xv[c] = lx[c * NP + b];
    } else {
      const int n = s - NSL;
      const int side = mp.sw[e * D + n] < 0 ? 1 : 0;
      const int f = 2 * n + side;
      const int64_t nb = mp.face_nbr[e * 2 * D + f];
      if (nb < 0) continue;
      int l, t;
      node_line<N1>(a, n, l, t);
      const int ca = mp.nbr_node[(e * 2 * D + f) * NL + l];
#pragma unroll
      for (int c = 0; c < M; ++c) xv[c] = x[(nb * M + c) * NP + ca];
    }
#pragma unroll
    for (int c = 0; c < M; ++c)
#pragma unroll
      for (int d = 0; d < D; ++d) acc[c][d] += wt[d] * xv[c];
  }
#pragma unroll
  for (int c = 0; c < M; ++c)
#pragma unroll
    for (int d = 0; d < D; ++d) w[((e * M + c) * D + d) * NP + a] = acc[c][d];
}

hipError_t launch_k21_weights(const DevCtx& dc, double* Wt) {
  LDG_DISPATCH(dc, {
    using L = K21Layout<D, P>;
    static_assert(L::bytes <= LDS_PER_CU, "weights workspace must fit one CU's LDS");
    auto k = k21_weights_kernel<D, P>;
    if (L::bytes > 65536) {
      hipError_t err = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L::bytes);
      if (err != hipSuccess) return err;
    }
    hipLaunchKernelGGL(k, dim3((unsigned)dc.E), dim3(NT_ELEM), L::bytes, dc.stream, dc.ops, dc.mp, Wt);
    return hipGetLastError();
  })
}

template <class TW>
static hipError_t k21_apply_any(const DevCtx& dc, const TW* Wt, const double* x, double* w) {
  LDG_DISPATCH(dc, {
    constexpr int NP = ipow(P + 1, D);
    constexpr int EPB = NP >= 256 ? 1 : 256 / NP;
    const unsigned grid = (unsigned)((dc.E + EPB - 1) / EPB);
    hipLaunchKernelGGL((k21_apply_kernel<D, P, EQ, TW>), dim3(grid), dim3(256), 0, dc.stream, dc.mp, Wt, x, w);
    return hipGetLastError();
  })
}

hipError_t launch_k21_apply(const DevCtx& dc, const double* Wt, const double* x, double* w) {
  return k21_apply_any(dc, Wt, x, w);
}
hipError_t launch_k21_apply_f32(const DevCtx& dc, const float* Wt, const double* x, double* w) {
  return k21_apply_any(dc, Wt, x, w);
}

__global__ void __launch_bounds__(256) to_f32_kernel(const double* __restrict__ in, float* __restrict__ out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (float)in[i];
}
hipError_t launch_k21_weights_f32(const DevCtx& dc, const double* Wt, float* Wf) {
  const int64_t n = (int64_t)(dc.D * dc.P + 1 + dc.D) * dc.D * dc.E * dc.NP;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(to_f32_kernel, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256), 0, dc.stream, Wt, Wf,
                     n);
  return hipGetLastError();
}

}  // namespace ldg
