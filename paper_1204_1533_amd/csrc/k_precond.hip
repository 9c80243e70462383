// Split Jacobian-vector product and the element-local line-pattern
// preconditioner (Section 4.2 of the paper).
//
// jacvec:   y = alpha x - gamma (K11 x + K12 w), w = K21 x computed by the
//           gradient kernel with zero boundary data (eq. matvecsplit).  One
//           thread per node streams its block row (node-fastest layout, so a
//           wavefront reads contiguous memory for every (slot, c, c')); the
//           workgroup holds whole elements and stages their x and w in LDS.
// form:     A~ = alpha I - gamma (K11 + K12 K21) restricted to the D lines
//           through each node, K21 taken inside the element.  The K21 weights
//           of a direction-n line are the scalar line operator
//             G[t][t'][d] = -sum_g V_tg I_gt' a_n(x_g)_d + L1_t n^+_d [t'=p, inside]
//                           + L0_t n^-_d [t'=0, inside]
//           (inside: the switch takes the trace from this element), divided
//           by J of the node t.  For a row a and a column b on its
//           direction-n line, (K12 K21)_ab = sum_{c on that line} K12_ac W_cb,
//           with W_cb = G_n[t_c][t_b] / J_c for c != b and W_bb the sum of the
//           diagonal entries of all D line operators through b over J_b; for
//           b = a the sum over c runs over all D lines.
// factor:   block ILU(0) in natural node order.  Row i depends only on the
//           earlier nodes of its own lines, so rows with equal i+j(+k) form
//           independent levels; each row's lower blocks k update only blocks
//           on the line they share.  The diagonal slot keeps the inverse of
//           the U diagonal block.
// apply:    forward / backward block substitution over the same levels.
#include <type_traits>

#include "ldg_dispatch.hpp"
#include "ldg_kernels.hpp"
#include "ldg_store.hpp"

namespace ldg {

// --------------------------------------------------------------------------- jacvec
// Elements per 256-thread workgroup of the product (one node per thread).
template <int NP>
__host__ __device__ constexpr int jv_epb() {
  return NP >= 256 ? 1 : 256 / NP;
}

template <int D, int P, int EQ, int PR>
__global__ void __launch_bounds__(256) jacvec_kernel(MeshParams mp, const void* __restrict__ K11,
                                                     const void* __restrict__ K12, double alpha, double gamma,
                                                     const double* __restrict__ x, const double* __restrict__ w,
                                                     double* __restrict__ y) {
  constexpr int N1 = P + 1, NP = ipow(N1, D), NL = ipow(N1, D - 1), M = Eq<D, EQ>::M;
  constexpr bool VIS = Eq<D, EQ>::VIS;
  constexpr int NSL = D * P + 1, NS11 = NSL + 2 * D, NS12 = NSL + D, MD = M * D;
  constexpr int EPB = jv_epb<NP>();
  // The block's elements' x and w (contiguous in HBM) are staged in LDS: every
  // node reads the x / w of its D lines many times, and those reads would
  // otherwise miss in L2 behind the stream of Jacobian blocks.
  __shared__ double sx[EPB * M * NP];
  __shared__ double sw[VIS ? EPB * MD * NP : 1];
  const int64_t NN = mp.E * NP;
  const int64_t e0 = xcd_block(blockIdx.x, gridDim.x) * EPB;
  const int nel = (int)(mp.E - e0 < EPB ? mp.E - e0 : EPB);
  for (int i = threadIdx.x; i < nel * M * NP; i += 256) sx[i] = x[e0 * M * NP + i];
  if constexpr (VIS)
    for (int i = threadIdx.x; i < nel * MD * NP; i += 256) sw[i] = w[e0 * MD * NP + i];
  __syncthreads();
  const int le = threadIdx.x / NP, a = threadIdx.x % NP;
  if (le >= nel) return;  // no barrier below this point
  const int64_t e = e0 + le;
  const int64_t gn = e * NP + a;
  const double* lx = sx + le * M * NP;
  double acc[M];
#pragma unroll
  for (int c = 0; c < M; ++c) acc[c] = 0.0;
  // slot loops are not unrolled: unrolled, every block load is hoisted and the
  // kernel spills and drops to one wavefront per SIMD
#pragma unroll 1
  for (int s = 0; s < NS11; ++s) {
    double xv[M];
    if (s < NSL) {
      const int b = slot_col<D, P>(a, s);
#pragma unroll
      for (int k = 0; k < M; ++k) xv[k] = lx[k * NP + b];
    } else {
      const int f = s - NSL, n = f / 2;
      const int64_t nb = mp.face_nbr[e * 2 * D + f];
      if (nb < 0) continue;
      int l, t;
      node_line<N1>(a, n, l, t);
      const int ca = mp.nbr_node[(e * 2 * D + f) * NL + l];
#pragma unroll
      for (int k = 0; k < M; ++k) xv[k] = x[(nb * M + k) * NP + ca];
    }
#pragma unroll
    for (int c = 0; c < M; ++c)
#pragma unroll
      for (int k = 0; k < M; ++k) acc[c] += Store<PR>::get(K11, ((int64_t)(s * M + c) * M + k) * NN + gn) * xv[k];
  }
  if constexpr (VIS) {
    const double* lw = sw + le * MD * NP;
#pragma unroll 1
    for (int s = 0; s < NS12; ++s) {
      const double* src;
      int64_t stride_base;
      int ca;
      if (s < NSL) {
        src = lw;
        stride_base = 0;
        ca = slot_col<D, P>(a, s);
      } else {
        const int n = s - NSL;
        const int side = mp.sw[e * D + n] > 0 ? 1 : 0;
        const int f = 2 * n + side;
        const int64_t nb = mp.face_nbr[e * 2 * D + f];
        if (nb < 0) continue;
        int l, t;
        node_line<N1>(a, n, l, t);
        src = w;
        stride_base = nb * MD * NP;
        ca = mp.nbr_node[(e * 2 * D + f) * NL + l];
      }
#pragma unroll
      for (int k = 0; k < MD; ++k) {
        const double wv = src[stride_base + k * NP + ca];
#pragma unroll
        for (int c = 0; c < M; ++c) acc[c] += Store<PR>::get(K12, ((int64_t)(s * M + c) * MD + k) * NN + gn) * wv;
      }
    }
  }
#pragma unroll
  for (int c = 0; c < M; ++c) {
    const int64_t i = (e * M + c) * NP + a;
    y[i] = alpha * lx[c * NP + a] - gamma * acc[c];
  }
}

hipError_t launch_jacvec(const DevCtx& dc, const void* K11, const void* K12, int prec, double alpha, double gamma,
                         const double* x, const double* w, double* y) {
  LDG_DISPATCH(dc, {
    constexpr int EPB = jv_epb<ipow(P + 1, D)>();
    const unsigned grid = (unsigned)((dc.E + EPB - 1) / EPB);
    LDG_PREC_DISPATCH(prec, {
      hipLaunchKernelGGL((jacvec_kernel<D, P, EQ, PR>), dim3(grid), dim3(256), 0, dc.stream, dc.mp, K11, K12, alpha,
                         gamma, x, w, y);
      return hipGetLastError();
    })
  })
}

// --------------------------------------------------------------------------- formation of A~
template <int D, int P, int EQ>
struct FormLayout {
  static constexpr int N1 = P + 1, NG = n_gauss(P), NP = ipow(N1, D), NL = ipow(N1, D - 1);
  static constexpr int oX = 0;
  static constexpr int oG = oX + D * NP;
  static constexpr int oJ = oG + D * D * NP;
  static constexpr int oAg = oJ + NP;
  static constexpr int oN = oAg + D * NL * NG * D;
  static constexpr int oW = oN + D * NL * 2 * D;
  static constexpr int oS = oW + D * NL * N1 * N1 * D;
  static constexpr int ndoubles = oS + NP * D;
  static constexpr size_t bytes = sizeof(double) * ndoubles;
};

// Writes A~ (line slots, [slot][c][c'][E*Np]) in the working precision WP of the factorisation.
template <int D, int P, int EQ, int PR, int WP>
__global__ void __launch_bounds__(NT_ELEM) form_kernel(LineOps ops, MeshParams mp, const void* __restrict__ K11,
                                                       const void* __restrict__ K12, double alpha, double gamma,
                                                       void* __restrict__ F) {
  using L = FormLayout<D, P, EQ>;
  constexpr int N1 = L::N1, NG = L::NG, NP = L::NP, NL = L::NL, M = Eq<D, EQ>::M;
  constexpr bool VIS = Eq<D, EQ>::VIS;
  constexpr int NSL = D * P + 1, MD = M * D;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* sm = reinterpret_cast<double*>(smem_raw);
  double* sX = sm + L::oX;
  double* sG = sm + L::oG;
  double* sJ = sm + L::oJ;
  double* sAg = sm + L::oAg;
  double* sN = sm + L::oN;
  double* sW = sm + L::oW;
  double* sS = sm + L::oS;  // full K21 self weight of each node: sum over its D lines, divided by J
  const int64_t e = blockIdx.x;
  const int tid = threadIdx.x;
  const int64_t NN = mp.E * NP;
  if constexpr (VIS) {
    for (int i = tid; i < D * NP; i += NT_ELEM) sX[i] = mp.xyz[e * D * NP + i];
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
    // scalar K21 line operators G_n[l][t][t'][d] (without the 1/J of row t)
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
      if (tp == P && Sp > 0 && mp.face_nbr[e * 2 * D + 2 * n + 1] >= 0)
        v += ops.L1[t] * sN[((n * NL + l) * 2 + 1) * D + d];
      if (tp == 0 && Sp < 0 && mp.face_nbr[e * 2 * D + 2 * n] >= 0)
        v += ops.L0[t] * sN[((n * NL + l) * 2 + 0) * D + d];
      sW[it] = v;
    }
    __syncthreads();
    for (int it = tid; it < NP * D; it += NT_ELEM) {
      const int b = it / D, d = it % D;
      double v = 0.0;
#pragma unroll
      for (int m = 0; m < D; ++m) {
        int lm, tm;
        node_line<N1>(b, m, lm, tm);
        v += sW[(((m * NL + lm) * N1 + tm) * N1 + tm) * D + d];
      }
      sS[it] = v * sJ[b];
    }
    __syncthreads();
  }
  // A~ rows: one work item per (row node a, row component c).  For each of the
  // D lines through a, row c of K12 on the line's p+1 slots is loaded once and
  // gives the p+1 output blocks on that line:
  //   (K12 K21)_ab[c][k] = sum_{c' on the line, c' != b} K12_ac'[c][k,:] . W_n[t_c'][t_b][:] / J_c'
  //                      + K12_ab[c][k,:] . S_b[:]        (S_b: self weight of b over its D lines)
  // The self block (b = a) collects the c' != a terms of all D lines.
  using KT = typename std::conditional<PR == PREC_F64, double, float>::type;
#pragma unroll 1
  for (int it = tid; it < NP * M; it += NT_ELEM) {
    const int a = it % NP, c = it / NP;
    const int self = a % N1;
    const int64_t gn = e * NP + a;
    double self_acc[M];
#pragma unroll
    for (int k = 0; k < M; ++k) self_acc[k] = 0.0;
#pragma unroll 1
    for (int n = 0; n < D; ++n) {
      int la, ta;
      node_line<N1>(a, n, la, ta);
      KT kc[VIS ? N1 : 1][VIS ? MD : 1];
      double jc[N1];
      if constexpr (VIS) {
#pragma unroll
        for (int tc = 0; tc < N1; ++tc) {
          const int sc = slot_of<N1>(n, ta, tc, self);
#pragma unroll
          for (int q = 0; q < MD; ++q) kc[tc][q] = (KT)Store<PR>::get(K12, ((int64_t)(sc * M + c) * MD + q) * NN + gn);
          jc[tc] = sJ[line_node<D, N1>(n, la, tc)];
        }
      }
#pragma unroll
      for (int tb = 0; tb < N1; ++tb) {
        const int b = line_node<D, N1>(n, la, tb);
        const bool is_self = tb == ta;
        if (is_self && !VIS) continue;
        double prod[M];
#pragma unroll
        for (int k = 0; k < M; ++k) prod[k] = 0.0;
        if constexpr (VIS) {
#pragma unroll
          for (int tc = 0; tc < N1; ++tc) {
            if (tc == tb) continue;
            double w[D];
#pragma unroll
            for (int d = 0; d < D; ++d) w[d] = sW[(((n * NL + la) * N1 + tc) * N1 + tb) * D + d] * jc[tc];
#pragma unroll
            for (int k = 0; k < M; ++k)
#pragma unroll
              for (int d = 0; d < D; ++d) prod[k] += (double)kc[tc][k * D + d] * w[d];
          }
        }
        if (is_self) {
#pragma unroll
          for (int k = 0; k < M; ++k) self_acc[k] += prod[k];
          continue;
        }
        if constexpr (VIS) {
#pragma unroll
          for (int k = 0; k < M; ++k)
#pragma unroll
            for (int d = 0; d < D; ++d) prod[k] += (double)kc[tb][k * D + d] * sS[b * D + d];
        }
        const int slot = slot_of<N1>(n, ta, tb, self);
#pragma unroll
        for (int k = 0; k < M; ++k) {
          const double v = Store<PR>::get(K11, ((int64_t)(slot * M + c) * M + k) * NN + gn) + prod[k];
          Store<WP>::put(F, ((int64_t)(slot * M + c) * M + k) * NN + gn, -gamma * v);
        }
      }
    }
    // self block: K11 + the c' != a terms of all lines + K12_aa . S_a
#pragma unroll
    for (int k = 0; k < M; ++k) {
      double v = Store<PR>::get(K11, ((int64_t)(self * M + c) * M + k) * NN + gn) + self_acc[k];
      if constexpr (VIS) {
#pragma unroll
        for (int d = 0; d < D; ++d)
          v += Store<PR>::get(K12, ((int64_t)(self * M + c) * MD + k * D + d) * NN + gn) * sS[a * D + d];
      }
      v = -gamma * v;
      if (c == k) v += alpha;
      Store<WP>::put(F, ((int64_t)(self * M + c) * M + k) * NN + gn, v);
    }
  }
}

// --------------------------------------------------------------------------- BILU(0)
template <int D, int P>
__device__ void level_table(int* rows, int* off) {
  // rows sorted by coordinate sum; off[L] .. off[L+1]
  constexpr int N1 = P + 1, NP = ipow(N1, D);
  int pos = 0;
  for (int L = 0; L <= D * P; ++L) {
    off[L] = pos;
    for (int a = 0; a < NP; ++a) {
      int s = 0, r = a;
      for (int d = 0; d < D; ++d) {
        s += r % N1;
        r /= N1;
      }
      if (s == L) rows[pos++] = a;
    }
  }
  off[D * P + 1] = pos;
}

template <int M>
__device__ __forceinline__ void invert_block(double A[M][M], double Inv[M][M]) {
  double W[M][2 * M];
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int j = 0; j < M; ++j) {
      W[i][j] = A[i][j];
      W[i][M + j] = (i == j) ? 1.0 : 0.0;
    }
#pragma unroll
  for (int c = 0; c < M; ++c) {
    int piv = c;
    double best = fabs(W[c][c]);
#pragma unroll
    for (int r = c + 1; r < M; ++r)
      if (fabs(W[r][c]) > best) {
        best = fabs(W[r][c]);
        piv = r;
      }
    // row swap with compile-time row indices (a runtime row index would put
    // W in scratch memory)
#pragma unroll
    for (int r = c + 1; r < M; ++r)
      if (r == piv) {
#pragma unroll
        for (int j = 0; j < 2 * M; ++j) {
          double t = W[c][j];
          W[c][j] = W[r][j];
          W[r][j] = t;
        }
      }
    const double id = 1.0 / W[c][c];
#pragma unroll
    for (int j = 0; j < 2 * M; ++j) W[c][j] *= id;
#pragma unroll
    for (int r = 0; r < M; ++r) {
      if (r == c) continue;
      const double f = W[r][c];
#pragma unroll
      for (int j = 0; j < 2 * M; ++j) W[r][j] -= f * W[c][j];
    }
  }
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int j = 0; j < M; ++j) Inv[i][j] = W[i][M + j];
}

// One wavefront per element; lanes = (row of the current level, component row c).
template <int D, int P, int EQ, int WP>
__global__ void __launch_bounds__(64) factor_kernel(int64_t E, void* __restrict__ F) {
  constexpr int N1 = P + 1, NP = ipow(N1, D), M = Eq<D, EQ>::M;
  constexpr int RPP = 64 / M;  // rows per pass
  constexpr int NSLMM = (D * P + 1) * M * M;
  // F: element-major [E Np][slot][c][c'], so one workgroup's rows are one
  // contiguous block
  __shared__ int rows[NP];
  __shared__ int off[D * P + 2];
  const int64_t e = blockIdx.x;
  const int lane = threadIdx.x;
  if (lane == 0) level_table<D, P>(rows, off);
  __syncthreads();
  for (int L = 0; L <= D * P; ++L) {
    const int nrow = off[L + 1] - off[L];
    for (int r0 = 0; r0 < nrow; r0 += RPP) {
      const int ri = r0 + lane / M, c = lane % M;
      const bool active = (lane < RPP * M) && ri < nrow;
      int i = 0;
      if (active) {
        i = rows[off[L] + ri];
        const int64_t gi = e * NP + i;
        const int self_i = i % N1;
        for (int n = 0; n < D; ++n) {
          int l, ti;
          node_line<N1>(i, n, l, ti);
          for (int tk = 0; tk < ti; ++tk) {
            const int k = line_node<D, N1>(n, l, tk);
            const int64_t gk = e * NP + k;
            const int sik = slot_of<N1>(n, ti, tk, self_i);
            // L_ik[c][:] = A_ik[c][:] Uinv_kk
            double arow[M], lrow[M];
#pragma unroll
            for (int q = 0; q < M; ++q) arow[q] = Store<WP>::get(F, gi * NSLMM + (sik * M + c) * M + q);
            const int self_k = k % N1;
#pragma unroll
            for (int j = 0; j < M; ++j) {
              double s = 0.0;
#pragma unroll
              for (int q = 0; q < M; ++q) s += arow[q] * Store<WP>::get(F, gk * NSLMM + (self_k * M + q) * M + j);
              lrow[j] = s;
            }
#pragma unroll
            for (int j = 0; j < M; ++j) Store<WP>::put(F, gi * NSLMM + (sik * M + c) * M + j, lrow[j]);
            // A_ij -= L_ik U_kj for j after k on the shared line
            for (int tj = tk + 1; tj < N1; ++tj) {
              const int sij = slot_of<N1>(n, ti, tj, self_i);
              const int skj = slot_of<N1>(n, tk, tj, self_k);
#pragma unroll
              for (int j = 0; j < M; ++j) {
                double s = 0.0;
#pragma unroll
                for (int q = 0; q < M; ++q) s += lrow[q] * Store<WP>::get(F, gk * NSLMM + (skj * M + q) * M + j);
                const int64_t idx = gi * NSLMM + (sij * M + c) * M + j;
                Store<WP>::put(F, idx, Store<WP>::get(F, idx) - s);
              }
            }
          }
        }
      }
      __syncthreads();
      if (active && c == 0) {
        const int64_t gi = e * NP + i;
        const int self_i = i % N1;
        double A[M][M], Inv[M][M];
#pragma unroll
        for (int a = 0; a < M; ++a)
#pragma unroll
          for (int b = 0; b < M; ++b) A[a][b] = Store<WP>::get(F, gi * NSLMM + (self_i * M + a) * M + b);
        invert_block<M>(A, Inv);
#pragma unroll
        for (int a = 0; a < M; ++a)
#pragma unroll
          for (int b = 0; b < M; ++b) Store<WP>::put(F, gi * NSLMM + (self_i * M + a) * M + b, Inv[a][b]);
      }
      __syncthreads();
    }
  }
}

template <int D, int P, int EQ, int FP>
__global__ void __launch_bounds__(64) apply_kernel(int64_t E, const void* __restrict__ F, const double* __restrict__ r,
                                                   double* __restrict__ z) {
  constexpr int N1 = P + 1, NP = ipow(N1, D), M = Eq<D, EQ>::M;
  constexpr int NSL = D * P + 1, RPP = 64 / M, NSLMM = NSL * M * M;
  // F: element-major copy of the factors, [E Np][slot][c][c'] (one element's
  // factors are contiguous, so a workgroup reads whole cache lines)
  __shared__ int rows[NP];
  __shared__ int off[D * P + 2];
  __shared__ double sy[NP * M];
  __shared__ double st[NP * M];
  const int64_t e = blockIdx.x;
  const int lane = threadIdx.x;
  if (lane == 0) level_table<D, P>(rows, off);
  for (int i = lane; i < NP * M; i += 64) sy[i] = r[e * M * NP + (i % M) * NP + i / M];
  __syncthreads();
  // forward: y_i = r_i - sum_{k < i on i's lines} L_ik y_k
  for (int L = 1; L <= D * P; ++L) {
    const int nrow = off[L + 1] - off[L];
    for (int r0 = 0; r0 < nrow; r0 += RPP) {
      const int ri = r0 + lane / M, c = lane % M;
      double acc = 0.0;
      int i = 0;
      const bool active = (lane < RPP * M) && ri < nrow;
      if (active) {
        i = rows[off[L] + ri];
        const int64_t gi = e * NP + i;
        const int self_i = i % N1;
        acc = sy[i * M + c];
        // all line slots with compile-time bounds; the strictly lower ones
        // (column before i in natural order) count, so every load of the row
        // can be in flight at once.  Slot order = direction-major, position-
        // ascending, the order of the elimination.
#pragma unroll
        for (int s = 0; s < NSL; ++s) {
          const int k = slot_col<D, P>(i, s);
          const double msk = k < i ? 1.0 : 0.0;
          double t = 0.0;
#pragma unroll
          for (int q = 0; q < M; ++q) t += Store<FP>::get(F, gi * NSLMM + (s * M + c) * M + q) * sy[k * M + q];
          acc -= msk * t;
        }
      }
      __syncthreads();
      if (active) sy[i * M + c] = acc;
      __syncthreads();
    }
  }
  // backward: z_i = Uinv_ii (y_i - sum_{j > i on i's lines} U_ij z_j); z overwrites y
  for (int L = D * P; L >= 0; --L) {
    const int nrow = off[L + 1] - off[L];
    for (int r0 = 0; r0 < nrow; r0 += RPP) {
      const int ri = r0 + lane / M, c = lane % M;
      const bool active = (lane < RPP * M) && ri < nrow;
      int i = 0;
      if (active) {
        i = rows[off[L] + ri];
        const int64_t gi = e * NP + i;
        const int self_i = i % N1;
        double acc = sy[i * M + c];
#pragma unroll
        for (int s = 0; s < NSL; ++s) {
          const int j = slot_col<D, P>(i, s);
          const double msk = j > i ? 1.0 : 0.0;
          double t = 0.0;
#pragma unroll
          for (int q = 0; q < M; ++q) t += Store<FP>::get(F, gi * NSLMM + (s * M + c) * M + q) * sy[j * M + q];
          acc -= msk * t;
        }
        st[i * M + c] = acc;
      }
      __syncthreads();
      if (active) {
        const int64_t gi = e * NP + i;
        const int self_i = i % N1;
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < M; ++q) v += Store<FP>::get(F, gi * NSLMM + (self_i * M + c) * M + q) * st[i * M + q];
        sy[i * M + c] = v;
      }
      __syncthreads();
    }
  }
  for (int i = lane; i < NP * M; i += 64) z[e * M * NP + (i % M) * NP + i / M] = sy[i];
}

template <int PIN, int POUT>
__global__ void convert_kernel(const void* __restrict__ in, void* __restrict__ out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    Store<POUT>::put(out, i, Store<PIN>::get(in, i));
}

// node-fastest [q][E Np] -> element-major [E Np][q], q = (slot, c, c'):
// a 32 (q) x 64 (node) tile goes through LDS so that both the reads (along
// nodes) and the writes (along q) are contiguous.
template <int PR>
__global__ void __launch_bounds__(256) relayout_kernel(const void* __restrict__ in, void* __restrict__ out, int64_t NN,
                                                       int nq) {
  using T = typename Store<PR>::type;
  __shared__ T tile[32][64 + 1];
  const int64_t g0 = (int64_t)blockIdx.x * 64;
  const int q0 = blockIdx.y * 32;
  const T* src = (const T*)in;
  T* dst = (T*)out;
  for (int i = threadIdx.x; i < 32 * 64; i += 256) {
    const int qq = i / 64, gg = i % 64;
    if (q0 + qq < nq && g0 + gg < NN) tile[qq][gg] = src[(int64_t)(q0 + qq) * NN + g0 + gg];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 32 * 64; i += 256) {
    const int gg = i / 32, qq = i % 32;
    if (q0 + qq < nq && g0 + gg < NN) dst[(g0 + gg) * nq + q0 + qq] = tile[qq][gg];
  }
}

static unsigned copy_grid(int64_t n) {
  const int64_t g = (n + 255) / 256;
  return (unsigned)(g > 65536 ? 65536 : g);
}

// A~ is formed node-fastest in Fwork, copied (At_copy, optional) in FP32,
// transposed to the element-major layout and factorised there in place; the
// factors end in Fem in storage precision fprec.  Fwork holds nF entries of
// the factorisation precision (FP64 for fprec = F64, FP32 otherwise) and, for
// BF16, a second FP32 array of nF after them (the element-major work copy).
hipError_t launch_precond_factor(const DevCtx& dc, const void* K11, const void* K12, int prec, double alpha,
                                 double gamma, void* Fwork, int fprec, void* Fem, float* At_copy) {
  const int64_t NN = dc.E * dc.NP;
  const int nq = (dc.D * dc.P + 1) * dc.M * dc.M;
  const int64_t nF = NN * (int64_t)nq;
  const dim3 tgrid((unsigned)((NN + 63) / 64), (unsigned)((nq + 31) / 32));
  LDG_DISPATCH(dc, {
    using L = FormLayout<D, P, EQ>;
    const size_t bytes = Eq<D, EQ>::VIS ? L::bytes : 0;
    LDG_PREC_DISPATCH(prec, {
      if (fprec == PREC_F64) {
        auto k = form_kernel<D, P, EQ, PR, PREC_F64>;
        if (bytes > 65536) hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        hipLaunchKernelGGL(k, dim3((unsigned)dc.E), dim3(NT_ELEM), bytes, dc.stream, dc.ops, dc.mp, K11, K12, alpha,
                           gamma, Fwork);
        if (At_copy)
          hipLaunchKernelGGL((convert_kernel<PREC_F64, PREC_F32>), dim3(copy_grid(nF)), dim3(256), 0, dc.stream, Fwork,
                             At_copy, nF);
        hipLaunchKernelGGL((relayout_kernel<PREC_F64>), tgrid, dim3(256), 0, dc.stream, Fwork, Fem, NN, nq);
        hipLaunchKernelGGL((factor_kernel<D, P, EQ, PREC_F64>), dim3((unsigned)dc.E), dim3(64), 0, dc.stream, dc.E,
                           Fem);
      } else {
        void* em = fprec == PREC_F32 ? Fem : (void*)((float*)Fwork + nF);
        auto k = form_kernel<D, P, EQ, PR, PREC_F32>;
        if (bytes > 65536) hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        hipLaunchKernelGGL(k, dim3((unsigned)dc.E), dim3(NT_ELEM), bytes, dc.stream, dc.ops, dc.mp, K11, K12, alpha,
                           gamma, Fwork);
        if (At_copy)
          hipLaunchKernelGGL((convert_kernel<PREC_F32, PREC_F32>), dim3(copy_grid(nF)), dim3(256), 0, dc.stream, Fwork,
                             At_copy, nF);
        hipLaunchKernelGGL((relayout_kernel<PREC_F32>), tgrid, dim3(256), 0, dc.stream, Fwork, em, NN, nq);
        hipLaunchKernelGGL((factor_kernel<D, P, EQ, PREC_F32>), dim3((unsigned)dc.E), dim3(64), 0, dc.stream, dc.E, em);
        if (fprec == PREC_BF16)
          hipLaunchKernelGGL((convert_kernel<PREC_F32, PREC_BF16>), dim3(copy_grid(nF)), dim3(256), 0, dc.stream, em,
                             Fem, nF);
      }
      return hipGetLastError();
    })
  })
}

// element-major factors -> FP64 [E][Np][slot][c][c'] (the same order)
hipError_t launch_factors_to_f64(const DevCtx& dc, const void* Fem, int fprec, double* out) {
  const int64_t n = dc.E * dc.NP * (int64_t)((dc.D * dc.P + 1) * dc.M * dc.M);
  LDG_PREC_DISPATCH(fprec, {
    hipLaunchKernelGGL((convert_kernel<PR, PREC_F64>), dim3(copy_grid(n)), dim3(256), 0, dc.stream, Fem, out, n);
    return hipGetLastError();
  })
}

// Fem: the element-major factors written by launch_precond_factor.
hipError_t launch_precond_apply(const DevCtx& dc, const void* F, int fprec, const double* r, double* z) {
  LDG_DISPATCH(dc, {
    LDG_PREC_DISPATCH(fprec, {
      hipLaunchKernelGGL((apply_kernel<D, P, EQ, PR>), dim3((unsigned)dc.E), dim3(64), 0, dc.stream, dc.E, F, r, z);
      return hipGetLastError();
    })
  })
}

}  // namespace ldg
