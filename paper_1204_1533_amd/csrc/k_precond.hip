// Split Jacobian-vector product and the element-local line-pattern
// preconditioner (Section 4.2 of the paper).
//
// jacvec:   y = alpha x - gamma (K11 x + K12 w), w = K21 x from the stored
//           K21 weights (eq. matvecsplit; K21 is the gradient operator with
//           zero boundary data, a function of the geometry only).  One
//           thread per node streams its block row (node-fastest layout, so a
//           wavefront reads contiguous memory for every (slot, c, c')); the
//           workgroup holds whole elements and stages their x and w in LDS.
// form:     A~ = alpha I - gamma (K11 + K12 K21) restricted to the D lines
//           through each node, K21 taken inside the element from its stored
//           weights: for a row a and a column b on its direction-n line,
//           (K12 K21)_ab = sum_{c on that line} K12_ac W_cb, with W_cb the
//           weight of row c at its slot of column b (for c = b the self slot,
//           which sums the D lines through b); for b = a the sum over c runs
//           over all D lines.
// factor:   block ILU(0) in natural node order.  Row i depends only on the
//           earlier nodes of its own lines, so rows with equal i+j(+k) form
//           independent levels; each row's lower blocks k update only blocks
//           on the line they share.  The diagonal slot keeps the inverse of
//           the U diagonal block.
// apply:    forward / backward block substitution over the same levels.
#include <type_traits>
#include <utility>

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
// Writes A~ = alpha I - gamma (K11 + K12 K21) on the line pattern in the
// working precision WP of the factorisation, node-fastest [slot][c][c'][E*Np]
// (EM = false) or element-major [E*Np][slot][c][c'] (EM = true).  K21 comes
// from its stored weights (row node, slot, d), the element's copied to LDS,
// so no geometry is recomputed.  One work item per (row node a, row component
// c); for each of the D lines through a, row c of K12 on the line's p+1 slots
// is loaded once and gives the p+1 output blocks on that line:
//   (K12 K21)_ab[c][k] = sum_{c' on the line, c' != b} K12_ac'[c][k,:] . W21(c' -> b)
//                      + K12_ab[c][k,:] . W21(b -> b)
// (W21(c' -> b): the weights of row c' at its slot of column b; W21(b -> b)
// the self slot, which sums b's D lines).  The self block (b = a) collects the
// c' != a terms of all D lines.
template <int D, int P>
__host__ __device__ constexpr size_t form_lds_bytes() {
  return sizeof(double) * (size_t)(D * P + 1) * D * ipow(P + 1, D);
}
template <int D, int P, int EQ, int PR, int WP, bool EM>
__global__ void __launch_bounds__(NT_ELEM) form_kernel(MeshParams mp, const void* __restrict__ K11,
                                                       const void* __restrict__ K12, const double* __restrict__ W21,
                                                       double alpha, double gamma, void* __restrict__ F) {
  constexpr int N1 = P + 1, NP = ipow(N1, D), M = Eq<D, EQ>::M;
  constexpr bool VIS = Eq<D, EQ>::VIS;
  constexpr int NSL = D * P + 1, MD = M * D;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* sK = reinterpret_cast<double*>(smem_raw);  // [line slot][d][node] of this element
  const int64_t e = blockIdx.x;
  const int64_t NN = mp.E * NP;
  if constexpr (VIS) {
    for (int i = threadIdx.x; i < NSL * D * NP; i += NT_ELEM) {
      const int sd = i / NP, node = i % NP;
      sK[i] = W21[sd * NN + e * NP + node];
    }
    __syncthreads();
  }
  using KT = typename std::conditional<PR == PREC_F64, double, float>::type;
#pragma unroll 1
  for (int it = threadIdx.x; it < NP * M; it += NT_ELEM) {
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
      if constexpr (VIS) {
#pragma unroll
        for (int tc = 0; tc < N1; ++tc) {
          const int sc = slot_of<N1>(n, ta, tc, self);
#pragma unroll
          for (int q = 0; q < MD; ++q) kc[tc][q] = (KT)Store<PR>::get(K12, ((int64_t)(sc * M + c) * MD + q) * NN + gn);
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
            const int cn = line_node<D, N1>(n, la, tc);
            const int sw = slot_of<N1>(n, tc, tb, cn % N1);  // column b in row c''s slots
            double w[D];
#pragma unroll
            for (int d = 0; d < D; ++d) w[d] = sK[(sw * D + d) * NP + cn];
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
            for (int d = 0; d < D; ++d) prod[k] += (double)kc[tb][k * D + d] * sK[((b % N1) * D + d) * NP + b];
        }
        const int slot = slot_of<N1>(n, ta, tb, self);
#pragma unroll
        for (int k = 0; k < M; ++k) {
          const double v = Store<PR>::get(K11, ((int64_t)(slot * M + c) * M + k) * NN + gn) + prod[k];
          Store<WP>::put(F, EM ? (gn * NSL + slot) * (M * M) + c * M + k : ((int64_t)(slot * M + c) * M + k) * NN + gn,
                         -gamma * v);
        }
      }
    }
    // self block: K11 + the c' != a terms of all lines + K12_aa . W21(a -> a)
#pragma unroll
    for (int k = 0; k < M; ++k) {
      double v = Store<PR>::get(K11, ((int64_t)(self * M + c) * M + k) * NN + gn) + self_acc[k];
      if constexpr (VIS) {
#pragma unroll
        for (int d = 0; d < D; ++d)
          v += Store<PR>::get(K12, ((int64_t)(self * M + c) * MD + k * D + d) * NN + gn) * sK[(self * D + d) * NP + a];
      }
      v = -gamma * v;
      if (c == k) v += alpha;
      Store<WP>::put(F, EM ? (gn * NSL + self) * (M * M) + c * M + k : ((int64_t)(self * M + c) * M + k) * NN + gn, v);
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

// Rows of the largest level of a (p+1)^D node grid: nodes with coordinate sum
// floor(D p / 2), times the m components.
template <int D, int P, int EQ>
__host__ __device__ constexpr int max_level_rows() {
  int best = 0;
  for (int L = 0; L <= D * P; ++L) {
    int cnt = 0;
    for (int a = 0; a < ipow(P + 1, D); ++a) {
      int s = 0, r = a;
      for (int d = 0; d < D; ++d) {
        s += r % (P + 1);
        r /= (P + 1);
      }
      cnt += s == L;
    }
    best = cnt > best ? cnt : best;
  }
  return best * Eq<D, EQ>::M;
}
// x = A^{-1} e_col by Gaussian elimination with partial pivoting (row swaps
// with compile-time indices, as in invert_block).
template <int M>
__device__ __forceinline__ void solve_unit_column(double A[M][M], int col, double x[M]) {
  double b[M];
#pragma unroll
  for (int i = 0; i < M; ++i) b[i] = i == col ? 1.0 : 0.0;
#pragma unroll
  for (int c = 0; c < M; ++c) {
    int piv = c;
    double best = fabs(A[c][c]);
#pragma unroll
    for (int r = c + 1; r < M; ++r)
      if (fabs(A[r][c]) > best) {
        best = fabs(A[r][c]);
        piv = r;
      }
#pragma unroll
    for (int r = c + 1; r < M; ++r)
      if (r == piv) {
#pragma unroll
        for (int j = 0; j < M; ++j) {
          const double t = A[c][j];
          A[c][j] = A[r][j];
          A[r][j] = t;
        }
        const double t = b[c];
        b[c] = b[r];
        b[r] = t;
      }
#pragma unroll
    for (int r = c + 1; r < M; ++r) {
      const double f = A[r][c] / A[c][c];
#pragma unroll
      for (int j = c; j < M; ++j) A[r][j] -= f * A[c][j];
      b[r] -= f * b[c];
    }
  }
#pragma unroll
  for (int i = M - 1; i >= 0; --i) {
    double s = b[i];
#pragma unroll
    for (int j = i + 1; j < M; ++j) s -= A[i][j] * x[j];
    x[i] = s / A[i][i];
  }
}

// Work items per element of the factorisation: enough for the largest level's
// rows in one pass (up to 256).
template <int D, int P, int EQ>
__host__ __device__ constexpr int factor_threads() {
  constexpr int r = max_level_rows<D, P, EQ>();
  return r <= 64 ? 64 : (r <= 128 ? 128 : 256);
}

// One workgroup per element; work items = (row of the current level, component row c).
template <int D, int P, int EQ, int WP>
__global__ void __launch_bounds__((factor_threads<D, P, EQ>())) factor_kernel(int64_t E, void* __restrict__ F) {
  constexpr int N1 = P + 1, NP = ipow(N1, D), M = Eq<D, EQ>::M;
  constexpr int NT = factor_threads<D, P, EQ>();
  constexpr int RPP = NT / M;  // rows per pass
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
      // inverse of the U diagonal block: work item c of the row takes column c
      // (A x = e_c by elimination with partial pivoting), all M in parallel
      double xcol[M];
      if (active) {
        const int64_t gi = e * NP + i;
        const int self_i = i % N1;
        double A[M][M];
#pragma unroll
        for (int a = 0; a < M; ++a)
#pragma unroll
          for (int b = 0; b < M; ++b) A[a][b] = Store<WP>::get(F, gi * NSLMM + (self_i * M + a) * M + b);
        solve_unit_column<M>(A, c, xcol);
      }
      __syncthreads();  // every column read the block before any is overwritten
      if (active) {
        const int64_t gi = e * NP + i;
        const int self_i = i % N1;
#pragma unroll
        for (int a = 0; a < M; ++a) Store<WP>::put(F, gi * NSLMM + (self_i * M + a) * M + c, xcol[a]);
      }
      __syncthreads();
    }
  }
}

// Block ILU(0) in FP32 working precision with each row in registers.  Work
// item (row node i, component c) of the current level loads row c of its
// node's line blocks once into registers: R[n][t] is the block of the node at
// position t of its direction-n line (the entry t = c_n, the node itself, is
// unused), Dg the diagonal block, shared by all D lines.  The elimination then
// touches memory only to read the finished rows k of earlier levels (their
// U diagonal inverse and right blocks), which no work item of the current
// level writes, so those loads carry no dependence on the row being
// eliminated.  Same operations in the same order as factor_kernel (FP64
// arithmetic on FP32 values), so the factors are the same.  Finished blocks go
// straight into the apply layout (precision FPOUT); of the element-major rows
// only the U parts, which later levels read, are written back.
template <int NR>
__device__ __forceinline__ int fac_off(int r, int j) {
  return ((j >> 2) * NR + r) * 4 + (j & 3);
}
template <int D, int P, int EQ, int FPOUT>
__global__ void __launch_bounds__((factor_threads<D, P, EQ>())) __attribute__((amdgpu_waves_per_eu(4)))
factor_reg_kernel(LevelOrder ord, float* __restrict__ F,
                                                                                void* __restrict__ Fem) {
  constexpr int N1 = P + 1, NP = ipow(N1, D), M = Eq<D, EQ>::M;
  constexpr int NT = factor_threads<D, P, EQ>();
  constexpr int RPP = NT / M;  // rows per pass
  constexpr int NSLMM = (D * P + 1) * M * M;
  constexpr int NR = NP * M, NJ = (D * P + 1) * M, NJP = (NJ + 3) / 4 * 4;
  __shared__ double sBlk[RPP][M][M];  // diagonal blocks of the pass's nodes
  const int64_t e = blockIdx.x;
  const int lane = threadIdx.x;
  const int gi = lane / M, c = lane % M;
  for (int L = 0; L <= D * P; ++L) {
    const int nrow = ord.off[L + 1] - ord.off[L];
    for (int r0 = 0; r0 < nrow; r0 += RPP) {
      const bool active = (lane < RPP * M) && r0 + gi < nrow;
      const int i = active ? ord.node[ord.off[L] + r0 + gi] : 0;
      int cd[D], lev = 0;
#pragma unroll
      for (int d = 0, r = i; d < D; ++d, r /= N1) {
        cd[d] = r % N1;
        lev += cd[d];
      }
      float* row = F + (e * NP + i) * NSLMM;
      const int rbase = M * (ord.off[L] + r0 + gi);  // apply-layout row of component 0 of node i
      // the element's factor rows: entry j of row r at ((j / 4) NR + r) 4 + j % 4
      void* fe = static_cast<char*>(Fem) + sizeof(typename Store<FPOUT>::type) * (size_t)(e * NR * NJP);
      if (active) {
        // the blocks of one direction's line change only while that direction
        // is eliminated: one line in registers at a time, the diagonal throughout
        float Dg[M];
#pragma unroll
        for (int q = 0; q < M; ++q) Dg[q] = row[(cd[0] * M + c) * M + q];
#pragma unroll
        for (int n = 0; n < D; ++n) {
          float R[N1][M];
#pragma unroll
          for (int t = 0; t < N1; ++t) {
            const int slot = n == 0 ? t : N1 + (n - 1) * P + (t < cd[n] ? t : t - 1);
#pragma unroll
            for (int q = 0; q < M; ++q) R[t][q] = t != cd[n] ? row[(slot * M + c) * M + q] : 0.0f;
          }
          int stride = 1;
#pragma unroll
          for (int d = 0; d < n; ++d) stride *= N1;
#pragma unroll
          for (int tk = 0; tk < P; ++tk) {
            if (tk < cd[n]) {
              const int k = i + (tk - cd[n]) * stride;
              const int self_k = n == 0 ? tk : cd[0];
              const float* krow = F + (e * NP + k) * NSLMM;
              // L_ik[c][:] = A_ik[c][:] Uinv_kk
              double lrow[M];
#pragma unroll
              for (int j = 0; j < M; ++j) {
                double s = 0.0;
#pragma unroll
                for (int q = 0; q < M; ++q) s += (double)R[tk][q] * (double)krow[(self_k * M + q) * M + j];
                lrow[j] = s;
              }
#pragma unroll
              for (int j = 0; j < M; ++j) R[tk][j] = (float)lrow[j];
              // A_ij -= L_ik U_kj for j after k on the line (the diagonal when t_j = c_n)
#pragma unroll
              for (int tj = tk + 1; tj < N1; ++tj) {
                const int skj = n == 0 ? tj : N1 + (n - 1) * P + tj - 1;
                const bool diag = tj == cd[n];
#pragma unroll
                for (int j = 0; j < M; ++j) {
                  double s = 0.0;
#pragma unroll
                  for (int q = 0; q < M; ++q) s += lrow[q] * (double)krow[(skj * M + q) * M + j];
                  const float v = (float)((double)(diag ? Dg[j] : R[tj][j]) - s);
                  if (diag)
                    Dg[j] = v;
                  else
                    R[tj][j] = v;
                }
              }
            }
          }
          // this line's L and U blocks are final: row positions (left blocks
          // of the earlier directions, then this line's; right blocks after
          // the diagonal likewise)
          int left = 0, right = lev + 1;
#pragma unroll
          for (int m = 0; m < n; ++m) {
            left += cd[m];
            right += P - cd[m];
          }
#pragma unroll
          for (int t = 0; t < N1; ++t) {
            const int slot = n == 0 ? t : N1 + (n - 1) * P + (t < cd[n] ? t : t - 1);
            if (t != cd[n]) {
              const int pos = t < cd[n] ? left + t : right + t - cd[n] - 1;
#pragma unroll
              for (int q = 0; q < M; ++q) {
                Store<FPOUT>::put(fe, fac_off<NR>(rbase + c, pos * M + q), R[t][q]);
                if (t > cd[n]) row[(slot * M + c) * M + q] = R[t][q];
              }
            }
          }
        }
#pragma unroll
        for (int j = NJ; j < NJP; ++j) Store<FPOUT>::put(fe, fac_off<NR>(rbase + c, j), 0.0);
#pragma unroll
        for (int q = 0; q < M; ++q) sBlk[gi][c][q] = Dg[q];
      }
      __syncthreads();
      // inverse of the U diagonal block: work item c takes column c
      if (active) {
        double A[M][M], xcol[M];
#pragma unroll
        for (int a = 0; a < M; ++a)
#pragma unroll
          for (int b = 0; b < M; ++b) A[a][b] = sBlk[gi][a][b];
        solve_unit_column<M>(A, c, xcol);
#pragma unroll
        for (int a = 0; a < M; ++a) {
          const float v = (float)xcol[a];
          row[(cd[0] * M + a) * M + c] = v;
          Store<FPOUT>::put(fe, fac_off<NR>(rbase + a, lev * M + c), v);
        }
      }
      __syncthreads();
    }
  }
}

// Registers of one factor row: NJP entries of precision FP, loaded 4 at a time
// (8 bytes for BF16, 16 for FP32, 32 for FP64) from the apply layout.
template <int FP, int NJP> struct RowRegs;
template <int NJP> struct RowRegs<PREC_BF16, NJP> {
  uint2 v[NJP / 4];
  __device__ __forceinline__ void load(const void* F, int64_t base, int NR) {
    const uint2* p = reinterpret_cast<const uint2*>(F);
#pragma unroll
    for (int ch = 0; ch < NJP / 4; ++ch) v[ch] = p[(base + (int64_t)ch * NR * 4) / 4];
  }
  __device__ __forceinline__ double get(int j) const {
    const uint32_t w = (j & 2) ? v[j >> 2].y : v[j >> 2].x;
    return bf16_to_f32((uint16_t)((j & 1) ? (w >> 16) : (w & 0xFFFFu)));
  }
};
template <int NJP> struct RowRegs<PREC_F32, NJP> {
  float4 v[NJP / 4];
  __device__ __forceinline__ void load(const void* F, int64_t base, int NR) {
    const float4* p = reinterpret_cast<const float4*>(F);
#pragma unroll
    for (int ch = 0; ch < NJP / 4; ++ch) v[ch] = p[(base + (int64_t)ch * NR * 4) / 4];
  }
  __device__ __forceinline__ double get(int j) const {
    const float4& q = v[j >> 2];
    const int k = j & 3;
    return k == 0 ? q.x : (k == 1 ? q.y : (k == 2 ? q.z : q.w));
  }
};
template <int NJP> struct RowRegs<PREC_F64, NJP> {
  double2 v[NJP / 2];
  __device__ __forceinline__ void load(const void* F, int64_t base, int NR) {
    const double2* p = reinterpret_cast<const double2*>(F);
#pragma unroll
    for (int ch = 0; ch < NJP / 4; ++ch) {
      v[2 * ch] = p[(base + (int64_t)ch * NR * 4) / 2];
      v[2 * ch + 1] = p[(base + (int64_t)ch * NR * 4) / 2 + 1];
    }
  }
  __device__ __forceinline__ double get(int j) const { return (j & 1) ? v[j >> 1].y : v[j >> 1].x; }
};

template <int D, int P>
__device__ __forceinline__ int node_level(int a) {
  constexpr int N1 = P + 1;
  int s = 0;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    s += a % N1;
    a /= N1;
  }
  return s;
}

template <int D, int P, int EQ>
struct ApplyShape {
  static constexpr int TPE = max_level_rows<D, P, EQ>();  // work items per element: one level's rows
  static constexpr int EPB = TPE >= 128 ? 1 : 128 / TPE;  // elements per workgroup
  static constexpr int NT = (EPB * TPE + 63) / 64 * 64;
};

// z = (L U)^{-1} r element by element, by level: rows with equal a_0 + .. +
// a_{D-1} are independent.  The work items of an element take the rows of one
// level at a time (one row each: node a, component c).  A row of level L
// stores its L left blocks first, then the diagonal block (the inverse of the
// U diagonal block), then the D p - L right blocks, so with the levels
// unrolled at compile time the forward sweep at level L reads exactly the
// row's first L blocks and the backward sweep the rest, each once, with no
// masked slots:
//   y_a = r_a - sum_{left k} L_ak y_k,   z_a = U_aa^{-1} (y_a - sum_{right j} U_aj z_j).
// The factor rows of a level are one contiguous run read 4 entries at a time;
// y and t live in LDS node-major (the m values of a node in one 16-byte
// aligned run, read with 16-byte loads).
template <int M>
struct NodeRun {
  static constexpr int YS = (M + 1) / 2 * 2;  // doubles per node in LDS
  double v[YS];
  __device__ __forceinline__ void load(const double* base) {
#pragma unroll
    for (int q = 0; q < YS; q += 2) {
      const double2 w = *reinterpret_cast<const double2*>(base + q);
      v[q] = w.x;
      v[q + 1] = w.y;
    }
  }
};

template <int D, int P>
__device__ __forceinline__ void node_coords(int a, int* cd) {
#pragma unroll
  for (int d = 0; d < D; ++d) {
    cd[d] = a % (P + 1);
    a /= P + 1;
  }
}

template <int D, int P, int EQ, int FP, int L>
__device__ __forceinline__ void apply_forward_level(const LevelOrder& ord, int64_t e, bool live, int lane,
                                                    const void* F, double* y) {
  using S = FacShape<D, P, EQ>;
  constexpr int N1 = P + 1, M = S::M, NR = S::NR, NJP = S::NJP, YS = NodeRun<M>::YS;
  constexpr int NCH = (L * M + 3) / 4;  // chunks holding the L left blocks
  const int row = ord.off[L] * M + lane;
  if (live && row < ord.off[L + 1] * M) {
    RowRegs<FP, 4 * NCH> f;
    f.load(F, fac_index(e, row, 0, NR, NJP), NR);
    const int a = ord.node[row / M], c = row % M;
    // the u-th left block sits on the line of the direction whose positions u falls in:
    // column = base_d + u stride_d with thresholds hi_d (positions before direction d + 1)
    int base[D], hi[D];
    {
      int cd[D];
      node_coords<D, P>(a, cd);
      int before = 0, stride = 1;
#pragma unroll
      for (int d = 0; d < D; ++d) {
        base[d] = a - (cd[d] + before) * stride;
        before += cd[d];
        hi[d] = before;
        stride *= N1;
      }
    }
    double acc = y[a * YS + c];
#pragma unroll
    for (int u = 0; u < L; ++u) {
      int col = base[D - 1] + u * ipow(N1, D - 1);
#pragma unroll
      for (int d = D - 2; d >= 0; --d) col = u < hi[d] ? base[d] + u * ipow(N1, d) : col;
      NodeRun<M> yk;
      yk.load(y + col * YS);
      double tt = 0.0;  // one block at a time: short dependency chains
#pragma unroll
      for (int q = 0; q < M; ++q) tt += f.get(u * M + q) * yk.v[q];
      acc -= tt;
      // blocks one after another: hoisting every block's loads would hold them all in registers
      // and cost resident wavefronts; the other wavefronts hide the LDS latency
      __builtin_amdgcn_sched_barrier(0);
    }
    y[a * YS + c] = acc;
  }
  __syncthreads();
}

template <int D, int P, int EQ, int FP, int L>
__device__ __forceinline__ void apply_backward_level(const LevelOrder& ord, int64_t e, bool live, int lane,
                                                     const void* F, double* y, double* t) {
  using S = FacShape<D, P, EQ>;
  constexpr int N1 = P + 1, M = S::M, NR = S::NR, NJP = S::NJP, YS = NodeRun<M>::YS;
  constexpr int NUP = D * P - L;            // right blocks
  constexpr int C0 = (L * M) / 4;           // first chunk holding the diagonal block
  constexpr int NCH = NJP / 4 - C0;
  constexpr int OFF = 4 * C0;               // entry held in register 0
  const int row = ord.off[L] * M + lane;
  const bool act = live && row < ord.off[L + 1] * M;
  RowRegs<FP, 4 * NCH> f;
  int a = 0, c = 0;
  if (act) {
    f.load(F, fac_index(e, row, OFF, NR, NJP), NR);
    a = ord.node[row / M];
    c = row % M;
    // the u-th right block: column = base_d + u stride_d, d the direction whose positions u falls in
    int base[D], hi[D];
    {
      int cd[D];
      node_coords<D, P>(a, cd);
      int before = 0, stride = 1;
#pragma unroll
      for (int d = 0; d < D; ++d) {
        base[d] = a + (1 - before) * stride;
        before += P - cd[d];
        hi[d] = before;
        stride *= N1;
      }
    }
    double acc = y[a * YS + c];
#pragma unroll
    for (int u = 0; u < NUP; ++u) {
      int col = base[D - 1] + u * ipow(N1, D - 1);
#pragma unroll
      for (int d = D - 2; d >= 0; --d) col = u < hi[d] ? base[d] + u * ipow(N1, d) : col;
      NodeRun<M> zj;
      zj.load(y + col * YS);
      double tt = 0.0;
#pragma unroll
      for (int q = 0; q < M; ++q) tt += f.get((L + 1 + u) * M + q - OFF) * zj.v[q];
      acc -= tt;
      __builtin_amdgcn_sched_barrier(0);
    }
    t[a * YS + c] = acc;
  }
  __syncthreads();
  if (act) {
    NodeRun<M> ta;
    ta.load(t + a * YS);
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < M; ++q) v += f.get(L * M + q - OFF) * ta.v[q];
    y[a * YS + c] = v;
  }
  __syncthreads();
}

template <int D, int P, int EQ, int FP, int... Ls>
__device__ __forceinline__ void apply_forward_all(std::integer_sequence<int, Ls...>, const LevelOrder& ord, int64_t e,
                                                  bool live, int lane, const void* F, double* y) {
  (apply_forward_level<D, P, EQ, FP, Ls + 1>(ord, e, live, lane, F, y), ...);
}
template <int D, int P, int EQ, int FP, int... Ls>
__device__ __forceinline__ void apply_backward_all(std::integer_sequence<int, Ls...>, const LevelOrder& ord, int64_t e,
                                                   bool live, int lane, const void* F, double* y, double* t) {
  (apply_backward_level<D, P, EQ, FP, D * P - Ls>(ord, e, live, lane, F, y, t), ...);
}

template <int D, int P, int EQ, int FP>
__global__ void __launch_bounds__((ApplyShape<D, P, EQ>::NT)) apply_kernel(LevelOrder ord, int64_t E,
                                                                          const void* __restrict__ F,
                                                                          const double* __restrict__ r,
                                                                          double* __restrict__ z) {
  using S = FacShape<D, P, EQ>;
  using A = ApplyShape<D, P, EQ>;
  constexpr int NP = S::NP, M = S::M, NR = S::NR;
  constexpr int TPE = A::TPE, EPB = A::EPB, YS = NodeRun<M>::YS;
  __shared__ __align__(16) double sy[EPB * NP * YS];
  __shared__ __align__(16) double st[EPB * NP * YS];
  const int tid = threadIdx.x;
  const int le = tid / TPE, lane = tid % TPE;
  const int64_t e = (int64_t)blockIdx.x * EPB + le;
  const bool live = le < EPB && e < E;
  double* y = sy + (le < EPB ? le : 0) * NP * YS;
  double* t = st + (le < EPB ? le : 0) * NP * YS;
  if (live)
    for (int i = lane; i < NR; i += TPE) y[(i % NP) * YS + i / NP] = r[e * NR + i];
  __syncthreads();
  // forward over levels 1 .. D p (level 0 has no left blocks), backward over D p .. 0
  apply_forward_all<D, P, EQ, FP>(std::make_integer_sequence<int, D * P>{}, ord, e, live, lane, F, y);
  apply_backward_all<D, P, EQ, FP>(std::make_integer_sequence<int, D * P + 1>{}, ord, e, live, lane, F, y, t);
  if (live)
    for (int i = lane; i < NR; i += TPE) z[e * NR + i] = y[(i % NP) * YS + i / NP];
}

// element-major factors [E Np][slot][c][c'] -> apply layout (zero padding):
// one work item per 4-entry chunk of a row, written with one 8- to 32-byte
// store; the slot at each row position comes from a table in LDS.
constexpr int FAC_TABLE_MAX = NPMAX * 13;  // Np (Dp + 1) for p <= 4
template <int PIN, int POUT>
__global__ void __launch_bounds__(256) em_to_fac_kernel(LevelOrder ord, const void* __restrict__ in,
                                                        void* __restrict__ out, int64_t E, int NP, int M, int NSL,
                                                        int D, int P) {
  using T = typename Store<POUT>::type;
  struct alignas(4 * sizeof(T)) T4 {
    T x[4];
  };
  __shared__ int8_t slot_at[FAC_TABLE_MAX];
  for (int i = threadIdx.x; i < NP * NSL; i += blockDim.x) slot_at[i] = (int8_t)row_slot_at(D, P, i / NSL, i % NSL);
  __syncthreads();
  const int NR = NP * M, NJ = NSL * M, NJP = (NJ + 3) / 4 * 4;
  const int64_t total = E * (int64_t)(NJP / 4) * NR;  // chunks
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int rr = (int)(i % NR);
    const int64_t q2 = i / NR;
    const int ch = (int)(q2 % (NJP / 4));
    const int64_t e = q2 / (NJP / 4);
    const int a = ord.node[rr / M], c = rr % M;
    T4 w;
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int j = ch * 4 + jj;
      double x = 0.0;
      if (j < NJ) {
        const int slot = slot_at[a * NSL + j / M];
        x = Store<PIN>::get(in, ((e * NP + a) * NSL + slot) * (int64_t)(M * M) + c * M + j % M);
      }
      Store<POUT>::put(w.x, jj, x);
    }
    reinterpret_cast<T4*>(out)[i] = w;
  }
}

// apply layout -> FP64 [E][Np][slot][c][c'] (the exchange layout of ldg_export_operators)
template <int PIN>
__global__ void fac_to_em64_kernel(LevelOrder ord, const void* __restrict__ in, double* __restrict__ out, int64_t E,
                                   int NP, int M, int NSL, int D, int P) {
  const int NR = NP * M, NJP = (NSL * M + 3) / 4 * 4;
  const int64_t total = E * NP * (int64_t)NSL * M * M;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int cp = (int)(i % M);
    const int c = (int)((i / M) % M);
    const int slot = (int)((i / (M * M)) % NSL);
    const int64_t gn = i / ((int64_t)M * M * NSL);
    const int64_t e = gn / NP;
    const int a = (int)(gn % NP);
    out[i] = Store<PIN>::get(in, fac_index(e, ord.rank[a] * M + c, row_pos_of(D, P, a, slot) * M + cp, NR, NJP));
  }
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

// A~ is formed element-major in the second half of Fwork (or, when the
// learned correction needs an FP32 node-fastest copy in At_copy, formed
// node-fastest in Fwork, copied and transposed there) and factorised in place (FP64 arithmetic for FP64 factors, FP32
// otherwise), then rearranged into the apply layout in Fem in storage
// precision fprec.  With dense != null the element-major A~ is instead
// expanded and factorised exactly (dense [E][NR][NR] LU in FP64).
hipError_t launch_precond_factor(const DevCtx& dc, const void* K11, const void* K12, const double* K21w, int prec,
                                 double alpha, double gamma, void* Fwork, int fprec, void* Fem, float* At_copy,
                                 double* dense) {
  const int64_t NN = dc.E * dc.NP;
  const int nsl = dc.D * dc.P + 1;
  const int nq = nsl * dc.M * dc.M;
  const int64_t nF = NN * (int64_t)nq;
  const int NR = dc.NP * dc.M, NJP = (nsl * dc.M + 3) / 4 * 4;
  const int64_t nFac = dc.E * (int64_t)NR * NJP;
  const dim3 tgrid((unsigned)((NN + 63) / 64), (unsigned)((nq + 31) / 32));
  LDG_DISPATCH(dc, {
    static_assert(form_lds_bytes<D, P>() <= LDS_PER_CU, "the element's K21 weights must fit one CU's LDS");
    const size_t bytes = Eq<D, EQ>::VIS ? form_lds_bytes<D, P>() : 0;
    if (Eq<D, EQ>::VIS && !K21w) return hipErrorInvalidValue;
    LDG_PREC_DISPATCH(prec, {
      if (fprec == PREC_F64) {
        double* em = (double*)Fwork + nF;
        auto k = At_copy ? form_kernel<D, P, EQ, PR, PREC_F64, false> : form_kernel<D, P, EQ, PR, PREC_F64, true>;
        if (bytes > 65536) {
          const hipError_t err =
              hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
          if (err != hipSuccess) return err;
        }
        hipLaunchKernelGGL(k, dim3((unsigned)dc.E), dim3(NT_ELEM), bytes, dc.stream, dc.mp, K11, K12, K21w, alpha,
                           gamma, At_copy ? Fwork : (void*)em);
        if (At_copy) {
          hipLaunchKernelGGL((convert_kernel<PREC_F64, PREC_F32>), dim3(copy_grid(nF)), dim3(256), 0, dc.stream, Fwork,
                             At_copy, nF);
          hipLaunchKernelGGL((relayout_kernel<PREC_F64>), tgrid, dim3(256), 0, dc.stream, Fwork, em, NN, nq);
        }
        if (dense) return launch_blocklu_factor(dc, em, PREC_F64, dense);
        hipLaunchKernelGGL((factor_kernel<D, P, EQ, PREC_F64>), dim3((unsigned)dc.E), dim3(factor_threads<D, P, EQ>()), 0,
                           dc.stream, dc.E,
                           em);
        hipLaunchKernelGGL((em_to_fac_kernel<PREC_F64, PREC_F64>), dim3(copy_grid(nFac / 4)), dim3(256), 0, dc.stream, dc.lev,
                           em, Fem, dc.E, dc.NP, dc.M, nsl, dc.D, dc.P);
      } else {
        float* em = (float*)Fwork + nF;
        auto k = At_copy ? form_kernel<D, P, EQ, PR, PREC_F32, false> : form_kernel<D, P, EQ, PR, PREC_F32, true>;
        if (bytes > 65536) {
          const hipError_t err =
              hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
          if (err != hipSuccess) return err;
        }
        hipLaunchKernelGGL(k, dim3((unsigned)dc.E), dim3(NT_ELEM), bytes, dc.stream, dc.mp, K11, K12, K21w, alpha,
                           gamma, At_copy ? Fwork : (void*)em);
        if (At_copy) {
          hipLaunchKernelGGL((convert_kernel<PREC_F32, PREC_F32>), dim3(copy_grid(nF)), dim3(256), 0, dc.stream, Fwork,
                             At_copy, nF);
          hipLaunchKernelGGL((relayout_kernel<PREC_F32>), tgrid, dim3(256), 0, dc.stream, Fwork, em, NN, nq);
        }
        if (dense) return launch_blocklu_factor(dc, em, PREC_F32, dense);
        if (fprec == PREC_BF16)
          hipLaunchKernelGGL((factor_reg_kernel<D, P, EQ, PREC_BF16>), dim3((unsigned)dc.E),
                             dim3(factor_threads<D, P, EQ>()), 0, dc.stream, dc.lev, em, Fem);
        else
          hipLaunchKernelGGL((factor_reg_kernel<D, P, EQ, PREC_F32>), dim3((unsigned)dc.E),
                             dim3(factor_threads<D, P, EQ>()), 0, dc.stream, dc.lev, em, Fem);
      }
      return hipGetLastError();
    })
  })
}

// apply-layout factors -> FP64 [E][Np][slot][c][c']
hipError_t launch_factors_to_f64(const DevCtx& dc, const void* Fem, int fprec, double* out) {
  const int nsl = dc.D * dc.P + 1;
  const int64_t n = dc.E * dc.NP * (int64_t)(nsl * dc.M * dc.M);
  LDG_PREC_DISPATCH(fprec, {
    hipLaunchKernelGGL((fac_to_em64_kernel<PR>), dim3(copy_grid(n)), dim3(256), 0, dc.stream, dc.lev, Fem, out, dc.E,
                       dc.NP, dc.M, nsl, dc.D, dc.P);
    return hipGetLastError();
  })
}

// Fem: the factors in the apply layout written by launch_precond_factor.
hipError_t launch_precond_apply(const DevCtx& dc, const void* F, int fprec, const double* r, double* z) {
  LDG_DISPATCH(dc, {
    using A = ApplyShape<D, P, EQ>;
    const unsigned grid = (unsigned)((dc.E + A::EPB - 1) / A::EPB);
    LDG_PREC_DISPATCH(fprec, {
      hipLaunchKernelGGL((apply_kernel<D, P, EQ, PR>), dim3(grid), dim3(A::NT), 0, dc.stream, dc.lev, dc.E, F, r, z);
      return hipGetLastError();
    })
  })
}

}  // namespace ldg
