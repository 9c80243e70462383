// Exact element-block preconditioner (Section 4.2): the element-local
// line-pattern block A~_e (alpha I - gamma (K11 + K12 K21) restricted to the D
// lines through each node, K21 inside the element) is factorised exactly,
// A~_e = L U, instead of by block ILU(0).  The paper factorises these blocks
// with a sparse direct LU; here each block is expanded to a dense NR x NR
// matrix (NR = Np m, row a m + c for node a, component c) and factorised in
// place by a blocked right-looking LU without pivoting (unit lower L), one
// workgroup per element:
//   panel    the B columns k0..k0+B of rows k0..NR-1, unblocked, rows held in
//            registers, the pivot row broadcast through LDS;
//   row blk  U12 = L11^{-1} A12, one column per work item;
//   update   A22 -= L21 U12 in 64 x 64 tiles, L21 and U12 tiles in LDS,
//            4 x 4 outputs per work item.
// No pivoting: A~ has the M-matrix-like diagonal dominance of alpha I - gamma A
// for the time steps used, and for alpha = 0 the Poisson block is definite.
// The apply solves L y = r, U z = y per element in 64-row blocks: the
// off-diagonal part of a block row as wavefront dot products (lanes along the
// row), the 64 x 64 diagonal block by one wavefront with shuffles.
#include "ldg_dispatch.hpp"
#include "ldg_kernels.hpp"
#include "ldg_store.hpp"

namespace ldg {

namespace {
constexpr int LU_B = 16;     // panel width
constexpr int LU_NT = 256;   // work items per element
constexpr int LU_RPT = 3;    // panel rows per work item: NR <= 768
constexpr int LU_TILE = 64;  // trailing-update tile
}  // namespace

template <int PR>
__global__ void zero_kernel(double* __restrict__ A, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    A[i] = 0.0;
}

// element-major A~ [E Np][slot][c][c'] (precision PR) -> dense [E][NR][NR]
template <int D, int P, int EQ, int PR>
__global__ void expand_kernel(const void* __restrict__ em, double* __restrict__ A, int64_t E) {
  constexpr int N1 = P + 1, NP = ipow(N1, D), M = Eq<D, EQ>::M, NSL = D * P + 1, NR = NP * M;
  constexpr int NQ = NSL * M * M;
  const int64_t total = E * NP * (int64_t)NQ;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int q = (int)(i % NQ);
    const int64_t gn = i / NQ;
    const int64_t e = gn / NP;
    const int a = (int)(gn % NP);
    const int s = q / (M * M), c = (q / M) % M, k = q % M;
    const int b = slot_col<D, P>(a, s);
    A[(e * NR + a * M + c) * NR + b * M + k] = Store<PR>::get(em, i);
  }
}

__global__ void __launch_bounds__(LU_NT) dense_lu_kernel(double* __restrict__ Aall, int NR) {
  double* A = Aall + (int64_t)blockIdx.x * NR * NR;
  __shared__ double sRow[LU_B];
  __shared__ double sP[LU_B][LU_B + 1];
  __shared__ double sL[LU_TILE][LU_B + 1];
  __shared__ double sU[LU_B][LU_TILE + 1];
  const int tid = threadIdx.x;
  for (int k0 = 0; k0 < NR; k0 += LU_B) {
    const int kb = NR - k0 < LU_B ? NR - k0 : LU_B;
    const int k1 = k0 + kb;
    // ---- panel: rows k0 + tid + LU_NT q, columns k0 .. k1-1
    double a[LU_RPT][LU_B];
#pragma unroll
    for (int q = 0; q < LU_RPT; ++q) {
      const int i = k0 + tid + LU_NT * q;
#pragma unroll
      for (int j = 0; j < LU_B; ++j) a[q][j] = (i < NR && j < kb) ? A[(int64_t)i * NR + k0 + j] : 0.0;
    }
    for (int j = 0; j < kb; ++j) {
      // row k0 + j is held by work item j (q = 0): its entries j..kb-1 are the pivot row
      if (tid == j) {
#pragma unroll
        for (int jj = 0; jj < LU_B; ++jj) sRow[jj] = a[0][jj];
      }
      __syncthreads();
      const double piv = sRow[j];
#pragma unroll
      for (int q = 0; q < LU_RPT; ++q) {
        const int i = k0 + tid + LU_NT * q;
        if (i > k0 + j && i < NR) {
          double l = 0.0;
#pragma unroll
          for (int jj = 0; jj < LU_B; ++jj)
            if (jj == j) l = a[q][jj] / piv;
#pragma unroll
          for (int jj = 0; jj < LU_B; ++jj) {
            if (jj == j) a[q][jj] = l;
            if (jj > j && jj < kb) a[q][jj] -= l * sRow[jj];
          }
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < LU_RPT; ++q) {
      const int i = k0 + tid + LU_NT * q;
      if (i < NR) {
#pragma unroll
        for (int j = 0; j < LU_B; ++j)
          if (j < kb) A[(int64_t)i * NR + k0 + j] = a[q][j];
      }
      if (q == 0 && tid < kb) {
#pragma unroll
        for (int j = 0; j < LU_B; ++j) sP[tid][j] = a[0][j];
      }
    }
    __syncthreads();
    if (k1 >= NR) break;
    // ---- row block: U12 = L11^{-1} A12 (L11 unit lower, in sP)
    for (int jc = k1 + tid; jc < NR; jc += LU_NT) {
      double x[LU_B];
#pragma unroll
      for (int i = 0; i < LU_B; ++i) {
        if (i < kb) {
          double v = A[(int64_t)(k0 + i) * NR + jc];
#pragma unroll
          for (int m = 0; m < LU_B; ++m)
            if (m < i) v -= sP[i][m] * x[m];
          x[i] = v;
          A[(int64_t)(k0 + i) * NR + jc] = v;
        } else {
          x[i] = 0.0;
        }
      }
    }
    __syncthreads();
    // ---- trailing update: A22 -= L21 U12
    const int n2 = NR - k1;
    const int nt = (n2 + LU_TILE - 1) / LU_TILE;
    for (int t = 0; t < nt * nt; ++t) {
      const int r0 = k1 + (t / nt) * LU_TILE, c0 = k1 + (t % nt) * LU_TILE;
      for (int i = tid; i < LU_TILE * LU_B; i += LU_NT) {
        const int rr = i / LU_B, m = i % LU_B;
        sL[rr][m] = (r0 + rr < NR && m < kb) ? A[(int64_t)(r0 + rr) * NR + k0 + m] : 0.0;
      }
      for (int i = tid; i < LU_TILE * LU_B; i += LU_NT) {
        const int m = i / LU_TILE, cc = i % LU_TILE;
        sU[m][cc] = (c0 + cc < NR && m < kb) ? A[(int64_t)(k0 + m) * NR + c0 + cc] : 0.0;
      }
      __syncthreads();
      const int ri = (tid / 16) * 4, ci = (tid % 16) * 4;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int r = r0 + ri + u;
        if (r >= NR) continue;
        double acc[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] = 0.0;
#pragma unroll
        for (int m = 0; m < LU_B; ++m) {
          const double l = sL[ri + u][m];
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[v] += l * sU[m][ci + v];
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int c = c0 + ci + v;
          if (c < NR) A[(int64_t)r * NR + c] -= acc[v];
        }
      }
      __syncthreads();
    }
  }
}

// z = U^{-1} L^{-1} r for every element; r, z component-major [E][m][Np]
__global__ void __launch_bounds__(LU_NT) dense_lu_apply_kernel(const double* __restrict__ LUall,
                                                              const double* __restrict__ r, double* __restrict__ z,
                                                              int NP, int M) {
  const int NR = NP * M;
  const int64_t e = blockIdx.x;
  const double* LU = LUall + e * (int64_t)NR * NR;
  __shared__ double y[768];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int i = tid; i < NR; i += LU_NT) y[(i % NP) * M + i / NP] = r[e * NR + i];
  __syncthreads();
  // ---- forward: L y = r (unit lower)
  for (int I0 = 0; I0 < NR; I0 += 64) {
    const int nb = NR - I0 < 64 ? NR - I0 : 64;
    // rows of the block minus the columns before it
    for (int rr = wv; rr < nb; rr += 4) {
      const int i = I0 + rr;
      double s = 0.0;
      for (int j = lane; j < I0; j += 64) s += LU[(int64_t)i * NR + j] * y[j];
      for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
      if (lane == 0) y[i] -= s;
    }
    __syncthreads();
    if (wv == 0) {
      double yi = lane < nb ? y[I0 + lane] : 0.0;
      for (int j = 0; j < nb; ++j) {
        const double yj = __shfl(yi, j, 64);
        if (lane > j && lane < nb) yi -= LU[(int64_t)(I0 + lane) * NR + I0 + j] * yj;
      }
      if (lane < nb) y[I0 + lane] = yi;
    }
    __syncthreads();
  }
  // ---- backward: U z = y
  const int nblk = (NR + 63) / 64;
  for (int bi = nblk - 1; bi >= 0; --bi) {
    const int I0 = bi * 64;
    const int nb = NR - I0 < 64 ? NR - I0 : 64;
    const int I1 = I0 + nb;
    for (int rr = wv; rr < nb; rr += 4) {
      const int i = I0 + rr;
      double s = 0.0;
      for (int j = I1 + lane; j < NR; j += 64) s += LU[(int64_t)i * NR + j] * y[j];
      for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
      if (lane == 0) y[i] -= s;
    }
    __syncthreads();
    if (wv == 0) {
      double yi = lane < nb ? y[I0 + lane] : 0.0;
      for (int j = nb - 1; j >= 0; --j) {
        double zj = 0.0;
        if (lane == j) zj = yi / LU[(int64_t)(I0 + j) * NR + I0 + j];
        zj = __shfl(zj, j, 64);
        if (lane == j) yi = zj;
        if (lane < j) yi -= LU[(int64_t)(I0 + lane) * NR + I0 + j] * zj;
      }
      if (lane < nb) y[I0 + lane] = yi;
    }
    __syncthreads();
  }
  for (int i = tid; i < NR; i += LU_NT) z[e * NR + i] = y[(i % NP) * M + i / NP];
}

hipError_t launch_blocklu_factor(const DevCtx& dc, const void* em, int emprec, double* A) {
  const int NR = dc.NP * dc.M;
  if (NR > LU_RPT * LU_NT || NR > 768) return hipErrorInvalidValue;
  const int64_t n = dc.E * (int64_t)NR * NR;
  const int64_t g = (n + 255) / 256;
  hipLaunchKernelGGL(zero_kernel<0>, dim3((unsigned)(g > 65536 ? 65536 : g)), dim3(256), 0, dc.stream, A, n);
  LDG_DISPATCH(dc, {
    const int64_t m = dc.E * ipow(P + 1, D) * (int64_t)((D * P + 1) * Eq<D, EQ>::M * Eq<D, EQ>::M);
    const int64_t g2 = (m + 255) / 256;
    const unsigned grid = (unsigned)(g2 > 65536 ? 65536 : g2);
    if (emprec == PREC_F64)
      hipLaunchKernelGGL((expand_kernel<D, P, EQ, PREC_F64>), dim3(grid), dim3(256), 0, dc.stream, em, A, dc.E);
    else
      hipLaunchKernelGGL((expand_kernel<D, P, EQ, PREC_F32>), dim3(grid), dim3(256), 0, dc.stream, em, A, dc.E);
    hipLaunchKernelGGL(dense_lu_kernel, dim3((unsigned)dc.E), dim3(LU_NT), 0, dc.stream, A, NR);
    return hipGetLastError();
  })
}

hipError_t launch_blocklu_apply(const DevCtx& dc, const double* LU, const double* r, double* z) {
  if (dc.NP * dc.M > 768) return hipErrorInvalidValue;
  hipLaunchKernelGGL(dense_lu_apply_kernel, dim3((unsigned)dc.E), dim3(LU_NT), 0, dc.stream, LU, r, z, dc.NP, dc.M);
  return hipGetLastError();
}

}  // namespace ldg
