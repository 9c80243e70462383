// Learned correction of the element-local line-pattern preconditioner (an
// addition beyond the paper; the preconditioner it corrects is the block
// ILU(0) of A~ from Section 4.2).
//
// Per element, with D_b the m x m diagonal block of A~ at node b:
//   features  X = [ D_b / sigma (node-major), G / max|G| (node-major) ],
//             sigma = max |entries of all D_b|, G = -gamma R(U) the residual
//             part of the Newton function at the assembly state;
//   network   Y = MLP(X) read as Np blocks Y_b (m x m);
//   blocks    C_b = Y_b D_b^{-1};
//   apply     z = z0 + C (r - A~ z0), z0 = ILU(0)^{-1} r, element by element,
//             so z stays linear in r;
//   training  samples (A~_e rows, s = v - A~ ILU^{-1} v, t = D^{-1} s, both
//             over ||v_e||) and the loss L = sum ||s - A~ (Y t)||^2 scaled by
//             1 / (n K), with dL/dY_b = -2 scale (A~^T rho)_b t_b^T.
// A~ is kept as an FP32 copy in the factor layout [slot][c][c'][E Np]; C is
// stored node-fastest [c][c'][E Np].
#include "ldg_dispatch.hpp"
#include "ldg_kernels.hpp"
#include "ldg_store.hpp"

namespace ldg {

template <int D, int P, int EQ>
struct LearnedDims {
  static constexpr int N1 = P + 1, NP = ipow(N1, D), M = Eq<D, EQ>::M, NSL = D * P + 1;
  static constexpr int NOUT = NP * M * M, NIN = NOUT + NP * M;
};

constexpr int NT_L = 128;

__device__ __forceinline__ float block_max(float v, float* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = NT_L / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  const float r = red[0];
  __syncthreads();
  return r;
}
__device__ __forceinline__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = NT_L / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// In-place inverse of an M x M matrix (Gauss-Jordan, partial pivoting).
template <int M>
__device__ __forceinline__ void invert(double (&A)[M][M], double (&I)[M][M]) {
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int j = 0; j < M; ++j) I[i][j] = i == j ? 1.0 : 0.0;
#pragma unroll
  for (int k = 0; k < M; ++k) {
    int piv = k;
    double best = fabs(A[k][k]);
#pragma unroll
    for (int i = k + 1; i < M; ++i)
      if (fabs(A[i][k]) > best) {
        best = fabs(A[i][k]);
        piv = i;
      }
#pragma unroll
    for (int i = k + 1; i < M; ++i)
      if (i == piv) {
#pragma unroll
        for (int j = 0; j < M; ++j) {
          double t = A[k][j];
          A[k][j] = A[i][j];
          A[i][j] = t;
          t = I[k][j];
          I[k][j] = I[i][j];
          I[i][j] = t;
        }
      }
    const double inv = 1.0 / A[k][k];
#pragma unroll
    for (int j = 0; j < M; ++j) {
      A[k][j] *= inv;
      I[k][j] *= inv;
    }
#pragma unroll
    for (int i = 0; i < M; ++i)
      if (i != k) {
        const double f = A[i][k];
#pragma unroll
        for (int j = 0; j < M; ++j) {
          A[i][j] -= f * A[k][j];
          I[i][j] -= f * I[k][j];
        }
      }
  }
}

// ---------------------------------------------------------------- features
template <int D, int P, int EQ>
__global__ void __launch_bounds__(NT_L) features_kernel(int64_t E, const float* __restrict__ At,
                                                        const double* __restrict__ R, double gscale,
                                                        float* __restrict__ X, uint16_t* __restrict__ Xb,
                                                        float* __restrict__ Dinv) {
  using L = LearnedDims<D, P, EQ>;
  constexpr int N1 = L::N1, NP = L::NP, M = L::M, NIN = L::NIN;
  __shared__ float red[NT_L];
  const int64_t e = blockIdx.x, NN = E * NP;
  float dmax = 0.f, gmax = 0.f;
  for (int a = threadIdx.x; a < NP; a += NT_L) {
    const int self = a % N1;
    const int64_t gn = e * NP + a;
    for (int c = 0; c < M * M; ++c) dmax = fmaxf(dmax, fabsf(At[((int64_t)self * M * M + c) * NN + gn]));
    for (int c = 0; c < M; ++c) gmax = fmaxf(gmax, (float)fabs(gscale * R[(e * M + c) * NP + a]));
  }
  dmax = block_max(dmax, red);
  gmax = block_max(gmax, red);
  const float sig = dmax > 0.f ? dmax : 1.f;
  for (int a = threadIdx.x; a < NP; a += NT_L) {
    const int self = a % N1;
    const int64_t gn = e * NP + a;
    double A[M][M], I[M][M];
    for (int c = 0; c < M; ++c)
      for (int k = 0; k < M; ++k) {
        const float v = At[((int64_t)(self * M + c) * M + k) * NN + gn];
        A[c][k] = v;
        const float f = v / sig;
        const int64_t o = e * NIN + (a * M + c) * M + k;
        if (X) X[o] = f;
        if (Xb) Xb[o] = f32_to_bf16(f);
      }
    for (int c = 0; c < M; ++c) {
      const float f = gmax > 0.f ? (float)(gscale * R[(e * M + c) * NP + a]) / gmax : 0.f;
      const int64_t o = e * NIN + L::NOUT + a * M + c;
      if (X) X[o] = f;
      if (Xb) Xb[o] = f32_to_bf16(f);
    }
    invert<M>(A, I);
    for (int c = 0; c < M; ++c)
      for (int k = 0; k < M; ++k) Dinv[gn * M * M + c * M + k] = (float)I[c][k];
  }
}

// ---------------------------------------------------------------- C = Y D^{-1}
template <int M>
__global__ void cblocks_kernel(int64_t NN, const float* __restrict__ Y, const float* __restrict__ Dinv,
                               float* __restrict__ C, int* __restrict__ bad) {
  const int64_t gn = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gn >= NN) return;
  float y[M][M], di[M][M];
  for (int c = 0; c < M; ++c)
    for (int k = 0; k < M; ++k) {
      y[c][k] = Y[gn * M * M + c * M + k];
      di[c][k] = Dinv[gn * M * M + c * M + k];
    }
  bool finite = true;
  for (int c = 0; c < M; ++c)
    for (int k = 0; k < M; ++k) {
      float s = 0.f;
      for (int q = 0; q < M; ++q) s += y[c][q] * di[q][k];
      finite = finite && isfinite(s);
      C[(int64_t)(c * M + k) * NN + gn] = s;
    }
  if (!finite) atomicOr(bad, 1);
}

// ---------------------------------------------------------------- corrected apply
template <int D, int P, int EQ>
__global__ void __launch_bounds__(256) apply_kernel(int64_t E, const float* __restrict__ At,
                                                    const float* __restrict__ C, const double* __restrict__ r,
                                                    const double* __restrict__ z0, double* __restrict__ z) {
  using L = LearnedDims<D, P, EQ>;
  constexpr int NP = L::NP, M = L::M, NSL = L::NSL;
  const int64_t NN = E * NP;
  const int64_t gn = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gn >= NN) return;
  const int64_t e = gn / NP;
  const int a = (int)(gn % NP);
  double s[M];
#pragma unroll
  for (int c = 0; c < M; ++c) s[c] = r[(e * M + c) * NP + a];
#pragma unroll
  for (int sl = 0; sl < NSL; ++sl) {
    const int b = slot_col<D, P>(a, sl);
    double zb[M];
#pragma unroll
    for (int k = 0; k < M; ++k) zb[k] = z0[(e * M + k) * NP + b];
#pragma unroll
    for (int c = 0; c < M; ++c)
#pragma unroll
      for (int k = 0; k < M; ++k) s[c] -= (double)At[((int64_t)(sl * M + c) * M + k) * NN + gn] * zb[k];
  }
#pragma unroll
  for (int c = 0; c < M; ++c) {
    double v = z0[(e * M + c) * NP + a];
#pragma unroll
    for (int k = 0; k < M; ++k) v += (double)C[(int64_t)(c * M + k) * NN + gn] * s[k];
    z[(e * M + c) * NP + a] = v;
  }
}

// ---------------------------------------------------------------- training samples
// One workgroup per sampled element: copies its features and A~ rows
// ([Np][NSL][m][m]) and forms s, t for K probes (V, Z0 = ILU^{-1} V given).
template <int D, int P, int EQ>
__global__ void __launch_bounds__(NT_L) sample_kernel(int64_t E, const int64_t* __restrict__ elems, int K,
                                                      const float* __restrict__ At, const float* __restrict__ Xf,
                                                      const float* __restrict__ Dinv, const double* __restrict__ V,
                                                      const double* __restrict__ Z0, int64_t ndof,
                                                      float* __restrict__ Xs, float* __restrict__ As,
                                                      float* __restrict__ S, float* __restrict__ T) {
  using L = LearnedDims<D, P, EQ>;
  constexpr int NP = L::NP, M = L::M, NSL = L::NSL, NIN = L::NIN;
  __shared__ double red[NT_L];
  const int64_t i = blockIdx.x, e = elems[i], NN = E * NP;
  for (int j = threadIdx.x; j < NIN; j += NT_L) Xs[i * NIN + j] = Xf[e * NIN + j];
  for (int a = threadIdx.x; a < NP; a += NT_L)
    for (int q = 0; q < NSL * M * M; ++q) As[(i * NP + a) * NSL * M * M + q] = At[(int64_t)q * NN + e * NP + a];
  for (int k = 0; k < K; ++k) {
    const double* v = V + (int64_t)k * ndof;
    const double* z0 = Z0 + (int64_t)k * ndof;
    double part = 0.0;
    for (int a = threadIdx.x; a < NP; a += NT_L)
      for (int c = 0; c < M; ++c) {
        const double x = v[(e * M + c) * NP + a];
        part += x * x;
      }
    const double vn = sqrt(block_sum(part, red));
    const double inv = vn > 0.0 ? 1.0 / vn : 0.0;
    for (int a = threadIdx.x; a < NP; a += NT_L) {
      const int64_t gn = e * NP + a;
      double s[M];
      for (int c = 0; c < M; ++c) s[c] = v[(e * M + c) * NP + a];
      for (int sl = 0; sl < NSL; ++sl) {
        const int b = slot_col<D, P>(a, sl);
        for (int c = 0; c < M; ++c)
          for (int q = 0; q < M; ++q)
            s[c] -= (double)At[((int64_t)(sl * M + c) * M + q) * NN + gn] * z0[(e * M + q) * NP + b];
      }
      for (int c = 0; c < M; ++c) {
        double t = 0.0;
        for (int q = 0; q < M; ++q) t += (double)Dinv[gn * M * M + c * M + q] * s[q];
        S[((i * K + k) * NP + a) * M + c] = (float)(s[c] * inv);
        T[((i * K + k) * NP + a) * M + c] = (float)(t * inv);
      }
    }
  }
}

// ---------------------------------------------------------------- loss and dL/dY
template <int D, int P, int EQ>
__global__ void __launch_bounds__(NT_L) loss_kernel(int K, const float* __restrict__ As, const float* __restrict__ S,
                                                    const float* __restrict__ T, const float* __restrict__ Y,
                                                    float scale, float* __restrict__ dY,
                                                    double* __restrict__ loss_part) {
  using L = LearnedDims<D, P, EQ>;
  constexpr int N1 = L::N1, NP = L::NP, M = L::M, NSL = L::NSL, NOUT = L::NOUT;
  static_assert(NP <= NT_L, "one node per thread");
  extern __shared__ float lds[];
  float* sA = lds;                   // [NP][NSL][M][M]
  float* sc = sA + NP * NSL * M * M;  // [NP][M]
  float* sr = sc + NP * M;            // [NP][M]
  double* red = (double*)(lds + (NP * NSL * M * M + 2 * NP * M + 1) / 2 * 2);  // 8-byte aligned
  const int64_t i = blockIdx.x;
  const int a = threadIdx.x;
  for (int q = threadIdx.x; q < NP * NSL * M * M; q += NT_L) sA[q] = As[i * NP * NSL * M * M + q];
  float y[M][M], g2[M][M];
  if (a < NP)
    for (int c = 0; c < M; ++c)
      for (int k = 0; k < M; ++k) {
        y[c][k] = Y[i * NOUT + (a * M + c) * M + k];
        g2[c][k] = 0.f;
      }
  double lsum = 0.0;
  __syncthreads();
  for (int k = 0; k < K; ++k) {
    float t[M], s[M];
    if (a < NP) {
      for (int c = 0; c < M; ++c) {
        t[c] = T[((i * K + k) * NP + a) * M + c];
        s[c] = S[((i * K + k) * NP + a) * M + c];
      }
      for (int c = 0; c < M; ++c) {
        float v = 0.f;
        for (int q = 0; q < M; ++q) v += y[c][q] * t[q];
        sc[a * M + c] = v;
      }
    }
    __syncthreads();
    if (a < NP) {
      float rho[M];
      for (int c = 0; c < M; ++c) rho[c] = s[c];
      for (int sl = 0; sl < NSL; ++sl) {
        const int b = slot_col<D, P>(a, sl);
        for (int c = 0; c < M; ++c)
          for (int q = 0; q < M; ++q) rho[c] -= sA[((a * NSL + sl) * M + c) * M + q] * sc[b * M + q];
      }
      for (int c = 0; c < M; ++c) {
        sr[a * M + c] = rho[c];
        lsum += (double)rho[c] * rho[c];
      }
    }
    __syncthreads();
    if (a < NP) {
      // g = A~^T rho at node a: rows a2 on the lines through a, slot of column a in row a2
      float g[M];
      for (int c = 0; c < M; ++c) g[c] = 0.f;
      for (int n = 0; n < D; ++n) {
        int l, ta;
        node_line<N1>(a, n, l, ta);
        for (int tp = 0; tp < N1; ++tp) {
          if (n > 0 && tp == ta) continue;
          const int a2 = line_node<D, N1>(n, l, tp);
          const int sl = n == 0 ? ta : N1 + (n - 1) * P + (ta < tp ? ta : ta - 1);
          for (int c = 0; c < M; ++c) {
            const float rc = sr[a2 * M + c];
            for (int q = 0; q < M; ++q) g[q] += sA[((a2 * NSL + sl) * M + c) * M + q] * rc;
          }
        }
      }
      for (int c = 0; c < M; ++c)
        for (int q = 0; q < M; ++q) g2[c][q] += g[c] * t[q];
    }
    __syncthreads();
  }
  if (a < NP)
    for (int c = 0; c < M; ++c)
      for (int q = 0; q < M; ++q) dY[i * NOUT + (a * M + c) * M + q] = -2.f * scale * g2[c][q];
  const double tot = block_sum(lsum, red);
  if (threadIdx.x == 0) loss_part[i] = tot * scale;
}

// ---------------------------------------------------------------- launchers
int learned_supported(const DevCtx& dc) {
  // the loss kernel keeps one sample's A~ rows in LDS and one node per thread
  const int NSL = dc.D * dc.P + 1;
  const size_t bytes = (size_t)(dc.NP * NSL * dc.M * dc.M + 2 * dc.NP * dc.M + 2) * 4 + NT_L * 8;
  return dc.NP <= NT_L && bytes <= 160 * 1024 - 1024;
}

hipError_t launch_learned_features(const DevCtx& dc, const float* At, const double* R, double gscale, float* X,
                                   uint16_t* Xb, float* Dinv) {
  LDG_DISPATCH(dc, {
    hipLaunchKernelGGL((features_kernel<D, P, EQ>), dim3((unsigned)dc.E), dim3(NT_L), 0, dc.stream, dc.E, At, R, gscale,
                       X, Xb, Dinv);
    return hipGetLastError();
  })
}

hipError_t launch_learned_cblocks(const DevCtx& dc, const float* Y, const float* Dinv, float* C, int* bad) {
  const int64_t NN = dc.E * dc.NP;
  const unsigned g = (unsigned)((NN + 255) / 256);
  switch (dc.M) {
    case 1: hipLaunchKernelGGL(cblocks_kernel<1>, dim3(g), dim3(256), 0, dc.stream, NN, Y, Dinv, C, bad); break;
    case 4: hipLaunchKernelGGL(cblocks_kernel<4>, dim3(g), dim3(256), 0, dc.stream, NN, Y, Dinv, C, bad); break;
    case 5: hipLaunchKernelGGL(cblocks_kernel<5>, dim3(g), dim3(256), 0, dc.stream, NN, Y, Dinv, C, bad); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_learned_apply(const DevCtx& dc, const float* At, const float* C, const double* r, const double* z0,
                                double* z) {
  const int64_t NN = dc.E * dc.NP;
  LDG_DISPATCH(dc, {
    hipLaunchKernelGGL((apply_kernel<D, P, EQ>), dim3((unsigned)((NN + 255) / 256)), dim3(256), 0, dc.stream, dc.E, At,
                       C, r, z0, z);
    return hipGetLastError();
  })
}

hipError_t launch_learned_samples(const DevCtx& dc, const int64_t* elems, int64_t n, int K, const float* At,
                                  const float* Xf, const float* Dinv, const double* V, const double* Z0, int64_t ndof,
                                  float* Xs, float* As, float* S, float* T) {
  if (n <= 0) return hipSuccess;
  LDG_DISPATCH(dc, {
    hipLaunchKernelGGL((sample_kernel<D, P, EQ>), dim3((unsigned)n), dim3(NT_L), 0, dc.stream, dc.E, elems, K, At, Xf,
                       Dinv, V, Z0, ndof, Xs, As, S, T);
    return hipGetLastError();
  })
}

hipError_t launch_learned_loss(const DevCtx& dc, int64_t n, int K, const float* As, const float* S, const float* T,
                               const float* Y, float scale, float* dY, double* loss_part) {
  if (n <= 0) return hipSuccess;
  LDG_DISPATCH(dc, {
    using L = LearnedDims<D, P, EQ>;
    if constexpr (L::NP <= NT_L) {
      const size_t bytes = (size_t)(L::NP * L::NSL * L::M * L::M + 2 * L::NP * L::M + 2) * 4 + NT_L * 8;
      if (bytes > 160 * 1024 - 1024) return hipErrorInvalidValue;
      auto k = loss_kernel<D, P, EQ>;
      if (bytes > 65536) {
        hipError_t st = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (st != hipSuccess) return st;
      }
      hipLaunchKernelGGL(k, dim3((unsigned)n), dim3(NT_L), bytes, dc.stream, K, As, S, T, Y, scale, dY, loss_part);
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  })
}

}  // namespace ldg
