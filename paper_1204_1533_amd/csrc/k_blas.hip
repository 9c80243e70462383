// FP64 vector kernels for the Krylov solver and the explicit Runge-Kutta loop.
//
// multidot : h_j = <V_j, w> for j < k (block partial sums, then a second pass);
//            one block row per tile of 8 basis vectors, so w is read k/8 times.
// update   : w -= sum_j h_j V_j   (classical Gram-Schmidt projection)
// lincomb  : y += sum_j c_j V_j   (GMRES solution update)
#include "ldg_kernels.hpp"

namespace ldg {

constexpr int NT_BLAS = 256;
constexpr int DOT_TILE = 8;

__global__ void __launch_bounds__(NT_BLAS) multidot_kernel(const double* __restrict__ V, int64_t ldv, int k,
                                                          const double* __restrict__ w, int64_t n,
                                                          double* __restrict__ partial) {
  // grid: x over row blocks, y over tiles of DOT_TILE basis vectors
  __shared__ double red[NT_BLAS / 64][DOT_TILE];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int j0 = blockIdx.y * DOT_TILE;
  const int nt = min(DOT_TILE, k - j0);
  double acc[DOT_TILE];
#pragma unroll
  for (int t = 0; t < DOT_TILE; ++t) acc[t] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * NT_BLAS + tid; i < n; i += (int64_t)gridDim.x * NT_BLAS) {
    const double wi = w[i];
#pragma unroll
    for (int t = 0; t < DOT_TILE; ++t)
      if (t < nt) acc[t] += V[(int64_t)(j0 + t) * ldv + i] * wi;
  }
#pragma unroll
  for (int t = 0; t < DOT_TILE; ++t) {
    double v = acc[t];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) red[wid][t] = v;
  }
  __syncthreads();
  if (tid < nt) {
    double s = 0.0;
    for (int q = 0; q < NT_BLAS / 64; ++q) s += red[q][tid];
    partial[(int64_t)blockIdx.x * k + j0 + tid] = s;
  }
}

__global__ void multidot_finish_kernel(const double* __restrict__ partial, int nblocks, int k,
                                       double* __restrict__ out) {
  const int j = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) s += partial[(int64_t)b * k + j];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < (int)(blockDim.x / 64); ++q) t += red[q];
    out[j] = t;
  }
}

__global__ void __launch_bounds__(NT_BLAS) update_kernel(double* __restrict__ w, const double* __restrict__ V,
                                                        int64_t ldv, int k, const double* __restrict__ h,
                                                        int64_t n, double sign, double scale) {
  __shared__ double sh[128];
  for (int j = threadIdx.x; j < k; j += NT_BLAS) sh[j] = h[j];
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * NT_BLAS + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT_BLAS) {
    double acc = 0.0;
    for (int j = 0; j < k; ++j) acc += V[(int64_t)j * ldv + i] * sh[j];
    w[i] = (w[i] + sign * acc) * scale;
  }
}

__global__ void axpby_kernel(double* __restrict__ y, double a, const double* __restrict__ x, double b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i] + b * y[i];
}

__global__ void rk4_stage_kernel(double* __restrict__ Us, const double* __restrict__ U, const double* __restrict__ K,
                                 double a, double* __restrict__ Acc, double b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double k = K[i];
    if (Us) Us[i] = U[i] + a * k;
    Acc[i] += b * k;
  }
}

__global__ void copy_kernel(double* __restrict__ y, const double* __restrict__ x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = x[i];
}

static unsigned grid_for(int64_t n, int nt) {
  int64_t g = (n + nt - 1) / nt;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (unsigned)g;
}

hipError_t launch_multidot(const double* V, int64_t ldv, int k, const double* w, int64_t n, double* partial,
                           int nblocks, hipStream_t s) {
  if (k > 128) return hipErrorInvalidValue;
  if (k < 1) return hipSuccess;
  hipLaunchKernelGGL(multidot_kernel, dim3(nblocks, (k + DOT_TILE - 1) / DOT_TILE), dim3(NT_BLAS), 0, s, V, ldv, k, w,
                     n, partial);
  return hipGetLastError();
}

hipError_t launch_multidot_finish(const double* partial, int nblocks, int k, double* out, hipStream_t s) {
  hipLaunchKernelGGL(multidot_finish_kernel, dim3(k), dim3(256), 0, s, partial, nblocks, k, out);
  return hipGetLastError();
}

hipError_t launch_update(double* w, const double* V, int64_t ldv, int k, const double* h, int64_t n, hipStream_t s,
                         double scale) {
  if (k > 128) return hipErrorInvalidValue;
  hipLaunchKernelGGL(update_kernel, dim3(grid_for(n, NT_BLAS)), dim3(NT_BLAS), 0, s, w, V, ldv, k, h, n, -1.0, scale);
  return hipGetLastError();
}

hipError_t launch_lincomb(double* y, const double* V, int64_t ldv, int k, const double* coef, int64_t n,
                          hipStream_t s) {
  if (k > 128) return hipErrorInvalidValue;
  hipLaunchKernelGGL(update_kernel, dim3(grid_for(n, NT_BLAS)), dim3(NT_BLAS), 0, s, y, V, ldv, k, coef, n, 1.0, 1.0);
  return hipGetLastError();
}

hipError_t launch_axpby(double* y, double a, const double* x, double b, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(axpby_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, y, a, x, b, n);
  return hipGetLastError();
}

hipError_t launch_rk4_stage(double* Us, const double* U, const double* K, double a, double* Acc, double b, int64_t n,
                            hipStream_t s) {
  hipLaunchKernelGGL(rk4_stage_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, Us, U, K, a, Acc, b, n);
  return hipGetLastError();
}

hipError_t launch_copy(double* y, const double* x, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(copy_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, y, x, n);
  return hipGetLastError();
}

}  // namespace ldg
