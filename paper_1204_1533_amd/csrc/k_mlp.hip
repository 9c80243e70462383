// Dense kernels of the per-element correction network: an MFMA GEMM with
// FP32 accumulation and a fused bias / tanh epilogue, the tanh backward, bias
// gradients (column sums), Adam, and FP32 -> BF16 conversion.
//
// GEMM: C[m][n] = sum_k A(m, k) B(k, n), A(m, k) = A[m sam + k sak],
// B(k, n) = B[k sbk + n sbn].  Generic strides let one kernel serve the
// forward products X W, the input gradients dY W^T and the weight gradients
// X^T dY.  Workgroup tile 64 x 64 with a 32-deep K step staged in LDS; four
// wavefronts each own a 32 x 32 sub-tile made of 2 x 2 16 x 16 MFMA tiles:
//   BF16 operands: v_mfma_f32_16x16x32_bf16 (lane holds row lane%16,
//                  k = 8 (lane/16) .. +7; the whole 32-deep step in one
//                  instruction),
//   FP32 operands: v_mfma_f32_16x16x4f32      (lane holds row lane%16,
//                  k = lane/16);
// the 16 x 16 FP32 result puts rows 4 (lane/16) + t, t = 0..3, of column
// lane%16 in each lane.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ldg_kernels.hpp"
#include "ldg_store.hpp"

namespace ldg {

typedef short short8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float float4_t __attribute__((ext_vector_type(4)));

constexpr int GT_M = 64, GT_N = 64, GT_K = 32;

template <class T>
__device__ __forceinline__ T zero_of() {
  return T(0);
}

// Stage a GT_R x GT_K tile of a strided operand into LDS as tile[r][k].  The
// loop order follows the unit stride so that neighbouring lanes read
// neighbouring addresses.
template <class T, int GT_R>
__device__ __forceinline__ void stage(T (*tile)[GT_K + 2], const T* __restrict__ X, int64_t sr, int64_t sk, int r0,
                                      int k0, int R, int K, int tid) {
  if (sk == 1 || sr != 1) {
    for (int i = tid; i < GT_R * GT_K; i += 256) {
      const int r = i / GT_K, kk = i % GT_K;
      const int gr = r0 + r, gk = k0 + kk;
      tile[r][kk] = (gr < R && gk < K) ? X[gr * sr + gk * sk] : zero_of<T>();
    }
  } else {
    for (int i = tid; i < GT_R * GT_K; i += 256) {
      const int r = i % GT_R, kk = i / GT_R;
      const int gr = r0 + r, gk = k0 + kk;
      tile[r][kk] = (gr < R && gk < K) ? X[gr * sr + gk * sk] : zero_of<T>();
    }
  }
}

template <class T>
__device__ __forceinline__ void mma_tile(const T (*sA)[GT_K + 2], const T (*sB)[GT_K + 2], int wm, int wn, int lane,
                                         float4_t (&acc)[2][2]);

template <>
__device__ __forceinline__ void mma_tile<uint16_t>(const uint16_t (*sA)[GT_K + 2], const uint16_t (*sB)[GT_K + 2],
                                                   int wm, int wn, int lane, float4_t (&acc)[2][2]) {
  static_assert(GT_K == 32, "one 16x16x32 step per staged K tile");
  const int kq = 8 * (lane >> 4);
  bf16x8_t a[2], b[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const uint16_t* p = sA[wm + 16 * i + (lane & 15)] + kq;
    short8_t v;
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = (short)p[q];
    a[i] = __builtin_bit_cast(bf16x8_t, v);
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const uint16_t* p = sB[wn + 16 * j + (lane & 15)] + kq;
    short8_t v;
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = (short)p[q];
    b[j] = __builtin_bit_cast(bf16x8_t, v);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
}

template <>
__device__ __forceinline__ void mma_tile<float>(const float (*sA)[GT_K + 2], const float (*sB)[GT_K + 2], int wm,
                                                int wn, int lane, float4_t (&acc)[2][2]) {
#pragma unroll
  for (int ks = 0; ks < GT_K; ks += 4) {
    const int kq = ks + (lane >> 4);
    float a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) a[i] = sA[wm + 16 * i + (lane & 15)][kq];
#pragma unroll
    for (int j = 0; j < 2; ++j) b[j] = sB[wn + 16 * j + (lane & 15)][kq];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
  }
}

// epilogue: 0 none, 1 + bias, 2 tanh(. + bias); beta != 0 adds beta C_old.
template <class T>
__global__ void __launch_bounds__(256) mfma_gemm_kernel(int M, int N, int K, const T* __restrict__ A, int64_t sam,
                                                        int64_t sak, const T* __restrict__ B, int64_t sbk, int64_t sbn,
                                                        float* __restrict__ C, int64_t ldc, uint16_t* __restrict__ Cb,
                                                        const float* __restrict__ bias, int epilogue, float beta) {
  __shared__ T sA[GT_M][GT_K + 2];
  __shared__ T sB[GT_N][GT_K + 2];  // B stored transposed: sB[n][k]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * GT_M, n0 = blockIdx.x * GT_N;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  float4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = float4_t{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += GT_K) {
    stage<T, GT_M>(sA, A, sam, sak, m0, k0, M, K, tid);
    stage<T, GT_N>(sB, B, sbn, sbk, n0, k0, N, K, tid);
    __syncthreads();
    mma_tile<T>(sA, sB, wm, wn, lane, acc);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int gm = m0 + wm + 16 * i + 4 * (lane >> 4) + t;
        const int gn = n0 + wn + 16 * j + (lane & 15);
        if (gm < M && gn < N) {
          float v = acc[i][j][t];
          if (epilogue >= 1) v += bias[gn];
          if (epilogue == 2) v = tanhf(v);
          const int64_t o = (int64_t)gm * ldc + gn;
          if (beta != 0.f) v += beta * C[o];
          C[o] = v;
          if (Cb) Cb[o] = f32_to_bf16(v);
        }
      }
}

template <class T>
static hipError_t gemm_launch(int M, int N, int K, const T* A, int64_t sam, int64_t sak, const T* B, int64_t sbk,
                              int64_t sbn, float* C, int64_t ldc, uint16_t* Cb, const float* bias, int epilogue,
                              float beta, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  dim3 grid((N + GT_N - 1) / GT_N, (M + GT_M - 1) / GT_M);
  hipLaunchKernelGGL(mfma_gemm_kernel<T>, grid, dim3(256), 0, s, M, N, K, A, sam, sak, B, sbk, sbn, C, ldc, Cb, bias,
                     epilogue, beta);
  return hipGetLastError();
}

hipError_t launch_gemm_bf16(int M, int N, int K, const uint16_t* A, int64_t sam, int64_t sak, const uint16_t* B,
                            int64_t sbk, int64_t sbn, float* C, int64_t ldc, uint16_t* Cb, const float* bias,
                            int epilogue, float beta, hipStream_t s) {
  return gemm_launch<uint16_t>(M, N, K, A, sam, sak, B, sbk, sbn, C, ldc, Cb, bias, epilogue, beta, s);
}
hipError_t launch_gemm_f32(int M, int N, int K, const float* A, int64_t sam, int64_t sak, const float* B, int64_t sbk,
                           int64_t sbn, float* C, int64_t ldc, uint16_t* Cb, const float* bias, int epilogue,
                           float beta, hipStream_t s) {
  return gemm_launch<float>(M, N, K, A, sam, sak, B, sbk, sbn, C, ldc, Cb, bias, epilogue, beta, s);
}

// dA = dH (1 - H^2) (tanh backward), also written as BF16 when dAb is given
__global__ void tanh_backward_kernel(const float* __restrict__ dH, const float* __restrict__ H, float* __restrict__ dA,
                                     uint16_t* __restrict__ dAb, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float h = H[i];
    const float v = dH[i] * (1.f - h * h);
    dA[i] = v;
    if (dAb) dAb[i] = f32_to_bf16(v);
  }
}

// out[j] = sum_i X[i][j]: 64 columns per workgroup, four row groups reduced in LDS
__global__ void __launch_bounds__(256) colsum_kernel(const float* __restrict__ X, int M, int N,
                                                     float* __restrict__ out) {
  __shared__ float part[4][64];
  const int j = blockIdx.x * 64 + (threadIdx.x & 63), g = threadIdx.x >> 6;
  float s = 0.f;
  if (j < N)
    for (int i = g; i < M; i += 4) s += X[(int64_t)i * N + j];
  part[g][threadIdx.x & 63] = s;
  __syncthreads();
  if (g == 0 && j < N) out[j] = part[0][threadIdx.x] + part[1][threadIdx.x] + part[2][threadIdx.x] + part[3][threadIdx.x];
}

// Adam with bias correction on FP32 master weights; refreshes the BF16 copy.
__global__ void adam_kernel(float* __restrict__ w, uint16_t* __restrict__ wb, const float* __restrict__ g,
                            float* __restrict__ m1, float* __restrict__ m2, int64_t n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.f - b1) * gi;
    const float b = b2 * m2[i] + (1.f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = b;
    const float v = w[i] - lr * (a / c1) / (sqrtf(b / c2) + eps);
    w[i] = v;
    if (wb) wb[i] = f32_to_bf16(v);
  }
}

__global__ void to_bf16_kernel(const float* __restrict__ x, uint16_t* __restrict__ y, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = f32_to_bf16(x[i]);
}

static unsigned grid1(int64_t n) {
  int64_t g = (n + 255) / 256;
  return (unsigned)(g > 65536 ? 65536 : (g < 1 ? 1 : g));
}

hipError_t launch_tanh_backward(const float* dH, const float* H, float* dA, uint16_t* dAb, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(tanh_backward_kernel, dim3(grid1(n)), dim3(256), 0, s, dH, H, dA, dAb, n);
  return hipGetLastError();
}
hipError_t launch_colsum(const float* X, int M, int N, float* out, hipStream_t s) {
  hipLaunchKernelGGL(colsum_kernel, dim3((N + 63) / 64), dim3(256), 0, s, X, M, N, out);
  return hipGetLastError();
}
hipError_t launch_adam(float* w, uint16_t* wb, const float* g, float* m1, float* m2, int64_t n, float lr, float b1,
                       float b2, float eps, int step, hipStream_t s) {
  const float c1 = (float)(1.0 - std::pow((double)b1, step)), c2 = (float)(1.0 - std::pow((double)b2, step));
  hipLaunchKernelGGL(adam_kernel, dim3(grid1(n)), dim3(256), 0, s, w, wb, g, m1, m2, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}
hipError_t launch_to_bf16(const float* x, uint16_t* y, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(to_bf16_kernel, dim3(grid1(n)), dim3(256), 0, s, x, y, n);
  return hipGetLastError();
}

}  // namespace ldg
