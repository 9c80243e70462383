// Host-visible launchers of the line-DG kernels and the shared device context.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ldg_device.hpp"

namespace ldg {

struct DevCtx {
  int D, P, EQ, M, N1, NP, NL, NG;
  int64_t E;
  LineOps ops;
  LevelOrder lev;
  MeshParams mp;
  hipStream_t stream;
};

// Block size of the element kernels.
constexpr int NT_ELEM = 256;
constexpr size_t LDS_PER_CU = 160 * 1024;  // bytes of LDS one workgroup may use on gfx950

// Geometry record of an element: [Ag: D][NLG][D] Gauss-point metric a_n,
// [Nf: D][NLS][D] outward non-unit normals of the line ends, [Js: NP] -1/J.
template <int D, int P>
struct GeoShape {
  static constexpr int N1 = P + 1, NG = n_gauss(P), NP = ipow(N1, D), NL = ipow(N1, D - 1);
  static constexpr int oAg = 0;
  static constexpr int oNf = oAg + D * NL * NG * D;
  static constexpr int oJs = oNf + D * NL * 2 * D;
  static constexpr int REC = oJs + NP;
};

// Elements per workgroup for the residual-type kernels: small 2-D elements
// are packed so that one workgroup still has several hundred work items.
__host__ __device__ constexpr int elems_per_block(int NP, int M) {
  int e = 512 / (NP * M);
  return e < 1 ? 1 : (e > 16 ? 16 : e);
}

// Layout of the BILU(0) factors read by the preconditioner apply.  Per
// element the NR = M Np factor rows r = M rank[a] + c (component c of node a,
// nodes in level order, LevelOrder) hold
// the NJ = (D p + 1) M entries j = slot M + c' of their line-slot blocks
// (slot order of the line pattern, the diagonal slot holding the inverse of
// the U diagonal block), padded with zeros to NJP = 4 ceil(NJ / 4).  Stored
// as [E][NJP / 4][NR][4]: a row's entries come in chunks of 4, and the same
// chunk of consecutive rows is contiguous, so that one load per chunk by
// consecutive rows reads one contiguous run.
// Order of a factor row's blocks in the apply layout: the blocks left of the
// diagonal (direction 0 positions 0 .. c_0 - 1, then direction 1, ..., each
// ascending), the diagonal block, then the blocks right of it (same order).
// A row of level L = c_0 + .. + c_{D-1} has exactly L blocks on the left, so
// every row of a level has its lower part in positions 0 .. L-1.
// row_slot_at: line slot (slot_col numbering) at position pos of node a's row;
// row_pos_of: the inverse.
__host__ __device__ inline int row_slot_at(int D, int P, int a, int pos) {
  const int N1 = P + 1;
  int cd[3] = {0, 0, 0}, L = 0;
  for (int d = 0, r = a; d < D; ++d, r /= N1) {
    cd[d] = r % N1;
    L += cd[d];
  }
  if (pos == L) return cd[0];
  if (pos < L) {
    for (int n = 0; n < D; ++n) {
      if (pos < cd[n]) return n == 0 ? pos : N1 + (n - 1) * P + pos;
      pos -= cd[n];
    }
  }
  int u = pos - L - 1;
  for (int n = 0; n < D; ++n) {
    const int cnt = P - cd[n];
    if (u < cnt) {
      const int t = cd[n] + 1 + u;
      return n == 0 ? t : N1 + (n - 1) * P + (t - 1);
    }
    u -= cnt;
  }
  return -1;
}
__host__ __device__ inline int row_pos_of(int D, int P, int a, int slot) {
  const int N1 = P + 1;
  int cd[3] = {0, 0, 0}, L = 0;
  for (int d = 0, r = a; d < D; ++d, r /= N1) {
    cd[d] = r % N1;
    L += cd[d];
  }
  int n, t;
  if (slot < N1) {
    n = 0;
    t = slot;
  } else {
    n = 1 + (slot - N1) / P;
    const int r = (slot - N1) % P;
    t = r < cd[n] ? r : r + 1;
  }
  if (t == cd[n]) return L;
  int before = 0;
  if (t < cd[n]) {
    for (int m = 0; m < n; ++m) before += cd[m];
    return before + t;
  }
  for (int m = 0; m < n; ++m) before += P - cd[m];
  return L + 1 + before + (t - cd[n] - 1);
}

__host__ __device__ constexpr int64_t fac_index(int64_t e, int r, int j, int NR, int NJP) {
  return ((e * (NJP / 4) + (j >> 2)) * NR + r) * 4 + (j & 3);
}
template <int D, int P, int EQ>
struct FacShape {
  static constexpr int NP = ipow(P + 1, D), M = Eq<D, EQ>::M, NSL = D * P + 1;
  static constexpr int NR = NP * M, NJ = NSL * M, NJP = (NJ + 3) / 4 * 4;
  static constexpr int EPB = NR >= 512 ? 1 : 512 / NR;  // elements per workgroup of the apply
  static constexpr int NT = (EPB * NR + 63) / 64 * 64;
};

// Q = D(U); with Qc (C22 != 0, the coupled system) the trace takes the jump of
// the normal viscous flux of the gradient field Qc: Q = G(U, Qc)
hipError_t launch_gradient(const DevCtx& c, const double* U, double* Q, bool homogeneous,
                           const double* Qc = nullptr);
hipError_t launch_residual(const DevCtx& c, const double* U, const double* Q, double* R);
// Rt = dR/dU . V (exact forward-mode tangent) with Qt = D_hom(V)
hipError_t launch_residual_tangent(const DevCtx& c, const double* U, const double* V, const double* Q,
                                   const double* Qt, double* Rt);

// K21 = dD/dU as stored FP64 weights [slot][d][E Np] (D p + 1 + D slots),
// computed once from the geometry; w = K21 x with them.
hipError_t launch_k21_weights(const DevCtx& c, double* Wt);
hipError_t launch_k21_apply(const DevCtx& c, const double* Wt, const double* x, double* w);
// FP32 copy of the weights, and the product with it (beside stored FP32 / BF16
// blocks, whose rounding is far larger)
hipError_t launch_k21_weights_f32(const DevCtx& c, const double* Wt, float* Wf);
hipError_t launch_k21_apply_f32(const DevCtx& c, const float* Wt, const double* x, double* w);

// Jacobian blocks; prec: 0 f64, 1 f32, 2 bf16.  Layout [slot][row comp][col comp][E*Np].
// Jacobian blocks in three launches: geometry record per element (once per
// context), point flux Jacobians into a workspace, contraction into the blocks
size_t jacobian_geometry_doubles(const DevCtx& c);
size_t jacobian_workspace_doubles(const DevCtx& c);
hipError_t launch_jacobian_geometry(const DevCtx& c, double* geo);
hipError_t launch_jacobian(const DevCtx& c, const double* U, const double* Q, void* K11, void* K12, int prec,
                           const double* geo, double* work);

// y = alpha x - gamma (K11 x + K12 w), w = D_hom(x) given.
hipError_t launch_jacvec(const DevCtx& c, const void* K11, const void* K12, int prec, double alpha, double gamma,
                         const double* x, const double* w, double* y);

// Preconditioner A~ (line pattern) formed from the stored K11/K12 and the
// stored K21 weights K21w (launch_k21_weights; unused without viscous terms),
// then factorised by block ILU(0): the factors end in Fem in the apply layout
// above (precision fprec).
hipError_t launch_precond_factor(const DevCtx& c, const void* K11, const void* K12, const double* K21w, int prec,
                                 double alpha, double gamma, void* Fwork, int fprec, void* Fem, float* At_copy,
                                 double* dense = nullptr);
// exact element-block LU of A~: element-major A~ (FP64 or FP32) -> dense
// [E][NR][NR] L\U (FP64, unit lower L), NR = Np m <= 768; and its apply
hipError_t launch_blocklu_factor(const DevCtx& c, const void* em, int emprec, double* dense);
hipError_t launch_blocklu_apply(const DevCtx& c, const double* dense, const double* r, double* z);
hipError_t launch_factors_to_f64(const DevCtx& c, const void* Fem, int fprec, double* out);
hipError_t launch_precond_apply(const DevCtx& c, const void* Fem, int fprec, const double* r, double* z);

// Conversions of the internal layouts to the FP64 exchange layouts of ldg.h.
hipError_t launch_export_blocks(const DevCtx& c, const void* K, int prec, int nslot, int ncol, double* out);

// Krylov helpers (FP64)
hipError_t launch_multidot(const double* V, int64_t ldv, int k, const double* w, int64_t n, double* partial,
                           int nblocks, hipStream_t s);
hipError_t launch_multidot_finish(const double* partial, int nblocks, int k, double* out, hipStream_t s);
hipError_t launch_update(double* w, const double* V, int64_t ldv, int k, const double* h, int64_t n,
                         hipStream_t s, double scale = 1.0);  // w = (w - V h) scale (h on device)
hipError_t launch_axpby(double* y, double a, const double* x, double b, int64_t n, hipStream_t s);  // y = a x + b y
hipError_t launch_lincomb(double* y, const double* V, int64_t ldv, int k, const double* coef, int64_t n,
                          hipStream_t s);  // y += V coef
hipError_t launch_copy(double* y, const double* x, int64_t n, hipStream_t s);  // y = x (a kernel, not a copy node)
hipError_t launch_rk4_stage(double* Ustage, const double* U, const double* K, double a, double* Acc, double b,
                            int64_t n, hipStream_t s);

// Learned correction (k_learned.hip) and the network kernels (k_mlp.hip).
int learned_supported(const DevCtx& c);
hipError_t launch_learned_features(const DevCtx& c, const float* At, const double* R, double gscale, float* X,
                                   uint16_t* Xb, float* Dinv);
hipError_t launch_learned_cblocks(const DevCtx& c, const float* Y, const float* Dinv, float* C, int* bad);
hipError_t launch_learned_apply(const DevCtx& c, const float* At, const float* C, const double* r, const double* z0,
                                double* z);
hipError_t launch_learned_samples(const DevCtx& c, const int64_t* elems, int64_t n, int K, const float* At,
                                  const float* Xf, const float* Dinv, const double* V, const double* Z0, int64_t ndof,
                                  float* Xs, float* As, float* S, float* T);
hipError_t launch_learned_loss(const DevCtx& c, int64_t n, int K, const float* As, const float* S, const float* T,
                               const float* Y, float scale, float* dY, double* loss_part);
hipError_t launch_gemm_bf16(int M, int N, int K, const uint16_t* A, int64_t sam, int64_t sak, const uint16_t* B,
                            int64_t sbk, int64_t sbn, float* C, int64_t ldc, uint16_t* Cb, const float* bias,
                            int epilogue, float beta, hipStream_t s);
hipError_t launch_gemm_f32(int M, int N, int K, const float* A, int64_t sam, int64_t sak, const float* B, int64_t sbk,
                           int64_t sbn, float* C, int64_t ldc, uint16_t* Cb, const float* bias, int epilogue,
                           float beta, hipStream_t s);
hipError_t launch_tanh_backward(const float* dH, const float* H, float* dA, uint16_t* dAb, int64_t n, hipStream_t s);
hipError_t launch_colsum(const float* X, int M, int N, float* out, hipStream_t s);
hipError_t launch_adam(float* w, uint16_t* wb, const float* g, float* m1, float* m2, int64_t n, float lr, float b1,
                       float b2, float eps, int step, hipStream_t s);
hipError_t launch_to_bf16(const float* x, uint16_t* y, int64_t n, hipStream_t s);

}  // namespace ldg
