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
  MeshParams mp;
  hipStream_t stream;
};

// Block size of the element kernels.
constexpr int NT_ELEM = 256;

// Elements per workgroup for the residual-type kernels: small 2-D elements
// are packed so that one workgroup still has several hundred work items.
__host__ __device__ constexpr int elems_per_block(int NP, int M) {
  int e = 512 / (NP * M);
  return e < 1 ? 1 : (e > 16 ? 16 : e);
}

hipError_t launch_gradient(const DevCtx& c, const double* U, double* Q, bool homogeneous);
hipError_t launch_residual(const DevCtx& c, const double* U, const double* Q, double* R);
// Rt = dR/dU . V (exact forward-mode tangent) with Qt = D_hom(V)
hipError_t launch_residual_tangent(const DevCtx& c, const double* U, const double* V, const double* Q,
                                   const double* Qt, double* Rt);

// Jacobian blocks; prec: 0 f64, 1 f32, 2 bf16.  Layout [slot][row comp][col comp][E*Np].
hipError_t launch_jacobian(const DevCtx& c, const double* U, const double* Q, void* K11, void* K12, int prec);

// y = alpha x - gamma (K11 x + K12 w), w = D_hom(x) given.
hipError_t launch_jacvec(const DevCtx& c, const void* K11, const void* K12, int prec, double alpha, double gamma,
                         const double* x, const double* w, double* y);

// Preconditioner A~ (line pattern) formed from the stored K11/K12 and the
// K21 weights, then factorised by block ILU(0); factors [slot][c][c'][E*Np].
hipError_t launch_precond_factor(const DevCtx& c, const void* K11, const void* K12, int prec, double alpha,
                                 double gamma, void* F, int fprec);
hipError_t launch_precond_apply(const DevCtx& c, const void* F, int fprec, const double* r, double* z);

// Conversions of the internal layouts to the FP64 exchange layouts of ldg.h.
hipError_t launch_export_blocks(const DevCtx& c, const void* K, int prec, int nslot, int ncol, double* out);

// Krylov helpers (FP64)
hipError_t launch_multidot(const double* V, int64_t ldv, int k, const double* w, int64_t n, double* partial,
                           int nblocks, hipStream_t s);
hipError_t launch_multidot_finish(const double* partial, int nblocks, int k, double* out, hipStream_t s);
hipError_t launch_update(double* w, const double* V, int64_t ldv, int k, const double* h, int64_t n,
                         hipStream_t s);  // w -= V h (h on device)
hipError_t launch_axpby(double* y, double a, const double* x, double b, int64_t n, hipStream_t s);  // y = a x + b y
hipError_t launch_lincomb(double* y, const double* V, int64_t ldv, int k, const double* coef, int64_t n,
                          hipStream_t s);  // y += V coef
hipError_t launch_rk4_stage(double* Ustage, const double* U, const double* K, double a, double* Acc, double b,
                            int64_t n, hipStream_t s);

}  // namespace ldg
