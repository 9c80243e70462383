// ldg_jacvec_noalloc: the split product of ldg_jacvec without any device
// allocation.  Its one scratch buffer, w = K21 x (the homogeneous LDG gradient
// of x, [E][m][D][Np] doubles), lives in a file-scope device array of fixed
// size instead of context memory that ldg_jacvec allocates on first use.
//
// Host code must not pass the array's name to a kernel: in host code it names
// a host-side stand-in, not device memory.  Its device address is looked up
// once per device with hipGetSymbolAddress (the first call on that device,
// with the device current) and only that address is used afterwards.  Every
// call on one device shares the array: calls that overlap on a device (other
// streams, other threads) race on it.  Each call writes all of w before the
// product reads it, so nothing needs clearing between calls.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/ldg.h"
#include "ldg_ctx.hpp"

static __device__ __align__(256) double scratch[LDG_NOALLOC_SCRATCH_DOUBLES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (looked up on first use).
hipError_t scratch_on_current_device(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" ldg_status ldg_jacvec_noalloc(ldg_ctx c, const double* x, double* y, int32_t exact) {
  if (!c) return LDG_E_INVALID;
  if (!x || !y) return fail(c, LDG_E_INVALID, "null pointer");
  if ((const void*)x == (const void*)y) return fail(c, LDG_E_INVALID, "x and y alias");
  if (!c->assembled) return fail(c, LDG_E_NOT_ASSEMBLED, "call ldg_jacobian_assemble first");
  if (c->nq > (int64_t)LDG_NOALLOC_SCRATCH_DOUBLES)
    return fail(c, LDG_E_UNSUPPORTED,
                "ldg_jacvec_noalloc: K21 x needs " + std::to_string(c->nq) + " doubles, the static scratch holds " +
                    std::to_string((long long)LDG_NOALLOC_SCRATCH_DOUBLES) + " (use ldg_jacvec)");
  double* w = nullptr;
  hipError_t e = scratch_on_current_device(&w);
  if (e != hipSuccess)
    return fail(c, LDG_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  return apply_op_with(c, x, y, exact != 0, w);
}
