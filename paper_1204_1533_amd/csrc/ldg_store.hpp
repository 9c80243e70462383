// Storage precisions of the Jacobian blocks and preconditioner factors.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ldg {

constexpr int PREC_F64 = 0, PREC_F32 = 1, PREC_BF16 = 2;

// float -> bfloat16, round to nearest even.  A NaN stays a (quiet) NaN: adding
// the rounding increment to its bits could carry into the sign or turn it into
// an infinity, so its upper half is kept with the quiet bit set instead.
// Finite values that round past the largest bfloat16 become infinities.
__host__ __device__ inline uint16_t f32_to_bf16(float f) {
  uint32_t b;
  __builtin_memcpy(&b, &f, sizeof(b));
  if ((b & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((b >> 16) | 0x0040u);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}
__host__ __device__ inline float bf16_to_f32(uint16_t h) {
  const uint32_t b = ((uint32_t)h) << 16;
  float f;
  __builtin_memcpy(&f, &b, sizeof(f));
  return f;
}

template <int PREC> struct Store;
template <> struct Store<PREC_F64> {
  typedef double type;
  static __host__ __device__ inline void put(void* p, int64_t i, double v) { ((double*)p)[i] = v; }
  static __host__ __device__ inline double get(const void* p, int64_t i) { return ((const double*)p)[i]; }
};
template <> struct Store<PREC_F32> {
  typedef float type;
  static __host__ __device__ inline void put(void* p, int64_t i, double v) { ((float*)p)[i] = (float)v; }
  static __host__ __device__ inline double get(const void* p, int64_t i) { return ((const float*)p)[i]; }
};
template <> struct Store<PREC_BF16> {
  typedef uint16_t type;
  static __host__ __device__ inline void put(void* p, int64_t i, double v) {
    ((uint16_t*)p)[i] = f32_to_bf16((float)v);
  }
  static __host__ __device__ inline double get(const void* p, int64_t i) {
    return bf16_to_f32(((const uint16_t*)p)[i]);
  }
};

#define LDG_PREC_DISPATCH(prec, ...)                 \
  switch (prec) {                                    \
    case PREC_F64: {                                 \
      constexpr int PR = PREC_F64;                   \
      __VA_ARGS__                                    \
    }                                                \
    case PREC_F32: {                                 \
      constexpr int PR = PREC_F32;                   \
      __VA_ARGS__                                    \
    }                                                \
    case PREC_BF16: {                                \
      constexpr int PR = PREC_BF16;                  \
      __VA_ARGS__                                    \
    }                                                \
    default:                                         \
      return hipErrorInvalidValue;                   \
  }

}  // namespace ldg
