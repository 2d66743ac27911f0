// Layout and BF16 conversions of the cost-model MLP 4 -> 64 -> 64 -> 1
// (ReLU), shared by its training kernels and the threshold tuner.
//
// Parameter vector (kMlpParams BF16 values):
//   W1 [64][4]   at 0      b1 [64] at 256
//   W2 [64][64]  at 320    b2 [64] at 4416   (row i = hidden unit i)
//   w3 [64]      at 4480   b3      at 4544
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sj {

constexpr int kH = 64, kF = 4;
constexpr int kOW1 = 0, kOB1 = 256, kOW2 = 320, kOB2 = 4416, kOW3 = 4480, kOB3 = 4544;
constexpr int kMlpParams = 4545;

__device__ __forceinline__ float bf2f(uint16_t u) { return __uint_as_float((uint32_t)u << 16); }

// Round to nearest, ties to even; NaN stays NaN.
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

}  // namespace sj
