// bfloat16 rounding helpers (round to nearest, ties to even) used by the
// table kernel (from float64) and the DFT epilogue (from float32).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace sht {

// Round a float64 to 8 significant bits in float64 arithmetic (ties to even),
// then take the bf16 bit pattern of that exactly representable value.  A
// single rounding: no float64 -> float32 -> bf16 double rounding.
__device__ __host__ inline uint16_t bf16_rn_from_double(double v) {
  uint64_t b;
  __builtin_memcpy(&b, &v, 8);
  const uint64_t lsb = (b >> 45) & 1u;
  b += 0x00000FFFFFFFFFFFull + lsb;  // 2^44 - 1 + lsb
  b &= ~((1ull << 45) - 1ull);
  double r;
  __builtin_memcpy(&r, &b, 8);
  const float f = static_cast<float>(r);
  uint32_t u;
  __builtin_memcpy(&u, &f, 4);
  return static_cast<uint16_t>(u >> 16);
}

__device__ __host__ inline double bf16_bits_to_double(uint16_t h) {
  const uint32_t u = static_cast<uint32_t>(h) << 16;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return static_cast<double>(f);
}

__device__ __host__ inline uint16_t bf16_rn_from_float(float v) {
  uint32_t u;
  __builtin_memcpy(&u, &v, 4);
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7FFFu + lsb;
  return static_cast<uint16_t>(u >> 16);
}

__device__ __host__ inline float bf16_bits_to_float(uint16_t h) {
  const uint32_t u = static_cast<uint32_t>(h) << 16;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return f;
}

}  // namespace sht
