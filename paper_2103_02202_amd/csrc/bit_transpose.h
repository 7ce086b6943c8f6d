// 64 x 64 bit-block transpose inside one wave (device code).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace stimgpu {

__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, int m) {
  const uint32_t lo = __shfl_xor((uint32_t)v, m, 64), hi = __shfl_xor((uint32_t)(v >> 32), m, 64);
  return ((uint64_t)hi << 32) | lo;
}

// Transposes a 64 x 64 bit block held one row per lane: on entry lane l holds
// row l (bit s = column s); on exit lane s holds column s (bit l = row l).
// Recursive exchange of off-diagonal blocks of halving size.
__device__ __forceinline__ uint64_t bit_transpose64(uint64_t x, uint32_t lane) {
  uint64_t m = 0x00000000FFFFFFFFull;
#pragma unroll
  for (int j = 32; j != 0; j >>= 1) {
    const uint64_t other = shfl_xor64(x, j);
    if ((lane & j) == 0) {
      const uint64_t t = ((x >> j) ^ other) & m;
      x ^= t << j;
    } else {
      const uint64_t t = ((other >> j) ^ x) & m;
      x ^= t;
    }
    m ^= m << (j >> 1);
  }
  return x;
}

}  // namespace stimgpu
