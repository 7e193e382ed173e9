// philox.h -- Philox4x64-10 counter-based generator (device side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rr {

// Philox4x64-10, Salmon et al., "Parallel random numbers: as easy as 1, 2, 3"
// (SC'11).
__device__ __forceinline__ void philox4x64_10(uint64_t k0, uint64_t k1, uint64_t x0, uint64_t x1,
                                              uint64_t x2, uint64_t x3, uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    uint64_t hi0 = __umul64hi(M0, x0), lo0 = M0 * x0;
    uint64_t hi1 = __umul64hi(M1, x2), lo1 = M1 * x2;
    uint64_t y0 = hi1 ^ x1 ^ k0;
    uint64_t y2 = hi0 ^ x3 ^ k1;
    x0 = y0;
    x1 = lo1;
    x2 = y2;
    x3 = lo0;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

}  // namespace rr
