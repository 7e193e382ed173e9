// philox.h -- Philox4x64-10 counter-based generator (device side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rr {

// 128-bit product of two 64-bit words from four 32 x 32 -> 64 partial
// products, each the multiply-add of a 64-bit accumulator; the low word
// shares the partial products of the high word
__device__ __forceinline__ void mulhilo64(uint64_t a, uint64_t b, uint64_t& hi, uint64_t& lo) {
  const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
  const uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
  const uint64_t p00 = (uint64_t)a0 * b0;
  const uint64_t m1 = (uint64_t)a0 * b1 + (p00 >> 32);        // < 2^64
  const uint64_t m2 = (uint64_t)a1 * b0 + (uint32_t)m1;         // < 2^64
  hi = (uint64_t)a1 * b1 + (m1 >> 32) + (m2 >> 32);
  lo = (m2 << 32) | (uint32_t)p00;
}

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
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo64(M0, x0, hi0, lo0);
    mulhilo64(M1, x2, hi1, lo1);
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
