// post.hip -- the polar-image epilogue on CDNA4 (gfx950): range blur
// (measurement noise), uniform system noise, gradient-noise ambient noise,
// dB and 8-bit map (Sec. III-B "Polar Image", Sec. III-C "Noise").
//
// One workgroup takes 1024 range bins of one azimuth column: it stages the
// column segment plus the blur halo in LDS as float64, the lattice gradients
// its bins need, and the blur weights; each lane then produces four
// consecutive pixels.  The
// arithmetic is float64 in a fixed order without contraction, so the only
// library function whose rounding can differ from another implementation is
// log10.
#include <hip/hip_runtime.h>

#include "philox.h"
#include "post.h"
#include "rr_internal.h"

#pragma clang fp contract(off)

namespace rr {

namespace {

__device__ __forceinline__ double u53(uint64_t x) { return (double)(x >> 11) * (1.0 / 9007199254740992.0); }

// quintic fade of improved gradient noise (Perlin, SIGGRAPH 2002)
__device__ __forceinline__ double fade5(double t) { return t * t * t * (t * (t * 6.0 - 15.0) + 10.0); }

// lattice gradient g in 0..7: (+-1, +-1), (+-1, 0), (0, +-1)
__device__ __forceinline__ double grad_dot(uint32_t g, double dx, double dy) {
  double gx = g < 6u ? ((g & 1u) ? -1.0 : 1.0) : 0.0;
  double gy = g < 4u ? ((g & 2u) ? -1.0 : 1.0) : (g < 6u ? 0.0 : ((g & 1u) ? -1.0 : 1.0));
  return gx * dx + gy * dy;
}

template <bool kFromAcc>
__global__ __launch_bounds__(kPostBlock) void k_post(PostArgs a) {
  __shared__ double tile[kPostTile + 2 * kPostMaxR];
  __shared__ double w[2 * kPostMaxR + 1];
  __shared__ uint8_t grad[2][kPostTile + 4];
  const uint32_t b0 = blockIdx.x * (uint32_t)kPostTile;
  const uint32_t k = blockIdx.y, img = blockIdx.z;
  const uint32_t nb = min((uint32_t)kPostTile, a.n_bins - b0);
  const int R = a.R;
  const size_t row = ((size_t)img * a.n_az + k) * a.n_bins;
  const uint32_t tid = threadIdx.x;
  for (int j = (int)tid; j < 2 * R + 1; j += kPostBlock) w[j] = a.w[j];
  for (int j = (int)tid; j < (int)nb + 2 * R; j += kPostBlock) {
    long b = (long)b0 - R + j;
    double v = 0.0;
    if (b >= 0 && b < (long)a.n_bins) {
      float f;
      if constexpr (kFromAcc) {
        f = (float)((double)a.acc[row + (size_t)b] * kFixedInv);
        if (a.image && j >= R && j < R + (int)nb) a.image[row + (size_t)b] = f;
      } else {
        f = a.img[row + (size_t)b];
      }
      v = (double)f;
    }
    tile[j] = v;
  }
  // gradient noise: lattice columns i0, i0 + 1 and rows jlo..jhi of this tile
  const bool perlin = a.pamp > 0.0;
  const double x = (double)k / a.cell_az;
  const double fx0 = floor(x);
  const int64_t i0 = (int64_t)fx0;
  const int64_t jlo = (int64_t)floor((double)b0 / a.cell_bins);
  const uint32_t scan = a.scan_id + img;
  if (perlin) {
    const int64_t jhi = (int64_t)floor((double)(b0 + nb - 1u) / a.cell_bins) + 1;
    // jhi - jlo <= nb for cell_bins >= 1 (one more than the exact bound for
    // the rounding of the two quotients); clamped to the table regardless
    const uint32_t cnt = min((uint32_t)(jhi - jlo + 1), (uint32_t)kPostTile + 4u);
    for (uint32_t t = tid; t < 2u * cnt; t += kPostBlock) {
      uint32_t side = t / cnt, jj = t - side * cnt;
      uint64_t r[4];
      philox4x64_10(a.seed, (uint64_t)scan, (uint64_t)(i0 + (int64_t)side), (uint64_t)(jlo + (int64_t)jj), 2u,
                    0u, r);
      grad[side][jj] = (uint8_t)(r[0] >> 61);
    }
  }
  __syncthreads();
  const double fx = x - fx0;
  const double fu = fade5(fx);
  const double span = 0.0 - a.db_floor;
  // lane t takes the four consecutive bins 4t..4t+3 of the tile: they share
  // one generator block (word s for bin 4t + s) and one 16-byte store
  const uint32_t q0 = 4u * tid;
  if (q0 >= nb) return;
  const uint32_t nq = min(4u, nb - q0);
  const uint32_t bq = b0 + q0;
  double e[4] = {0.0, 0.0, 0.0, 0.0};
  // each tap value is read once and added to the pixels it reaches, every
  // pixel still summing its taps in order
  for (int j = 0; j < 2 * R + 4; ++j) {
    const double v = tile[q0 + (uint32_t)j];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int m = j - t;
      if (m >= 0 && m <= 2 * R) e[t] += w[m] * v;
    }
  }
  if (a.uamp > 0.0) {
    uint64_t r[4];
    philox4x64_10(a.seed, (uint64_t)scan, (uint64_t)k, (uint64_t)(bq >> 2), 1u, 0u, r);
#pragma unroll
    for (int t = 0; t < 4; ++t) e[t] += a.uamp * u53(r[t]);
  }
  if (perlin) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const double y = (double)(bq + (uint32_t)t) / a.cell_bins;
      const double fy0 = floor(y);
      // rows of the last (ragged) group beyond the tile stay inside grad[]
      const uint32_t jj = min((uint32_t)((int64_t)fy0 - jlo), (uint32_t)kPostTile + 2u);
      const double fy = y - fy0;
      double n00 = grad_dot(grad[0][jj], fx, fy);
      double n10 = grad_dot(grad[1][jj], fx - 1.0, fy);
      double n01 = grad_dot(grad[0][jj + 1u], fx, fy - 1.0);
      double n11 = grad_dot(grad[1][jj + 1u], fx - 1.0, fy - 1.0);
      double fv = fade5(fy);
      double nx0 = n00 + fu * (n10 - n00);
      double nx1 = n01 + fu * (n11 - n01);
      double n = nx0 + fv * (nx1 - nx0);
      e[t] += a.pamp * (0.5 + 0.5 * n);
    }
  }
  float db[4];
  uint8_t px[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    if (e[t] > 0.0) {
      double L = 10.0 * log10(e[t]);
      double pre = a.max_value * (L - a.db_floor) / span;
      double qv = floor(pre + 0.5);
      if (!(qv > 0.0)) qv = 0.0;
      if (qv > a.max_value) qv = a.max_value;
      db[t] = (float)L;
      px[t] = (uint8_t)qv;
    } else {
      db[t] = -__builtin_huge_valf();
      px[t] = 0;
    }
  }
  const size_t o = row + bq;
  if (a.db) {
    float* d = a.db + o;
    if (nq == 4u && (reinterpret_cast<uintptr_t>(d) & 15u) == 0u)
      *reinterpret_cast<float4*>(d) = make_float4(db[0], db[1], db[2], db[3]);
    else
      for (uint32_t t = 0; t < nq; ++t) d[t] = db[t];
  }
  if (a.u8) {
    uint8_t* u = a.u8 + o;
    if (nq == 4u && (reinterpret_cast<uintptr_t>(u) & 3u) == 0u)
      *reinterpret_cast<uint32_t*>(u) =
          (uint32_t)px[0] | ((uint32_t)px[1] << 8) | ((uint32_t)px[2] << 16) | ((uint32_t)px[3] << 24);
    else
      for (uint32_t t = 0; t < nq; ++t) u[t] = px[t];
  }
}

}  // namespace

hipError_t launch_post(const PostArgs& a, hipStream_t st) {
  if (a.n_az == 0 || a.n_bins == 0 || a.n_images == 0) return hipSuccess;
  dim3 grid((a.n_bins + kPostTile - 1) / kPostTile, a.n_az, a.n_images);
  if (a.acc)
    hipLaunchKernelGGL(k_post<true>, grid, dim3(kPostBlock), 0, st, a);
  else
    hipLaunchKernelGGL(k_post<false>, grid, dim3(kPostBlock), 0, st, a);
  return hipGetLastError();
}

}  // namespace rr
