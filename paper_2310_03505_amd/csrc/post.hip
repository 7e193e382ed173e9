// post.hip -- the polar-image epilogue on CDNA4 (gfx950): range blur
// (measurement noise), uniform system noise, gradient-noise ambient noise,
// dB and 8-bit map (Sec. III-B "Polar Image", Sec. III-C "Noise").
//
// One workgroup takes 1024 range bins of one azimuth column; each lane
// produces four consecutive pixels.  The workgroup issues all its global
// loads first, builds the table of lattice gradients its bins need while they
// are in flight, then stages the column segment plus the blur halo in LDS as
// float64.  The
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

// 10 log10(e) for finite e > 0, denormals included.  e = 2^k m with m in
// [sqrt(1/2), sqrt(2)); ln m = 2 atanh(s), s = (m - 1) / (m + 1), |s| < 0.1716,
// from the odd Taylor series of atanh truncated after s^19 (relative
// truncation error below 3e-17); s from a reciprocal refined by two Newton
// steps and a residual correction.  A few ulp from the correctly rounded
// value, in about a third of the instructions of the library's
// double-double log10.
__device__ __forceinline__ double ten_log10(double e) {
  int k;
  double m = frexp(e, &k);
  if (m < 0.70710678118654752440) {
    m = m + m;
    k -= 1;
  }
  const double num = m - 1.0, den = m + 1.0;
  double r = __builtin_amdgcn_rcp(den);
  r = __builtin_fma(r, __builtin_fma(-den, r, 1.0), r);
  r = __builtin_fma(r, __builtin_fma(-den, r, 1.0), r);
  double s = num * r;
  s = __builtin_fma(__builtin_fma(-s, den, num), r, s);
  const double s2 = s * s;
  double p = 1.0 / 19.0;
  p = __builtin_fma(p, s2, 1.0 / 17.0);
  p = __builtin_fma(p, s2, 1.0 / 15.0);
  p = __builtin_fma(p, s2, 1.0 / 13.0);
  p = __builtin_fma(p, s2, 1.0 / 11.0);
  p = __builtin_fma(p, s2, 1.0 / 9.0);
  p = __builtin_fma(p, s2, 1.0 / 7.0);
  p = __builtin_fma(p, s2, 1.0 / 5.0);
  p = __builtin_fma(p, s2, 1.0 / 3.0);
  const double ln_m = __builtin_fma(2.0 * (s * s2), p, 2.0 * s);
  // 10 log10(2) and 10 / ln(10)
  return __builtin_fma(ln_m, 4.3429448190325182765, (double)k * 3.0102999566398119521);
}

// lattice gradient g in 0..7: (1,1), (-1,1), (1,-1), (-1,-1), (1,0), (-1,0),
// (0,1), (0,-1)
__device__ __forceinline__ float2 lattice_gradient(uint32_t g) {
  float gx = g < 6u ? ((g & 1u) ? -1.0f : 1.0f) : 0.0f;
  float gy = g < 4u ? ((g & 2u) ? -1.0f : 1.0f) : (g < 6u ? 0.0f : ((g & 1u) ? -1.0f : 1.0f));
  return make_float2(gx, gy);
}

// g . (dx, dy) with the components exact in float: the products are exact
// and the sum rounds once
__device__ __forceinline__ double grad_dot(float2 g, double dx, double dy) {
  return (double)g.x * dx + (double)g.y * dy;
}

// energy of cell j of the image (or of the fixed-point accumulator, as the
// scan's finalize converts it)
template <bool kFromAcc>
__device__ __forceinline__ float load_cell(const PostArgs& a, size_t j) {
  if constexpr (kFromAcc)
    return (float)((double)a.acc[j] * kFixedInv);
  else
    return a.img[j];
}

template <bool kFromAcc>
__global__ __launch_bounds__(kPostBlock) void k_post(PostArgs a) {
  extern __shared__ double smem[];
  float2* grad = reinterpret_cast<float2*>(smem);  // [2][gcap]
  double* tile = smem + 2u * a.gcap;                // [kPostTile + 2R]
  const uint32_t b0 = blockIdx.x * (uint32_t)kPostTile;
  const uint32_t k = blockIdx.y, img = blockIdx.z;
  const uint32_t nb = min((uint32_t)kPostTile, a.n_bins - b0);
  const int R = a.R;
  const size_t row = ((size_t)img * a.n_az + k) * a.n_bins;
  const uint32_t tid = threadIdx.x;
  // lane t takes the four consecutive bins 4t..4t+3 of the tile: they share
  // one generator block (word s for bin 4t + s) and one 16-byte store
  const uint32_t q0 = 4u * tid;
  const uint32_t nq = q0 < nb ? min(4u, nb - q0) : 0u;
  const uint32_t bq = b0 + q0;
  const size_t o = row + bq;

  // 1. every global load of the block is issued before anything waits on it:
  //    the lane's own four cells and, for lanes below 2R, one halo cell
  // (branch-free: lanes past the tile's end re-read an in-bounds cell and
  // drop it, so the compiler places no wait before the gradient table)
  float c[4];
  {
    const uint32_t last = nq ? nq - 1u : 0u;
    const size_t base = nq ? o : row + b0;
    // (c[t] for t >= nq is a duplicate that no store uses)
#pragma unroll
    for (uint32_t t = 0; t < 4u; ++t) c[t] = load_cell<kFromAcc>(a, base + min(t, last));
  }
  const bool has_halo = (int)tid < 2 * R;
  const long hb = (int)tid < R ? (long)b0 - R + (long)tid : (long)b0 + (long)nb + (long)tid - R;
  const bool halo_in = has_halo && hb >= 0 && hb < (long)a.n_bins;
  const size_t hcell = row + (size_t)(halo_in ? hb : (long)b0);
  const float hv = load_cell<kFromAcc>(a, hcell);
  const float h = halo_in ? hv : 0.0f;
  const int hslot = has_halo ? ((int)tid < R ? (int)tid : R + (int)nb + (int)tid - R) : -1;

  // 2. gradient noise: lattice columns i0, i0 + 1 and rows jlo..jhi of this
  //    tile, computed while the loads are in flight
  const bool perlin = a.pamp > 0.0;
  // (lattice coordinates fit in int: k, b <= 65535 and the cells are >= 1)
  const double x = (double)k / a.cell_az;
  const double fx0 = floor(x);
  const int i0 = (int)fx0;
  const int jlo = (int)floor((double)b0 / a.cell_bins);
  const uint32_t scan = a.scan_id + img;
  if (perlin) {
    const int jhi = (int)floor((double)(b0 + nb - 1u) / a.cell_bins) + 1;
    // the host sizes gcap for the longest row range a tile can span
    const uint32_t cnt = min((uint32_t)(jhi - jlo + 1), a.gcap);
    for (uint32_t t = tid; t < 2u * cnt; t += kPostBlock) {
      uint32_t side = t / cnt, jj = t - side * cnt;
      uint64_t r[4];
      philox4x64_10(a.seed, (uint64_t)scan, (uint64_t)(int64_t)(i0 + (int)side),
                    (uint64_t)(int64_t)(jlo + (int)jj), 2u, 0u, r);
      grad[side * a.gcap + jj] = lattice_gradient((uint32_t)(r[0] >> 61));
    }
  }

  // 3. the scan's float image, and the blur's LDS tile with its halo
  if constexpr (kFromAcc) {
    if (a.image) {
      if (nq == 4u && (reinterpret_cast<uintptr_t>(a.image + o) & 15u) == 0u) {
        *reinterpret_cast<float4*>(a.image + o) = make_float4(c[0], c[1], c[2], c[3]);
      } else {
        for (uint32_t t = 0; t < nq; ++t) a.image[o + t] = c[t];
      }
    }
  }
  if (R > 0) {
#pragma unroll
    for (uint32_t t = 0; t < 4u; ++t)
      if (t < nq) tile[(uint32_t)R + q0 + t] = (double)c[t];
    if (hslot >= 0) tile[hslot] = (double)h;
  }
  __syncthreads();
  if (nq == 0u) return;

  // 4. measurement noise: taps m = 0..2R of tile[q0 + t + m] for bin q0 + t,
  //    each pixel summing its taps in order; a sliding window of four
  //    values reads each tile entry once
  double e[4];
  if (R == 0) {
#pragma unroll
    for (int t = 0; t < 4; ++t) e[t] = 0.0 + 1.0 * (double)c[t];
  } else {
    e[0] = e[1] = e[2] = e[3] = 0.0;
    double v0 = tile[q0], v1 = tile[q0 + 1u], v2 = tile[q0 + 2u];
    for (int m = 0; m <= 2 * R; ++m) {
      const double v3 = tile[q0 + (uint32_t)m + 3u];
      const double wm = a.w[m];
      e[0] += wm * v0;
      e[1] += wm * v1;
      e[2] += wm * v2;
      e[3] += wm * v3;
      v0 = v1;
      v1 = v2;
      v2 = v3;
    }
  }
  // 5. system noise
  if (a.uamp > 0.0) {
    uint64_t r[4];
    philox4x64_10(a.seed, (uint64_t)scan, (uint64_t)k, (uint64_t)(bq >> 2), 1u, 0u, r);
#pragma unroll
    for (int t = 0; t < 4; ++t) e[t] += a.uamp * u53(r[t]);
  }
  // 6. ambient noise
  if (perlin) {
    const double fx = x - fx0;
    const double fu = fade5(fx);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const double y = (double)(bq + (uint32_t)t) / a.cell_bins;
      const double fy0 = floor(y);
      // rows of the last (ragged) group beyond the tile stay inside the table
      const uint32_t jj = min((uint32_t)((int)fy0 - jlo), a.gcap - 2u);
      const double fy = y - fy0;
      const float2* g0 = grad + jj;
      const float2* g1 = grad + a.gcap + jj;
      double n00 = grad_dot(g0[0], fx, fy);
      double n10 = grad_dot(g1[0], fx - 1.0, fy);
      double n01 = grad_dot(g0[1], fx, fy - 1.0);
      double n11 = grad_dot(g1[1], fx - 1.0, fy - 1.0);
      double fv = fade5(fy);
      double nx0 = n00 + fu * (n10 - n00);
      double nx1 = n01 + fu * (n11 - n01);
      double n = nx0 + fv * (nx1 - nx0);
      e[t] += a.pamp * (0.5 + 0.5 * n);
    }
  }
  // 7. dB and 8-bit pixel
  float db[4];
  uint8_t px[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    if (e[t] > 0.0) {
      double L = e[t] <= 1.7976931348623157e308 ? ten_log10(e[t]) : 10.0 * log10(e[t]);
      // one multiply by max / (0 - floor) instead of the division: the
      // pixel value moves by a few ulp at most, far inside the 1e-9 band
      // around rounding boundaries where the two orders may disagree
      double pre = (L - a.db_floor) * a.px_scale;
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
  const size_t lds = post_lds_bytes(a);
  if (a.acc)
    hipLaunchKernelGGL(k_post<true>, grid, dim3(kPostBlock), lds, st, a);
  else
    hipLaunchKernelGGL(k_post<false>, grid, dim3(kPostBlock), lds, st, a);
  return hipGetLastError();
}

}  // namespace rr
