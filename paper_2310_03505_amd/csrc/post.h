// post.h -- launch interface of the polar-image epilogue (Sec. III-B "Polar
// Image", Sec. III-C "Noise").
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rr {

constexpr int kPostMaxR = 48;     // blur half-width ceil(3 sigma) for sigma <= 16 bins
constexpr int kPostTile = 1024;   // range bins per workgroup
constexpr int kPostBlock = 256;

// One launch processes n_images images of n_az x n_bins, row-major
// [image][azimuth][bin].  Exactly one of img (float energies) and acc (the
// 2^56 fixed-point accumulator, converted to float as the scan's finalize
// does) is set; with acc, image (optional) receives the converted floats.
struct PostArgs {
  const float* img;
  const unsigned long long* acc;
  float* image;
  float* db;        // optional: 10 log10(E), float32
  uint8_t* u8;      // optional: 8-bit pixel
  uint32_t n_az, n_bins, n_images;
  int R;            // blur half-width in bins (0: no blur)
  double w[2 * kPostMaxR + 1];  // blur weights, normalised to sum 1
  double uamp, pamp;            // uniform and gradient-noise amplitudes
  double cell_az, cell_bins;    // gradient-noise lattice spacing (>= 1)
  double db_floor, max_value;
  double px_scale;              // max_value / (0 - db_floor)
  uint64_t seed;
  uint32_t scan_id;             // image i uses scan_id + i
  uint32_t gcap;                // gradient-table rows per lattice column (0: no gradient noise)
};

// Dynamic LDS of one k_post workgroup: the gradient table (2 x gcap float2)
// and, with a blur, the float64 tile of 1024 bins plus the halo.
inline size_t post_lds_bytes(const PostArgs& a) {
  return (size_t)2 * a.gcap * 8 + (a.R > 0 ? (size_t)(kPostTile + 2 * a.R) * 8 : 0);
}

hipError_t launch_post(const PostArgs& a, hipStream_t st);

}  // namespace rr
