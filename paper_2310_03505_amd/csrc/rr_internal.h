// rr_internal.h -- layouts shared by the host side (BVH builder, C ABI) and
// the HIP kernels.  Not part of the public ABI.
#pragma once

#include <stddef.h>
#include <stdint.h>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define RR_HD __host__ __device__ __forceinline__
#else
#include <cmath>
#define RR_HD inline
struct alignas(16) float4 {
  float x, y, z, w;
};
struct alignas(16) int4 {
  int x, y, z, w;
};
struct alignas(16) uint4 {
  unsigned x, y, z, w;
};
#endif

namespace rr {

constexpr int kMaxDepth = 32;  // two-wide build: inner-node depth bound
constexpr int kStack = 16;     // traversal stack entries per lane held in LDS
constexpr int kSpill = 80;     // further entries per lane in workspace memory

// Four-wide node with quantised child boxes, 64 bytes (four 16-byte loads):
//   w0 = (origin.x, origin.y, origin.z, exponent bytes ex | ey << 8 | ez << 16)
//   w1 = (qlo.x[4], qhi.x[4], qlo.y[4], qhi.y[4])   one byte per child
//   w2 = (qlo.z[4], qhi.z[4], 0, 0)
//   w3 = child refs: inner node index (< 2^30), kEmpty for no child, or a
//        leaf: bit 31 | (count - 1) << 27 | first leaf triangle (< 2^27)
// Child j covers origin + q * 2^(e - 127) on each axis, rounded outward from
// the padded float box, so decoding never shrinks a box.  A slot without a
// child (ref kEmpty) holds the inverted box qlo = 255, qhi = 0 on every
// axis, which no ray interval meets (node4_slabs relies on it).
struct alignas(64) Node4 {
  float4 w0;
  uint4 w1, w2;
  int4 w3;
};
static_assert(sizeof(Node4) == 64, "node layout");
constexpr int32_t kEmpty = 0x7fffffff;
constexpr uint32_t kMaxLeafTris = 1u << 27;
RR_HD int32_t leaf_ref_encode(uint32_t start, uint32_t count) {
  return (int32_t)(0x80000000u | ((count - 1u) << 27) | start);
}
RR_HD uint32_t leaf_start(int32_t ref) { return (uint32_t)ref & (kMaxLeafTris - 1u); }
// Every slot j with ref[j] == kEmpty gets the inverted box: low bytes 255,
// high bytes 0 on each axis (qlo / qhi hold one byte per slot and axis).
RR_HD void invert_empty_slots(const int32_t ref[4], uint32_t qlo[3], uint32_t qhi[3]) {
  for (int j = 0; j < 4; ++j) {
    if (ref[j] != kEmpty) continue;
    for (int a = 0; a < 3; ++a) {
      qlo[a] |= 0xffu << (8 * j);
      qhi[a] &= ~(0xffu << (8 * j));
    }
  }
}
RR_HD uint32_t leaf_count(int32_t ref) { return (((uint32_t)ref >> 27) & 15u) + 1u; }

// Leaf-ordered triangle, 48 bytes: v0 with the original id in w, then the
// edges e1 = v1 - v0 and e2 = v2 - v0 (float32, computed on the host).
// A second 16-byte array holds (geometric unit normal, material id bits).

// Material table entry on the device.  a, beta, s: beam-window coefficients
// of the normalised standard BRDF (Eq. 3-5), see api.cpp; for the
// Cook-Torrance kind: diffuse amount, roughness and the beam cone's solid
// angle.
struct DevMaterial {
  uint32_t kind;
  float n;
  float refl;
  float C;
  double a, beta, s;
  double pad;
};
static_assert(sizeof(DevMaterial) == 48, "material layout");

// Per-scan constants on the device.
struct DevScan {
  double R[9];      // sensor-to-world rotation (row-major)
  double sigma_r;   // Eq. 2 radius scale
  float pos[3];     // sensor position
  float e0;         // 1/N_s, float32
  float bin_size;
  float r_max;      // n_bins * bin_size, float32
  float e_cut;
  uint32_t n_az, n_s, max_b, n_bins, flags, scan_id;
  uint64_t seed;
  float stretch_az, stretch_inc;  // elliptic beam: factors of the cone offsets (1 = circular)
  uint32_t prim_base;  // first global primary of this scan
  uint32_t n_prim;     // n_az * n_s
  uint64_t acc_base;   // first accumulator cell of this scan
  float* image;
  int32_t* records;
  const uint8_t* mask;
};

// Ray-queue entry, split in four arrays:
//   a = (o.x, o.y, o.z, L)        L = optical path length so far
//   b = (d.x, d.y, d.z, g)        g = receive gain of the primary
//   c = (E lo, E hi, pid, excl)   E float64 energy; pid = primary within the
//                                 scan; excl = original id of the triangle
//                                 last hit (0xffffffff for a primary)
//   m = heap | medium << 8 | scan << 16   (medium 255 = air)
constexpr uint32_t kAir = 255u;
constexpr size_t kRayBytes = 16 + 16 + 16 + 4;

// counters block (uint32): [0..8] rays per depth, [32] overflow flag, [40]
// air-path visibility rays of the scan, [64..) the claim cursors of the
// traversal levels and of the visibility launch; only the first 64 words are
// read back to the host
constexpr int kCtrCount = 0;
constexpr int kCtrOverflow = 32;
// bits of the overflow word: 1, a ray queue or the visibility queue was
// full; 2, a tail-helping traversal reached its iteration bound
constexpr uint32_t kOverflowSteps = 2u;
constexpr int kCtrShadow = 40;
constexpr int kCtrHostWords = 64;   // the part of the block read back to the host
// per level, sixteen claim cursors (one per segment of the level's queue),
// each on its own 128-byte line
constexpr int kCtrCursor = 64;
constexpr int kCtrSegs = 16;
constexpr int kCtrCursorStride = 32;
constexpr int kCtrWords = kCtrCursor + 9 * kCtrSegs * kCtrCursorStride;  // eight levels at most, then visibility

// Air-path visibility ray (one per air-path return to test), three arrays:
//   a = (o.x, o.y, o.z, dist)   offset origin, distance to the sensor
//   b = (s.x, s.y, s.z, slot)   unit direction to the sensor; slot = record
//                               index of the outcome (bits), 0xffffffff none
//   c = (q lo, q hi, cell, excl) fixed-point energy of the return, its
//                               accumulator cell, the triangle just hit
constexpr size_t kShadowBytes = 16 + 16 + 16;
constexpr uint32_t kFlagAirPath = 16u;

constexpr double kFixedScale = 72057594037927936.0;  // 2^56
constexpr double kFixedInv = 1.0 / 72057594037927936.0;

// ---------------------------------------------------------------- geometry
// float32, fixed operation order, no contraction: the closest-hit decision
// must be identical wherever it is evaluated.
RR_HD float dot3(float ax, float ay, float az, float bx, float by, float bz) {
  float xy = ax * bx + ay * by;
  return xy + az * bz;
}

// Moller & Trumbore 1997 on (v0, e1, e2), both faces, inclusive bounds,
// accepts 0 < t <= tmax.
RR_HD bool ray_tri(float ox, float oy, float oz, float dx, float dy, float dz, float v0x,
                   float v0y, float v0z, float e1x, float e1y, float e1z, float e2x, float e2y,
                   float e2z, float tmax, float& t_out) {
  float px = dy * e2z - dz * e2y;
  float py = dz * e2x - dx * e2z;
  float pz = dx * e2y - dy * e2x;
  float det = dot3(e1x, e1y, e1z, px, py, pz);
  if (det == 0.0f) return false;
  float inv = 1.0f / det;
  float sx = ox - v0x, sy = oy - v0y, sz = oz - v0z;
  float u = dot3(sx, sy, sz, px, py, pz) * inv;
  if (u < 0.0f || u > 1.0f) return false;
  float qx = sy * e1z - sz * e1y;
  float qy = sz * e1x - sx * e1z;
  float qz = sx * e1y - sy * e1x;
  float v = dot3(dx, dy, dz, qx, qy, qz) * inv;
  if (v < 0.0f || u + v > 1.0f) return false;
  float t = dot3(e2x, e2y, e2z, qx, qy, qz) * inv;
  if (!(t > 0.0f && t <= tmax)) return false;
  t_out = t;
  return true;
}

// ---------------------------------------------------------------- boxes
// Entry and exit distances of the four children of a quantised node.
// hit[j] is set for children whose (conservative) box meets [0, tmax].
RR_HD float byte_f(uint32_t w, int j) { return (float)((w >> (8 * j)) & 0xffu); }

RR_HD float pow2_from_byte(uint32_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __uint_as_float(b << 23);
#else
  uint32_t u = b << 23;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return f;
#endif
}
// Slab test of both child boxes of a node.  The builder pads every box by a
// fixed absolute margin and the far distance gets a relative slack, so a
// triangle hit accepted by ray_tri is never culled by rounding here.
constexpr float kSlabSlack = 1.0f + 1.0f / 1048576.0f;

struct RayBox {
  float ix, iy, iz;     // 1 / d (zero components replaced by +-1e-20)
  float oix, oiy, oiz;  // o / d
};

RR_HD void ray_box_setup(float ox, float oy, float oz, float dx, float dy, float dz, RayBox& r) {
  const float tiny = 1e-20f;
  float sx = fabsf(dx) > tiny ? dx : copysignf(tiny, dx);
  float sy = fabsf(dy) > tiny ? dy : copysignf(tiny, dy);
  float sz = fabsf(dz) > tiny ? dz : copysignf(tiny, dz);
  r.ix = 1.0f / sx;
  r.iy = 1.0f / sy;
  r.iz = 1.0f / sz;
  r.oix = ox * r.ix;
  r.oiy = oy * r.iy;
  r.oiz = oz * r.iz;
}

// Entry distances of the four children of a quantised node; returns the mask
// of children whose box meets [0, tmax].  Per axis the child bounds decode as
// t = q * (2^e / d) + (origin - o) / d, one fused multiply-add per bound.
// The near plane of an axis is its low bound when the direction component
// is positive and its high bound otherwise; fma(q, s, b) is monotone in q,
// so choosing the byte planes by the sign of 1/d equals taking min / max of
// both decoded bounds.
RR_HD uint32_t node4_boxes(const float4& w0, const uint4& w1, const uint4& w2, const int4& w3,
                           const RayBox& r, float tmax, float tn[4]) {
  uint32_t eb;
#if defined(__HIP_DEVICE_COMPILE__)
  eb = __float_as_uint(w0.w);
#else
  __builtin_memcpy(&eb, &w0.w, 4);
#endif
  const float sx = pow2_from_byte(eb & 0xffu) * r.ix;
  const float sy = pow2_from_byte((eb >> 8) & 0xffu) * r.iy;
  const float sz = pow2_from_byte((eb >> 16) & 0xffu) * r.iz;
  const float bx = fmaf(w0.x, r.ix, -r.oix);
  const float by = fmaf(w0.y, r.iy, -r.oiy);
  const float bz = fmaf(w0.z, r.iz, -r.oiz);
  const bool px = r.ix >= 0.0f, py = r.iy >= 0.0f, pz = r.iz >= 0.0f;
  const uint32_t nx = px ? w1.x : w1.y, fx = px ? w1.y : w1.x;
  const uint32_t ny = py ? w1.z : w1.w, fy = py ? w1.w : w1.z;
  const uint32_t nz = pz ? w2.x : w2.y, fz = pz ? w2.y : w2.x;
  const int32_t ref[4] = {w3.x, w3.y, w3.z, w3.w};
  uint32_t mask = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float tnx = fmaf(byte_f(nx, j), sx, bx), tfx = fmaf(byte_f(fx, j), sx, bx);
    const float tny = fmaf(byte_f(ny, j), sy, by), tfy = fmaf(byte_f(fy, j), sy, by);
    const float tnz = fmaf(byte_f(nz, j), sz, bz), tfz = fmaf(byte_f(fz, j), sz, bz);
    const float a = fmaxf(fmaxf(tnx, tny), fmaxf(tnz, 0.0f));
    const float f = fminf(fminf(tfx, tfy), fminf(tfz, tmax));
    tn[j] = a;
    if (a <= f * kSlabSlack && ref[j] != kEmpty) mask |= 1u << j;
  }
  return mask;
}

// The slab tests of node4_boxes without the empty-slot test, for the trace
// kernel: an empty slot holds an inverted box (see Node4), whose entry
// distance exceeds its exit distance by at least 255 quantisation steps.
// hit[j]: child j's box meets [0, tmax]; tn[j]: its entry distance (>= 0).
RR_HD void node4_slabs(const float4& w0, const uint4& w1, const uint4& w2, const RayBox& r, float tmax,
                       float tn[4], bool hit[4]) {
  uint32_t eb;
#if defined(__HIP_DEVICE_COMPILE__)
  eb = __float_as_uint(w0.w);
#else
  __builtin_memcpy(&eb, &w0.w, 4);
#endif
  const float sx = pow2_from_byte(eb & 0xffu) * r.ix;
  const float sy = pow2_from_byte((eb >> 8) & 0xffu) * r.iy;
  const float sz = pow2_from_byte((eb >> 16) & 0xffu) * r.iz;
  const float bx = fmaf(w0.x, r.ix, -r.oix);
  const float by = fmaf(w0.y, r.iy, -r.oiy);
  const float bz = fmaf(w0.z, r.iz, -r.oiz);
  const bool px = r.ix >= 0.0f, py = r.iy >= 0.0f, pz = r.iz >= 0.0f;
  const uint32_t nx = px ? w1.x : w1.y, fx = px ? w1.y : w1.x;
  const uint32_t ny = py ? w1.z : w1.w, fy = py ? w1.w : w1.z;
  const uint32_t nz = pz ? w2.x : w2.y, fz = pz ? w2.y : w2.x;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float tnx = fmaf(byte_f(nx, j), sx, bx), tfx = fmaf(byte_f(fx, j), sx, bx);
    const float tny = fmaf(byte_f(ny, j), sy, by), tfy = fmaf(byte_f(fy, j), sy, by);
    const float tnz = fmaf(byte_f(nz, j), sz, bz), tfz = fmaf(byte_f(fz, j), sz, bz);
    const float a = fmaxf(fmaxf(tnx, tny), fmaxf(tnz, 0.0f));
    const float f = fminf(fminf(tfx, tfy), fminf(tfz, tmax));
    tn[j] = a;
    hit[j] = a <= f * kSlabSlack;
  }
}

// Eight-wide node, 80 bytes (five 16-byte loads):
//   w0 = (origin.x, origin.y, origin.z, ex | ey << 8 | ez << 16 | imask << 24)
//   w1 = (first inner child, first triangle | leafmask << 24, meta[0..3], meta[4..7])
//   w2 = (qlo.x[0..3], qlo.x[4..7], qhi.x[0..3], qhi.x[4..7])   one byte per slot
//   w3 = (qlo.y[0..3], qlo.y[4..7], qhi.y[0..3], qhi.y[4..7])
//   w4 = (qlo.z[0..3], qlo.z[4..7], qhi.z[0..3], qhi.z[4..7])
// Slot s holds an inner child (imask bit s: node first + number of inner
// slots below s, so the inner children of a node are consecutive), a leaf
// (leafmask bit s: meta[s] = (count - 1) << 5 | offset, its triangles at
// first triangle + offset ...), or nothing.  The builder puts the child that
// lies toward the box corner with sign bits s (bit a set: high side of axis
// a) into slot s, so a ray whose direction has sign bits o (bit a set:
// negative) meets the children roughly in the order of slot i ^ o, i = 0..7.
struct alignas(16) Node8 {
  float4 w0;
  uint4 w1, w2, w3, w4;
};
static_assert(sizeof(Node8) == 80, "node layout");
constexpr uint32_t kMaxTris8 = 1u << 24;  // triangle references an eight-wide tree addresses

// Hit mask of the eight children of a quantised node (bit s: slot s's box
// meets [0, tmax]); tn[s] receives the entry distances.  Same decode and
// conservative rounding as node4_boxes.
RR_HD uint32_t node8_boxes(const Node8& n, const RayBox& r, float tmax) {
  uint32_t eb;
#if defined(__HIP_DEVICE_COMPILE__)
  eb = __float_as_uint(n.w0.w);
#else
  __builtin_memcpy(&eb, &n.w0.w, 4);
#endif
  const float sx = pow2_from_byte(eb & 0xffu) * r.ix;
  const float sy = pow2_from_byte((eb >> 8) & 0xffu) * r.iy;
  const float sz = pow2_from_byte((eb >> 16) & 0xffu) * r.iz;
  const float bx = fmaf(n.w0.x, r.ix, -r.oix);
  const float by = fmaf(n.w0.y, r.iy, -r.oiy);
  const float bz = fmaf(n.w0.z, r.iz, -r.oiz);
  const bool px = r.ix >= 0.0f, py = r.iy >= 0.0f, pz = r.iz >= 0.0f;
  // near / far planes: (lo, hi) bytes for a positive direction, else swapped
  const uint32_t nx0 = px ? n.w2.x : n.w2.z, nx1 = px ? n.w2.y : n.w2.w;
  const uint32_t fx0 = px ? n.w2.z : n.w2.x, fx1 = px ? n.w2.w : n.w2.y;
  const uint32_t ny0 = py ? n.w3.x : n.w3.z, ny1 = py ? n.w3.y : n.w3.w;
  const uint32_t fy0 = py ? n.w3.z : n.w3.x, fy1 = py ? n.w3.w : n.w3.y;
  const uint32_t nz0 = pz ? n.w4.x : n.w4.z, nz1 = pz ? n.w4.y : n.w4.w;
  const uint32_t fz0 = pz ? n.w4.z : n.w4.x, fz1 = pz ? n.w4.w : n.w4.y;
  const uint32_t present = (eb >> 24) | (n.w1.y >> 24);
  uint32_t mask = 0;
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int j = s & 3;
    const uint32_t nx = s < 4 ? nx0 : nx1, fx = s < 4 ? fx0 : fx1;
    const uint32_t ny = s < 4 ? ny0 : ny1, fy = s < 4 ? fy0 : fy1;
    const uint32_t nz = s < 4 ? nz0 : nz1, fz = s < 4 ? fz0 : fz1;
    const float tnx = fmaf(byte_f(nx, j), sx, bx), tfx = fmaf(byte_f(fx, j), sx, bx);
    const float tny = fmaf(byte_f(ny, j), sy, by), tfy = fmaf(byte_f(fy, j), sy, by);
    const float tnz = fmaf(byte_f(nz, j), sz, bz), tfz = fmaf(byte_f(fz, j), sz, bz);
    const float a = fmaxf(fmaxf(tnx, tny), fmaxf(tnz, 0.0f));
    const float f = fminf(fminf(tfx, tfy), fminf(tfz, tmax));
    if (a <= f * kSlabSlack) mask |= 1u << s;
  }
  return mask & present;
}

// Octant code of a ray (bit a set: negative direction on axis a) and the
// hit mask reordered so that bit i stands for slot i ^ octant.
RR_HD uint32_t ray_octant(const RayBox& r) {
  return (r.ix < 0.0f ? 1u : 0u) | (r.iy < 0.0f ? 2u : 0u) | (r.iz < 0.0f ? 4u : 0u);
}
RR_HD uint32_t octant_order(uint32_t m, uint32_t oct) {
  if (oct & 1u) m = ((m & 0x55u) << 1) | ((m >> 1) & 0x55u);
  if (oct & 2u) m = ((m & 0x33u) << 2) | ((m >> 2) & 0x33u);
  if (oct & 4u) m = ((m & 0x0fu) << 4) | ((m >> 4) & 0x0fu);
  return m;
}

}  // namespace rr
