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

// BVH2 node, 64 bytes: the boxes of both children are stored in the parent
// so one 64-byte fetch decides both (Aila & Laine 2009 layout).
//   n0 = (c0.lo.x, c0.hi.x, c0.lo.y, c0.hi.y)
//   n1 = (c1.lo.x, c1.hi.x, c1.lo.y, c1.hi.y)
//   n2 = (c0.lo.z, c0.hi.z, c1.lo.z, c1.hi.z)
//   n3 = (child0, child1, count0, count1)
// child >= 0: inner node index; child < 0: leaf whose triangles start at
// ~child in the leaf-ordered triangle array, count in n3.z / n3.w.
struct alignas(64) Node {
  float4 n0, n1, n2;
  int4 n3;
};
static_assert(sizeof(Node) == 64, "node layout");

constexpr int kMaxDepth = 32;  // two-wide build: inner-node depth bound
constexpr int kStack = 20;     // traversal stack entries per lane held in LDS
constexpr int kSpill = 76;     // further entries per lane in workspace memory

// Four-wide node with quantised child boxes, 64 bytes (four 16-byte loads):
//   w0 = (origin.x, origin.y, origin.z, exponent bytes ex | ey << 8 | ez << 16)
//   w1 = (qlo.x[4], qhi.x[4], qlo.y[4], qhi.y[4])   one byte per child
//   w2 = (qlo.z[4], qhi.z[4], 0, 0)
//   w3 = child refs: inner node index (< 2^30), kEmpty for no child, or a
//        leaf: bit 31 | (count - 1) << 27 | first leaf triangle (< 2^27)
// Child j covers origin + q * 2^(e - 127) on each axis, rounded outward from
// the padded float box, so decoding never shrinks a box.
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
RR_HD uint32_t leaf_count(int32_t ref) { return (((uint32_t)ref >> 27) & 15u) + 1u; }

// Leaf-ordered triangle, 48 bytes: v0 with the original id in w, then the
// edges e1 = v1 - v0 and e2 = v2 - v0 (float32, computed on the host).
// A second 16-byte array holds (geometric unit normal, material id bits).

// Material table entry on the device.  a, beta, s: beam-window coefficients
// of the normalised standard BRDF (Eq. 3-5), see api.cpp.
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
//                                 scan; excl = leaf index of the last hit
//   m = heap | medium << 8 | scan << 16   (medium 255 = air)
constexpr uint32_t kAir = 255u;
constexpr size_t kRayBytes = 16 + 16 + 16 + 4;

// counters block (uint32): [0..8] rays per depth, [16..24] work cursors,
// [32] overflow flag
constexpr int kCtrCount = 0;
constexpr int kCtrWork = 16;
constexpr int kCtrOverflow = 32;
constexpr int kCtrWords = 64;

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

RR_HD void node_boxes(const float4& n0, const float4& n1, const float4& n2, const RayBox& r,
                      float tmax, bool& hit0, bool& hit1, float& tn0, float& tn1) {
  float l0x = fmaf(n0.x, r.ix, -r.oix), h0x = fmaf(n0.y, r.ix, -r.oix);
  float l0y = fmaf(n0.z, r.iy, -r.oiy), h0y = fmaf(n0.w, r.iy, -r.oiy);
  float l0z = fmaf(n2.x, r.iz, -r.oiz), h0z = fmaf(n2.y, r.iz, -r.oiz);
  float l1x = fmaf(n1.x, r.ix, -r.oix), h1x = fmaf(n1.y, r.ix, -r.oix);
  float l1y = fmaf(n1.z, r.iy, -r.oiy), h1y = fmaf(n1.w, r.iy, -r.oiy);
  float l1z = fmaf(n2.z, r.iz, -r.oiz), h1z = fmaf(n2.w, r.iz, -r.oiz);
  tn0 = fmaxf(fmaxf(fminf(l0x, h0x), fminf(l0y, h0y)), fmaxf(fminf(l0z, h0z), 0.0f));
  float tf0 = fminf(fminf(fmaxf(l0x, h0x), fmaxf(l0y, h0y)), fminf(fmaxf(l0z, h0z), tmax));
  tn1 = fmaxf(fmaxf(fminf(l1x, h1x), fminf(l1y, h1y)), fmaxf(fminf(l1z, h1z), 0.0f));
  float tf1 = fminf(fminf(fmaxf(l1x, h1x), fmaxf(l1y, h1y)), fminf(fmaxf(l1z, h1z), tmax));
  hit0 = tn0 <= tf0 * kSlabSlack;
  hit1 = tn1 <= tf1 * kSlabSlack;
}

}  // namespace rr
