// bvh_gpu.hip -- linear BVH on the GPU: Morton codes of the triangle
// centroids, a radix sort, the binary radix tree of Karras ("Maximizing
// parallelism in the construction of BVHs, octrees, and k-d trees", HPG
// 2012), bottom-up boxes with one visit counter per inner node, and a
// collapse of every other level into the four-wide quantised nodes the
// traversal kernels read.  Every inner node covers a contiguous range of the
// sorted triangles, so a subtree of at most max_leaf triangles becomes one
// leaf without copying.  A refit keeps the tree and recomputes triangles,
// normals, boxes and node frames from moved vertices; a four-wide tree built
// on the host is refitted the same way, one launch per depth of its nodes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "bvh_gpu.h"

#pragma clang fp contract(off)

namespace rr {

namespace {

constexpr int kB = 256;
// misc words: [0..2] centroid minimum and [3..5] maximum (order-preserving
// encodings), [6] largest coordinate magnitude (float bits, >= 1), [7]
// hittable triangles, [8] four-wide nodes, [9] leaves, [10] deepest
// four-wide node, [11] deepest binary inner node
constexpr int kMiscWords = 16;

__device__ __forceinline__ uint32_t fenc(float f) {
  const uint32_t b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float fdec(uint32_t u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

// triangle j: vertices, edges, geometric normal (the host build's float32
// operations, so normals match bit for bit); nn > 0 marks a hittable one
struct Tri {
  float p0[3], p1[3], p2[3], e1[3], e2[3], n[3], nn;
};
__device__ __forceinline__ void load_tri(const GpuBvh& g, uint32_t j, Tri& t) {
  const float* a = g.V + 3u * g.F[3u * j + 0u];
  const float* b = g.V + 3u * g.F[3u * j + 1u];
  const float* c = g.V + 3u * g.F[3u * j + 2u];
  for (int k = 0; k < 3; ++k) {
    t.p0[k] = a[k];
    t.p1[k] = b[k];
    t.p2[k] = c[k];
    t.e1[k] = t.p1[k] - t.p0[k];
    t.e2[k] = t.p2[k] - t.p0[k];
  }
  t.n[0] = t.e1[1] * t.e2[2] - t.e1[2] * t.e2[1];
  t.n[1] = t.e1[2] * t.e2[0] - t.e1[0] * t.e2[2];
  t.n[2] = t.e1[0] * t.e2[1] - t.e1[1] * t.e2[0];
  t.nn = dot3(t.n[0], t.n[1], t.n[2], t.n[0], t.n[1], t.n[2]);
}

__device__ __forceinline__ void tri_box(const Tri& t, float lo[3], float hi[3]) {
  for (int k = 0; k < 3; ++k) {
    lo[k] = fminf(fminf(t.p0[k], t.p1[k]), t.p2[k]);
    hi[k] = fmaxf(fmaxf(t.p0[k], t.p1[k]), t.p2[k]);
  }
}

__device__ __forceinline__ float4 aux_of(const GpuBvh& g, uint32_t j, const Tri& t) {
  if (!(t.nn > 0.0f)) return make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  const float len = sqrtf(t.nn);
  return make_float4(t.n[0] / len, t.n[1] / len, t.n[2] / len, __uint_as_float((uint32_t)g.M[j]));
}

// leaf record of triangle `orig`: first vertex and id, the two edges.  A
// triangle that a refit made degenerate keeps zero edges, so the ray test's
// determinant is exactly zero and it is never hit (a build leaves it out).
__device__ __forceinline__ void store_tri(float4* rec, uint32_t orig, const Tri& t) {
  const float k = t.nn > 0.0f ? 1.0f : 0.0f;
  rec[0] = make_float4(t.p0[0], t.p0[1], t.p0[2], __uint_as_float(orig));
  rec[1] = make_float4(k * t.e1[0], k * t.e1[1], k * t.e1[2], 0.0f);
  rec[2] = make_float4(k * t.e2[0], k * t.e2[1], k * t.e2[2], 0.0f);
}

__global__ void k_init_misc(uint32_t* misc, bool refit) {
  const uint32_t i = threadIdx.x;
  if (i >= (uint32_t)kMiscWords) return;
  if (refit) {
    if (i == 6) misc[i] = __float_as_uint(1.0f);
    return;
  }
  misc[i] = i < 3 ? 0xffffffffu : (i == 6 ? __float_as_uint(1.0f) : 0u);
}

// per triangle: normal record, hittable count, centroid (into `cen`),
// centroid bounds and the largest coordinate magnitude (block-reduced)
__global__ void __launch_bounds__(kB) k_prep(GpuBvh g, float4* aux, float4* cen, bool build) {
  __shared__ uint32_t s_lo[3], s_hi[3], s_mag, s_cnt;
  if (threadIdx.x < 3) {
    s_lo[threadIdx.x] = 0xffffffffu;
    s_hi[threadIdx.x] = 0u;
  }
  if (threadIdx.x == 0) {
    s_mag = __float_as_uint(1.0f);
    s_cnt = 0;
  }
  __syncthreads();
  const uint32_t j = blockIdx.x * kB + threadIdx.x;
  if (j < g.nt) {
    Tri t;
    load_tri(g, j, t);
    aux[j] = aux_of(g, j, t);
    const bool ok = t.nn > 0.0f;
    if (ok) {
      float lo[3], hi[3], mag = 1.0f;
      tri_box(t, lo, hi);
      float c[3];
      for (int k = 0; k < 3; ++k) {
        c[k] = 0.5f * (lo[k] + hi[k]);
        mag = fmaxf(mag, fmaxf(fabsf(lo[k]), fabsf(hi[k])));
      }
      atomicMax(&s_mag, __float_as_uint(mag));  // positive floats order as their bits
      if (build) {
        cen[j] = make_float4(c[0], c[1], c[2], 1.0f);
        for (int k = 0; k < 3; ++k) {
          atomicMin(&s_lo[k], fenc(c[k]));
          atomicMax(&s_hi[k], fenc(c[k]));
        }
        atomicAdd(&s_cnt, 1u);
      }
    } else if (build) {
      cen[j] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicMax(g.misc + 6, s_mag);
    if (build) {
      for (int k = 0; k < 3; ++k) {
        atomicMin(g.misc + k, s_lo[k]);
        atomicMax(g.misc + 3 + k, s_hi[k]);
      }
      atomicAdd(g.misc + 7, s_cnt);
    }
  }
}

__device__ __forceinline__ uint32_t spread10(uint32_t x) {
  x = (x * 0x00010001u) & 0xFF0000FFu;
  x = (x * 0x00000101u) & 0x0F00F00Fu;
  x = (x * 0x00000011u) & 0xC30C30C3u;
  x = (x * 0x00000005u) & 0x49249249u;
  return x;
}

// 30-bit Morton key of the centroid in the centroid bounds; unhittable
// triangles get a key above every valid one and sort last
__global__ void __launch_bounds__(kB) k_morton(GpuBvh g, const float4* cen) {
  const uint32_t j = blockIdx.x * kB + threadIdx.x;
  if (j >= g.nt) return;
  const float4 c = cen[j];
  uint32_t key = 0xffffffffu;
  if (c.w > 0.0f) {
    const float cc[3] = {c.x, c.y, c.z};
    uint32_t q[3];
    for (int k = 0; k < 3; ++k) {
      const float lo = fdec(g.misc[k]), hi = fdec(g.misc[3 + k]);
      const float ext = hi - lo;
      float u = ext > 0.0f ? (cc[k] - lo) / ext * 1024.0f : 0.0f;
      u = fminf(fmaxf(u, 0.0f), 1023.0f);
      q[k] = (uint32_t)u;
    }
    key = (spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]);
  }
  g.keys[j] = key;
  g.ids[j] = j;
}

// common-prefix length of sorted keys a and b (index bits break ties)
__device__ __forceinline__ int delta(const uint32_t* key, int m, int a, int b) {
  if (b < 0 || b >= m) return -1;
  const uint32_t ka = key[a], kb = key[b];
  if (ka == kb) return 32 + __clz((uint32_t)(a ^ b));
  return __clz(ka ^ kb);
}

// inner node i of the binary radix tree: its key range and split
__global__ void __launch_bounds__(kB) k_internal(GpuBvh g) {
  const int m = (int)g.misc[7];
  const int i = (int)(blockIdx.x * kB + threadIdx.x);
  if (i >= m - 1) return;
  const uint32_t* key = g.keys + g.nt;  // sorted keys
  const int d = (delta(key, m, i, i + 1) - delta(key, m, i, i - 1)) >= 0 ? 1 : -1;
  const int dmin = delta(key, m, i, i - d);
  int lmax = 2;
  while (delta(key, m, i, i + lmax * d) > dmin) lmax *= 2;
  int l = 0;
  for (int t = lmax / 2; t >= 1; t /= 2)
    if (delta(key, m, i, i + (l + t) * d) > dmin) l += t;
  const int j = i + l * d;
  const int dnode = delta(key, m, i, j);
  int s = 0;
  for (int t = (l + 1) / 2; t >= 1; t = t == 1 ? 0 : (t + 1) / 2)
    if (delta(key, m, i, i + (s + t) * d) > dnode) s += t;
  const int split = i + s * d + (d < 0 ? -1 : 0);
  const int first = min(i, j), last = max(i, j);
  const int left = first == split ? ~split : split;
  const int right = last == split + 1 ? ~(split + 1) : split + 1;
  g.child[2 * i + 0] = left;
  g.child[2 * i + 1] = right;
  g.range[2 * i + 0] = (uint32_t)first;
  g.range[2 * i + 1] = (uint32_t)last;
  g.parent[left >= 0 ? left : (m - 1) + ~left] = i;
  g.parent[right >= 0 ? right : (m - 1) + ~right] = i;
  if (i == 0) g.parent[0] = -1;
}

// per sorted position: the leaf-order triangle and its box
__global__ void __launch_bounds__(kB) k_leaves(GpuBvh g, float4* tris) {
  const int m = (int)g.misc[7];
  const int p = (int)(blockIdx.x * kB + threadIdx.x);
  if (p >= m) return;
  const uint32_t orig = g.sorted[p];
  Tri t;
  load_tri(g, orig, t);
  store_tri(tris + 3 * p, orig, t);
  float lo[3], hi[3];
  tri_box(t, lo, hi);
  float* b = g.box + 6u * (uint32_t)((m - 1) + p);
  for (int k = 0; k < 3; ++k) {
    b[k] = lo[k];
    b[3 + k] = hi[k];
  }
}

// boxes of the inner nodes of one depth from their children (one launch per
// depth, deepest first, so the children are complete without any fence)
__global__ void __launch_bounds__(kB) k_box_level(GpuBvh g, uint32_t first, uint32_t count) {
  const uint32_t k = blockIdx.x * kB + threadIdx.x;
  if (k >= count) return;
  const int m = (int)g.misc[7];
  const int node = (int)g.order[first + k];
  const int l = g.child[2 * node], r = g.child[2 * node + 1];
  const float* bl = g.box + 6u * (uint32_t)(l >= 0 ? l : (m - 1) + ~l);
  const float* br = g.box + 6u * (uint32_t)(r >= 0 ? r : (m - 1) + ~r);
  float* bn = g.box + 6u * (uint32_t)node;
  for (int a = 0; a < 3; ++a) {
    bn[a] = fminf(bl[a], br[a]);
    bn[3 + a] = fmaxf(bl[3 + a], br[3 + a]);
  }
}

// inner nodes into depth buckets (positions from the host's prefix sums):
// ranks within the workgroup from LDS, one global reservation per
// workgroup and depth
__global__ void __launch_bounds__(kB) k_scatter(GpuBvh g) {
  __shared__ uint32_t s_cnt[kMaxTreeDepth], s_base[kMaxTreeDepth];
  for (uint32_t d = threadIdx.x; d < kMaxTreeDepth; d += kB) s_cnt[d] = 0u;
  __syncthreads();
  const int m = (int)g.misc[7];
  const int i = (int)(blockIdx.x * kB + threadIdx.x);
  const bool live = i < m - 1;
  const uint32_t d = live ? g.depth[i] : 0u;
  const uint32_t rank = live ? atomicAdd(&s_cnt[d], 1u) : 0u;
  __syncthreads();
  for (uint32_t e = threadIdx.x; e < kMaxTreeDepth; e += kB)
    s_base[e] = s_cnt[e] ? atomicAdd(g.level + kMaxTreeDepth + e, s_cnt[e]) : 0u;
  __syncthreads();
  if (live) g.order[s_base[d] + rank] = (uint32_t)i;
}

// four-wide nodes sit at even binary depths; a subtree of at most max_leaf
// triangles is a leaf and is not opened
// (the per-depth counts are summed in LDS first: one global atomic per
// workgroup and depth instead of one per node on a few dozen addresses)
__global__ void __launch_bounds__(kB) k_heads(GpuBvh g) {
  __shared__ uint32_t s_cnt[kMaxTreeDepth];
  for (uint32_t d = threadIdx.x; d < kMaxTreeDepth; d += kB) s_cnt[d] = 0u;
  __syncthreads();
  const int m = (int)g.misc[7];
  const int i = (int)(blockIdx.x * kB + threadIdx.x);
  uint32_t is_head = 0;
  if (i < m - 1) {
    int depth = 0;
    for (int n = g.parent[i]; n >= 0 && depth < (int)kMaxTreeDepth - 1; n = g.parent[n]) ++depth;
    g.depth[i] = (uint32_t)depth;
    atomicAdd(&s_cnt[depth], 1u);
    const uint32_t count = g.range[2 * i + 1] - g.range[2 * i] + 1u;
    is_head = (i == 0 || ((depth & 1) == 0 && count > g.max_leaf)) ? 1u : 0u;
    atomicMax(g.misc + 11, (uint32_t)depth);
    if (is_head) atomicMax(g.misc + 10, (uint32_t)depth / 2u);
  }
  if (i < (int)g.nt) g.flag[i] = is_head;
  __syncthreads();
  for (uint32_t d = threadIdx.x; d < kMaxTreeDepth; d += kB)
    if (s_cnt[d]) atomicAdd(g.level + d, s_cnt[d]);
}

__global__ void __launch_bounds__(kB) k_head_index(GpuBvh g, const uint32_t* scanned) {
  const int m = (int)g.misc[7];
  const int i = (int)(blockIdx.x * kB + threadIdx.x);
  if (i >= m - 1) return;
  g.head[i] = g.flag[i] ? (int32_t)scanned[i] : -1;
  if (i == m - 2) g.misc[8] = scanned[i] + g.flag[i];
}

// the host build's node frame: origin at the low corner, the smallest power
// of two step with the extent within 255 steps
__device__ __forceinline__ void quantise_axis(float lo, float hi, float& origin, uint32_t& ebyte) {
  origin = lo;
  const double ext = (double)hi - (double)lo;
  int e = 0;  // a node with no box at all keeps step 1 (see the host build)
  if (ext > 0.0) {
    frexp(ext / 255.0, &e);
    while (e > -126 && ext <= 255.0 * ldexp(1.0, e - 1)) --e;
    while (ext > 255.0 * ldexp(1.0, e)) ++e;
    e = max(e, -126);
  }
  ebyte = (uint32_t)(e + 127);
}

struct Kid {
  int32_t ref;
  float lo[3], hi[3];
  bool empty;
};

__device__ void write_node(Node4* out, const Kid* kids, int n_kids, float pad) {
  float clo[4][3], chi[4][3];
  float nlo[3] = {INFINITY, INFINITY, INFINITY}, nhi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int j = 0; j < n_kids; ++j)
    for (int a = 0; a < 3; ++a) {
      clo[j][a] = kids[j].empty ? 0.0f : kids[j].lo[a] - pad;
      chi[j][a] = kids[j].empty ? 0.0f : kids[j].hi[a] + pad;
      if (!kids[j].empty) {
        nlo[a] = fminf(nlo[a], clo[j][a]);
        nhi[a] = fmaxf(nhi[a], chi[j][a]);
      }
    }
  for (int a = 0; a < 3; ++a)
    if (!(nlo[a] <= nhi[a])) nlo[a] = nhi[a] = 0.0f;
  float origin[3];
  uint32_t eb[3];
  for (int a = 0; a < 3; ++a) quantise_axis(nlo[a], nhi[a], origin[a], eb[a]);
  uint32_t qlo[3] = {0u, 0u, 0u}, qhi[3] = {0u, 0u, 0u};
  int32_t ref[4] = {kEmpty, kEmpty, kEmpty, kEmpty};
  for (int j = 0; j < n_kids; ++j) {
    for (int a = 0; a < 3; ++a) {
      const double sc = ldexp(1.0, (int)eb[a] - 127);
      const double lo = floor(((double)clo[j][a] - (double)origin[a]) / sc);
      const double hi = ceil(((double)chi[j][a] - (double)origin[a]) / sc);
      const uint32_t ql = (uint32_t)fmin(255.0, fmax(0.0, lo));
      const uint32_t qh = (uint32_t)fmin(255.0, fmax(0.0, hi));
      qlo[a] |= ql << (8 * j);
      qhi[a] |= qh << (8 * j);
    }
    ref[j] = kids[j].ref;
  }
  invert_empty_slots(ref, qlo, qhi);
  Node4 nd;
  nd.w0 = make_float4(origin[0], origin[1], origin[2], __uint_as_float(eb[0] | (eb[1] << 8) | (eb[2] << 16)));
  nd.w1 = make_uint4(qlo[0], qhi[0], qlo[1], qhi[1]);
  nd.w2 = make_uint4(qlo[2], qhi[2], 0u, 0u);
  nd.w3 = make_int4(ref[0], ref[1], ref[2], ref[3]);
  *out = nd;
}

__device__ __forceinline__ void kid_of(const GpuBvh& g, int m, int x, bool as_leaf, Kid& k) {
  const uint32_t slot = (uint32_t)(x >= 0 ? x : (m - 1) + ~x);
  const float* b = g.box + 6u * slot;
  for (int a = 0; a < 3; ++a) {
    k.lo[a] = b[a];
    k.hi[a] = b[3 + a];
  }
  k.empty = false;
  if (as_leaf) {
    const uint32_t first = x >= 0 ? g.range[2 * x] : (uint32_t)~x;
    const uint32_t last = x >= 0 ? g.range[2 * x + 1] : (uint32_t)~x;
    k.ref = leaf_ref_encode(first, last - first + 1u);
  } else {
    k.ref = g.head[x];
  }
}

__device__ __forceinline__ bool leaf_sized(const GpuBvh& g, int x) {
  return x < 0 || g.range[2 * x + 1] - g.range[2 * x] + 1u <= g.max_leaf;
}

// one four-wide node per head: its two binary children, each opened into
// its own two children unless it is a leaf
__global__ void __launch_bounds__(kB) k_emit(GpuBvh g, Node4* nodes, bool count) {
  const int m = (int)g.misc[7];
  const int i = (int)(blockIdx.x * kB + threadIdx.x);
  const float pad = __uint_as_float(g.misc[6]) * (1.0f / 262144.0f);
  if (m < 2) {
    // the root must be an inner node: at most one triangle hangs below it
    if (i == 0) {
      Kid k[2];
      int n = 0;
      if (m == 1) {
        kid_of(g, m, ~0, true, k[0]);
        n = 1;
      }
      write_node(nodes, k, n, pad);
      if (count) g.misc[9] = (uint32_t)n;
    }
    return;
  }
  if (i >= m - 1 || g.head[i] < 0) return;
  Kid kids[4];
  int n = 0;
  uint32_t leaves = 0;
  for (int s = 0; s < 2; ++s) {
    const int x = g.child[2 * i + s];
    if (leaf_sized(g, x)) {
      kid_of(g, m, x, true, kids[n++]);
      ++leaves;
    } else {
      for (int u = 0; u < 2; ++u) {
        const int y = g.child[2 * x + u];
        const bool lf = leaf_sized(g, y);
        kid_of(g, m, y, lf, kids[n++]);
        leaves += lf ? 1u : 0u;
      }
    }
  }
  write_node(nodes + g.head[i], kids, n, pad);
  if (count) atomicAdd(g.misc + 9, leaves);
}

__global__ void k_zero_u32(uint32_t* p, uint32_t n) {
  const uint32_t i = blockIdx.x * kB + threadIdx.x;
  if (i < n) p[i] = 0u;
}

inline dim3 grid_for(uint32_t n) { return dim3(n ? (n + kB - 1) / kB : 1u); }

}  // namespace

hipError_t gpu_bvh_build(GpuBvh& g, Node4* nodes, float4* tris, float4* aux, hipStream_t st) {
  const uint32_t nt = g.nt;
  hipError_t e;
#define RR_GB(x)                           \
  do {                                     \
    if ((e = (x)) != hipSuccess) return e; \
  } while (0)
  hipLaunchKernelGGL(k_init_misc, dim3(1), dim3(64), 0, st, g.misc, false);
  RR_GB(hipGetLastError());
  hipLaunchKernelGGL(k_zero_u32, grid_for(2 * kMaxTreeDepth), dim3(kB), 0, st, g.level, 2 * kMaxTreeDepth);
  RR_GB(hipGetLastError());
  float4* cen = reinterpret_cast<float4*>(g.box);  // scratch until the boxes are formed
  hipLaunchKernelGGL(k_prep, grid_for(nt), dim3(kB), 0, st, g, aux, cen, true);
  RR_GB(hipGetLastError());
  hipLaunchKernelGGL(k_morton, grid_for(nt), dim3(kB), 0, st, g, cen);
  RR_GB(hipGetLastError());
  size_t bytes = g.temp_bytes;
  RR_GB(rocprim::radix_sort_pairs(g.temp, bytes, g.keys, g.keys + nt, g.ids, g.sorted, nt, 0u, 32u, st));
  hipLaunchKernelGGL(k_internal, grid_for(nt), dim3(kB), 0, st, g);
  RR_GB(hipGetLastError());
  hipLaunchKernelGGL(k_heads, grid_for(nt), dim3(kB), 0, st, g);
  RR_GB(hipGetLastError());
  // node index of each head: exclusive scan of the head flags into the
  // first half of the key array (free after the sort)
  bytes = g.temp_bytes;
  RR_GB(rocprim::exclusive_scan(g.temp, bytes, g.flag, g.keys, 0u, (size_t)nt, rocprim::plus<uint32_t>(), st));
  hipLaunchKernelGGL(k_head_index, grid_for(nt), dim3(kB), 0, st, g, g.keys);
  RR_GB(hipGetLastError());
  // depth buckets: counts to the host, prefix sums back as scatter cursors
  uint32_t h[kMiscWords];
  std::vector<uint32_t> cnt(kMaxTreeDepth), off(kMaxTreeDepth);
  RR_GB(hipMemcpyAsync(h, g.misc, sizeof h, hipMemcpyDeviceToHost, st));
  RR_GB(hipMemcpyAsync(cnt.data(), g.level, 4 * kMaxTreeDepth, hipMemcpyDeviceToHost, st));
  RR_GB(hipStreamSynchronize(st));
  uint32_t acc = 0;
  for (uint32_t d = 0; d < kMaxTreeDepth; ++d) {
    off[d] = acc;
    acc += cnt[d];
  }
  RR_GB(hipMemcpyAsync(g.level + kMaxTreeDepth, off.data(), 4 * kMaxTreeDepth, hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_scatter, grid_for(nt), dim3(kB), 0, st, g);
  RR_GB(hipGetLastError());
  g.level_cnt = cnt;
  g.level_off = off;
  RR_GB(gpu_bvh_refit(g, nodes, tris, aux, st, false));
  RR_GB(hipMemcpyAsync(h, g.misc, sizeof h, hipMemcpyDeviceToHost, st));
  RR_GB(hipStreamSynchronize(st));
  g.m = h[7];
  g.n_nodes = g.m >= 2 ? h[8] : 1u;
  g.n_leaves = h[9];
  g.max_depth = g.m >= 2 ? h[10] : 0u;
  // a node pushes at most three of its children; the path to the deepest
  // node has max_depth + 1 nodes
  g.max_stack = 3u * (g.max_depth + 1u);
  g.pad = __builtin_bit_cast(float, h[6]) * (1.0f / 262144.0f);
  return hipSuccess;
}

hipError_t gpu_bvh_refit(GpuBvh& g, Node4* nodes, float4* tris, float4* aux, hipStream_t st, bool refit) {
  const uint32_t nt = g.nt;
  hipError_t e;
  if (refit) {
    hipLaunchKernelGGL(k_init_misc, dim3(1), dim3(64), 0, st, g.misc, true);
    RR_GB(hipGetLastError());
    hipLaunchKernelGGL(k_prep, grid_for(nt), dim3(kB), 0, st, g, aux, nullptr, false);
    RR_GB(hipGetLastError());
  }
  hipLaunchKernelGGL(k_leaves, grid_for(nt), dim3(kB), 0, st, g, tris);
  RR_GB(hipGetLastError());
  for (int d = (int)g.level_cnt.size() - 1; d >= 0; --d) {
    const uint32_t c = g.level_cnt[(size_t)d];
    if (!c) continue;
    hipLaunchKernelGGL(k_box_level, grid_for(c), dim3(kB), 0, st, g, g.level_off[(size_t)d], c);
    RR_GB(hipGetLastError());
  }
  hipLaunchKernelGGL(k_emit, grid_for(nt), dim3(kB), 0, st, g, nodes, !refit);
  RR_GB(hipGetLastError());
#undef RR_GB
  return hipSuccess;
}

// ---------------------------------------------------------------- refit of a host-built tree
namespace {

// leaf-order triangle li: vertex and edges from the moved vertices of its
// original triangle (the original id stays in the first word's w)
__global__ void __launch_bounds__(kB) k_hr_tris(GpuBvh g, float4* tris, uint32_t n) {
  const uint32_t li = blockIdx.x * kB + threadIdx.x;
  if (li >= n) return;
  const uint32_t orig = __float_as_uint(tris[3u * li].w);
  if (orig >= g.nt) return;
  Tri t;
  load_tri(g, orig, t);
  store_tri(tris + 3u * li, orig, t);
}

// the nodes of one depth: child boxes (inner children from the deeper level
// just refitted, leaves from their triangles), the quantised node and its
// own box for its parent.  All four slots are rewritten; a slot without a
// child gets the inverted box, as in the builds, so a refit with unmoved
// vertices rewrites every byte as built.
__global__ void __launch_bounds__(kB) k_hr_level(GpuBvh g, Node4* nodes, const float4* tris, float* nbox,
                                                 const uint32_t* order, uint32_t first, uint32_t count,
                                                 uint32_t n_nodes, uint32_t n_leaf_tris) {
  const uint32_t k = blockIdx.x * kB + threadIdx.x;
  if (k >= count) return;
  const uint32_t id = order[first + k];
  if (id >= n_nodes) return;
  const float pad = __uint_as_float(g.misc[6]) * (1.0f / 262144.0f);
  const Node4 nd = nodes[id];
  const int32_t refs[4] = {nd.w3.x, nd.w3.y, nd.w3.z, nd.w3.w};
  Kid kids[4];
  const int n_kids = 4;
  float nlo[3] = {INFINITY, INFINITY, INFINITY}, nhi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int j = 0; j < 4; ++j) {
    Kid& kd = kids[j];
    kd.ref = refs[j];
    kd.empty = true;
    for (int a = 0; a < 3; ++a) {
      kd.lo[a] = INFINITY;
      kd.hi[a] = -INFINITY;
    }
    if (refs[j] == kEmpty) continue;
    if (refs[j] >= 0) {
      if ((uint32_t)refs[j] < n_nodes) {
        const float* b = nbox + 6u * (uint32_t)refs[j];
        for (int a = 0; a < 3; ++a) {
          kd.lo[a] = b[a];
          kd.hi[a] = b[3 + a];
        }
      }
    } else {
      const uint32_t start = leaf_start(refs[j]), cnt = leaf_count(refs[j]);
      for (uint32_t u = 0; u < cnt; ++u) {
        const uint32_t li = start + u;
        if (li >= n_leaf_tris) break;
        const uint32_t orig = __float_as_uint(tris[3u * li].w);
        if (orig >= g.nt) continue;
        Tri t;
        load_tri(g, orig, t);
        float lo[3], hi[3];
        tri_box(t, lo, hi);
        for (int a = 0; a < 3; ++a) {
          kd.lo[a] = fminf(kd.lo[a], lo[a]);
          kd.hi[a] = fmaxf(kd.hi[a], hi[a]);
        }
      }
    }
    kd.empty = !(kd.lo[0] <= kd.hi[0] && kd.lo[1] <= kd.hi[1] && kd.lo[2] <= kd.hi[2]);
    if (!kd.empty)
      for (int a = 0; a < 3; ++a) {
        nlo[a] = fminf(nlo[a], kd.lo[a]);
        nhi[a] = fmaxf(nhi[a], kd.hi[a]);
      }
  }
  write_node(nodes + id, kids, n_kids, pad);
  for (int a = 0; a < 3; ++a) {
    nbox[6u * id + (uint32_t)a] = nlo[a];
    nbox[6u * id + 3u + (uint32_t)a] = nhi[a];
  }
}

}  // namespace

hipError_t host_refit_setup(HostRefit& r, const Node4* nodes, uint32_t n_nodes, uint32_t n_leaf_tris,
                            const uint32_t* F, const uint16_t* M, uint32_t nt) {
  hipError_t e;
  host_refit_free(r);
  r.nt = nt;
  r.n_nodes = n_nodes;
  r.n_leaf_tris = n_leaf_tris;
  // depth of every node from the root (children are emitted after parents)
  std::vector<uint32_t> depth(n_nodes, 0u);
  uint32_t max_d = 0;
  for (uint32_t i = 0; i < n_nodes; ++i) {
    const int32_t refs[4] = {nodes[i].w3.x, nodes[i].w3.y, nodes[i].w3.z, nodes[i].w3.w};
    for (int j = 0; j < 4; ++j) {
      if (refs[j] == kEmpty || refs[j] < 0) continue;
      if ((uint32_t)refs[j] >= n_nodes || (uint32_t)refs[j] <= i) return hipErrorInvalidValue;
      depth[(uint32_t)refs[j]] = depth[i] + 1u;
      max_d = std::max(max_d, depth[i] + 1u);
    }
  }
  r.level_cnt.assign(max_d + 1u, 0u);
  r.level_off.assign(max_d + 1u, 0u);
  for (uint32_t i = 0; i < n_nodes; ++i) ++r.level_cnt[depth[i]];
  for (uint32_t d = 1; d <= max_d; ++d) r.level_off[d] = r.level_off[d - 1] + r.level_cnt[d - 1];
  std::vector<uint32_t> order(std::max<uint32_t>(n_nodes, 1u)), cur = r.level_off;
  for (uint32_t i = 0; i < n_nodes; ++i) order[cur[depth[i]]++] = i;
  if ((e = hipMalloc(&r.F, 12 * (size_t)std::max<uint32_t>(nt, 1u))) != hipSuccess) return e;
  if ((e = hipMalloc(&r.M, 2 * (size_t)std::max<uint32_t>(nt, 1u))) != hipSuccess) return e;
  if ((e = hipMalloc(&r.order, 4 * order.size())) != hipSuccess) return e;
  if ((e = hipMalloc(&r.nbox, 24 * (size_t)std::max<uint32_t>(n_nodes, 1u))) != hipSuccess) return e;
  if ((e = hipMalloc(&r.misc, 4 * (size_t)kMiscWords)) != hipSuccess) return e;
  if (nt) {
    if ((e = hipMemcpy(r.F, F, 12 * (size_t)nt, hipMemcpyHostToDevice)) != hipSuccess) return e;
    if ((e = hipMemcpy(r.M, M, 2 * (size_t)nt, hipMemcpyHostToDevice)) != hipSuccess) return e;
  }
  return hipMemcpy(r.order, order.data(), 4 * order.size(), hipMemcpyHostToDevice);
}

hipError_t host_refit(HostRefit& r, const float* V, uint32_t nv, Node4* nodes, float4* tris, float4* aux,
                      hipStream_t st) {
  GpuBvh g;  // a view: the mesh and the scalars only
  g.nv = nv;
  g.nt = r.nt;
  g.V = const_cast<float*>(V);
  g.F = r.F;
  g.M = r.M;
  g.misc = r.misc;
  hipError_t e;
  hipLaunchKernelGGL(k_init_misc, dim3(1), dim3(64), 0, st, r.misc, true);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_prep, grid_for(r.nt), dim3(kB), 0, st, g, aux, nullptr, false);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_hr_tris, grid_for(r.n_leaf_tris), dim3(kB), 0, st, g, tris, r.n_leaf_tris);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  for (int d = (int)r.level_cnt.size() - 1; d >= 0; --d) {
    const uint32_t c = r.level_cnt[(size_t)d];
    if (!c) continue;
    hipLaunchKernelGGL(k_hr_level, grid_for(c), dim3(kB), 0, st, g, nodes, tris, r.nbox, r.order,
                       r.level_off[(size_t)d], c, r.n_nodes, r.n_leaf_tris);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

void host_refit_free(HostRefit& r) {
  if (r.F) (void)hipFree(r.F);
  if (r.M) (void)hipFree(r.M);
  if (r.order) (void)hipFree(r.order);
  if (r.nbox) (void)hipFree(r.nbox);
  if (r.misc) (void)hipFree(r.misc);
  r.F = nullptr;
  r.M = nullptr;
  r.order = nullptr;
  r.nbox = nullptr;
  r.misc = nullptr;
}

hipError_t rocprim_sizes(size_t n, size_t* sort_bytes, size_t* scan_bytes) {
  hipError_t e = rocprim::radix_sort_pairs(nullptr, *sort_bytes, (uint32_t*)nullptr, (uint32_t*)nullptr,
                                           (uint32_t*)nullptr, (uint32_t*)nullptr, n, 0u, 32u);
  if (e != hipSuccess) return e;
  return rocprim::exclusive_scan(nullptr, *scan_bytes, (uint32_t*)nullptr, (uint32_t*)nullptr, 0u, n,
                                 rocprim::plus<uint32_t>());
}

void gpu_bvh_free(GpuBvh& g) {
  void* ptrs[] = {g.V, g.F, g.M, g.sorted, g.child, g.parent, g.range, g.head, g.box, g.flag, g.misc, g.temp,
                  g.keys, g.ids, g.depth, g.order, g.level};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  g = GpuBvh();
}

}  // namespace rr
