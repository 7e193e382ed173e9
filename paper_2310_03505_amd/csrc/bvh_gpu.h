// bvh_gpu.h -- BVH build and refit on the GPU (linear BVH, four-wide
// quantised output in the format the traversal kernels read).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "rr_internal.h"

namespace rr {

constexpr uint32_t kMaxTreeDepth = 128;  // binary depth bound (30-bit keys + index bits)

// Device state of a GPU-built tree, kept for refits (same triangles, moved
// vertices).  m = hittable (non-degenerate) triangles; the binary radix tree
// has m - 1 inner nodes over the m Morton-sorted triangles.
struct GpuBvh {
  uint32_t nv = 0, nt = 0, m = 0, max_leaf = 2;
  float* V = nullptr;          // [nv][3] vertices
  uint32_t* F = nullptr;       // [nt][3]
  uint16_t* M = nullptr;       // [nt] material ids
  uint32_t* sorted = nullptr;  // [nt] original triangle per sorted position (first m hittable)
  int32_t* child = nullptr;    // [m - 1][2] inner index, or ~position for a single triangle
  int32_t* parent = nullptr;   // [m - 1 + m] parent inner node of inner i, then of position p
  uint32_t* range = nullptr;   // [m - 1][2] first and last sorted position under inner i
  int32_t* head = nullptr;     // [m - 1] four-wide node index of inner i, or -1
  float* box = nullptr;        // [m - 1 + m][6] boxes of inner nodes, then of single triangles
  uint32_t* flag = nullptr;    // [nt] head flags during the build
  uint32_t* depth = nullptr;   // [m - 1] depth of inner i (root 0)
  uint32_t* order = nullptr;   // [m - 1] inner nodes grouped by depth
  uint32_t* level = nullptr;   // [2][kMaxTreeDepth] nodes per depth, then scatter cursors
  std::vector<uint32_t> level_off, level_cnt;  // host copies: where each depth's nodes start
  uint32_t* misc = nullptr;    // scalars (bounds, counts), see bvh_gpu.hip
  void* temp = nullptr;        // sort / scan scratch
  size_t temp_bytes = 0;
  uint32_t* keys = nullptr;    // [2][nt] Morton keys (sort in / out)
  uint32_t* ids = nullptr;     // [nt] sort values in
  uint32_t n_nodes = 0, n_leaves = 0, max_depth = 0, max_stack = 0;
  float pad = 0.0f;
};

// Builds a tree over V (device, nv x 3) / F / M (device copies held by g):
// fills g and the output arrays nodes[max(1, m - 1)], tris[3 max(1, m)],
// aux[max(1, nt)] (allocated by the caller with these sizes).  Waits for the
// stream at the end (it reads back the counts).
hipError_t gpu_bvh_build(GpuBvh& g, Node4* nodes, float4* tris, float4* aux, hipStream_t st);

// Recomputes triangles, normals, boxes and node frames of the existing tree
// from g.V (updated by the caller): the leaves, then one launch per depth,
// deepest first, then the four-wide nodes; stream-ordered, no allocation.
// (refit = false: the tail of a build, normals already written.)
hipError_t gpu_bvh_refit(GpuBvh& g, Node4* nodes, float4* tris, float4* aux, hipStream_t st, bool refit = true);

void gpu_bvh_free(GpuBvh& g);

// Device state for refitting a four-wide tree built on the host: its nodes
// and the order of its leaf triangles stay, moved vertices give new
// triangles, normals, child boxes and node frames.  Holds the mesh's indices
// and materials and the nodes grouped by depth (set up once per tree).
struct HostRefit {
  uint32_t nt = 0, n_nodes = 0, n_leaf_tris = 0;
  uint32_t* F = nullptr;      // [nt][3]
  uint16_t* M = nullptr;      // [nt] material ids
  uint32_t* order = nullptr;  // [n_nodes] node indices grouped by depth
  float* nbox = nullptr;      // [n_nodes][6] refitted box of each node
  uint32_t* misc = nullptr;   // [16]; [6] the largest coordinate magnitude
  std::vector<uint32_t> level_off, level_cnt;
};

// Allocates r and uploads the indices, materials and the depth order of the
// host tree `nodes` (root 0, children after their parents); synchronous.
hipError_t host_refit_setup(HostRefit& r, const Node4* nodes, uint32_t n_nodes, uint32_t n_leaf_tris,
                            const uint32_t* F, const uint16_t* M, uint32_t nt);

// Refits the tree in place from V (device, nv x 3): normals and the padding
// magnitude, the leaf triangles, then the nodes one depth at a time, deepest
// first, with the conservative quantisation of a build; stream-ordered, no
// allocation.  A refit with the build's vertices reproduces the build's
// nodes (for trees without split references).
hipError_t host_refit(HostRefit& r, const float* V, uint32_t nv, Node4* nodes, float4* tris, float4* aux,
                      hipStream_t st);

void host_refit_free(HostRefit& r);

// Scratch bytes of the sort and the scan of a build over n triangles.
hipError_t rocprim_sizes(size_t n, size_t* sort_bytes, size_t* scan_bytes);

}  // namespace rr
