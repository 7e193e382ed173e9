// bvh.h -- host BVH build over a triangle mesh and its host self-check.
#pragma once

#include <stdint.h>

#include <vector>

#include "rr_internal.h"

namespace rr {

struct BvhBuildOptions {
  uint32_t max_leaf = 2;
  uint32_t bins = 16;
  uint32_t threads = 0;
  uint32_t split_pct = 0;  // early split clipping budget, percent of the triangles
  uint32_t spatial_pct = 10;  // spatial-split budget (extra references), percent of the triangles; 0 = none
  uint32_t width = 4;      // 4: Node4 tree; 8: Node8 tree
  bool merge_leaves = true;  // binary tree to single triangles, leaves formed by the wide collapse
  uint32_t collapse = 0;     // four-wide collapse: 0 cost-optimal, 1 greedy (largest area opened first)
};

struct BuiltBvh {
  uint32_t width = 4;             // which of the two node arrays is built
  std::vector<Node4> nodes;       // four-wide inner nodes, node 0 is the root
  std::vector<Node8> nodes8;      // eight-wide inner nodes, node 0 is the root
  std::vector<float4> tris;       // 3 per leaf triangle: (v0, orig), (e1, 0), (e2, 0)
  std::vector<float4> aux;        // 1 per scene triangle, original order: (unit normal, material bits)
  uint32_t n_tris = 0;            // triangles in the scene
  uint32_t n_hittable = 0;        // non-degenerate triangles in the leaves
  uint32_t n_refs = 0;            // triangle references in the leaves (>= n_hittable)
  uint32_t n_leaves = 0;
  uint32_t max_depth = 0;         // deepest wide inner node (root = 0)
  uint32_t max_depth2 = 0;        // deepest node of the two-wide build tree
  uint32_t max_stack = 0;         // worst-case traversal stack entries
  float pad = 0.0f;               // absolute box padding
  float lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};  // scene bounds (unpadded)
  double sah_cost = 0.0;
  double build_ms = 0.0;
};

// vertices nv x 3, indices nt x 3 (validated by the caller), materials nt.
void build_bvh(const float* vertices, const uint32_t* indices, uint32_t nt,
               const uint16_t* tri_material, const BvhBuildOptions& opt, BuiltBvh& out);

// Closest hit through the hierarchy on the host (the same box test the GPU
// kernel uses).  Returns the leaf index or -1; excl is an original triangle
// id that is never hit.
int32_t host_traverse(const BuiltBvh& b, const float o[3], const float d[3], float tmax,
                      int32_t excl_leaf, float* t_out);

// Closest hit by testing every leaf triangle.
int32_t host_brute(const BuiltBvh& b, const float o[3], const float d[3], float tmax,
                   int32_t excl_leaf, float* t_out);

// Random rays through both; number of differing closest hits.
uint64_t bvh_selfcheck(const BuiltBvh& b, uint32_t n_rays, uint64_t seed);

}  // namespace rr
