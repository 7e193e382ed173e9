// kernels.h -- host-side launch interface of the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "rr_internal.h"

namespace rr {

struct QueueView {
  float4* a;
  float4* b;
  uint4* c;
  uint32_t* m;
};

struct BounceArgs {
  const Node* nodes;
  uint32_t n_nodes;  // inner nodes (bounds the traversal loop)
  const float4* tris;
  const float4* aux;
  const DevScan* scans;
  uint32_t n_scans;
  uint32_t depth;
  const DevMaterial* mats;
  unsigned long long* acc;
  QueueView in, out;
  uint32_t out_cap;  // capacity of each of the two queues
  uint32_t n_first;  // rays of the first level (primaries of every scan)
  uint32_t* counters;
  unsigned long long* prof;  // non-null: counting kernel (node visits, triangle tests, rays)
};

// Copies `bytes` (multiple of 4) from host memory into device memory by
// kernel arguments, in chunks; stream-ordered and safe to reuse `src` on
// return.
hipError_t put_blob(void* dst_dev, const void* src, size_t bytes, hipStream_t st);

hipError_t launch_clear(unsigned long long* acc, size_t n_acc, uint32_t* counters, uint32_t n_first,
                        hipStream_t st);
hipError_t launch_fill_i32(int32_t* p, size_t n, int32_t v, hipStream_t st);
hipError_t launch_bounce(const BounceArgs& a, uint32_t grid, hipStream_t st);
hipError_t launch_finalize(const DevScan* scans, uint32_t n_scans, const unsigned long long* acc,
                           uint32_t max_cells, hipStream_t st);

constexpr int kBlock = 256;

}  // namespace rr
