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

struct ShadowView {
  float4* a;
  float4* b;
  uint4* c;
};

// Arguments shared by the per-level kernels.
struct LevelArgs {
  const Node4* nodes;   // four-wide tree, or
  const Node8* nodes8;  // eight-wide tree (exactly one is set)
  uint32_t n_nodes;  // inner nodes (bounds the node visits of one ray)
  uint32_t depth;
  uint32_t levels;  // bounce levels of the launch: the largest max_b of its scans
  const float4* tris;
  const float4* aux;
  const DevScan* scans;
  uint32_t n_scans;
  uint32_t cap;       // capacity of each of the two ray queues and of the hit buffer
  const DevMaterial* mats;
  unsigned long long* acc;
  QueueView in, out;  // rays of this level / children appended for the next
  uint2* hits;        // per ray of this level: (t bits, original triangle id or -1)
  uint32_t n_first;   // primaries of every scan (raygen work items)
  uint32_t masked;    // some scan has a primary mask: raygen compacts with atomics
  uint32_t refill;    // trace: refill a wave once this many lanes are idle
  uint32_t pool;      // trace: rays a wave claims per atomic
  uint32_t tri_batch;   // trace: queued leaves that start a triangle phase (1..64)
  int32_t* spill;     // trace: stack entries beyond kStack, kSpill per lane (lane-major)
  float4* wq;         // fused scan: per-wave child pool and hit ring (4 float4 per entry)
  uint32_t wq_pool;   // fused scan: child-pool entries per wave
  uint32_t wq_hits;   // fused scan: hit-ring entries per wave (power of two, >= 128)
  uint32_t shade_batch;  // fused scan: finished rays that start a shade phase (1..64)
  uint32_t* counters;
  unsigned long long* prof;  // non-null: counting variants (nodes, triangles, rays, hits)
  uint32_t air;         // some scan returns along the air path: shade emits visibility rays
  ShadowView shq;       // visibility rays of every level, traced after the last one
  uint32_t shq_cap;     // their capacity
  int32_t* air_rec;     // air-path outcome records of the one scan that has records, or null
};

// Copies `bytes` (multiple of 4) from host memory into device memory by
// kernel arguments, in chunks; stream-ordered and safe to reuse `src` on
// return.
hipError_t put_blob(void* dst_dev, const void* src, size_t bytes, hipStream_t st);

hipError_t launch_clear(unsigned long long* acc, size_t n_acc, uint32_t* counters, uint32_t count0,
                        hipStream_t st);
hipError_t launch_fill_i32(int32_t* p, size_t n, int32_t v, hipStream_t st);
// `threads` (a multiple of 256) lanes, each reading 16 B per step from a
// hashed 64-byte row of `buf` (n_rows rows); one float per lane to `out`.
hipError_t launch_gather(const float4* buf, uint32_t n_rows, uint32_t steps, float* out, uint32_t threads,
                         hipStream_t st);
hipError_t launch_raygen(const LevelArgs& a, uint32_t grid, hipStream_t st);
hipError_t launch_trace(const LevelArgs& a, uint32_t grid, bool help, hipStream_t st);
hipError_t launch_shade(const LevelArgs& a, uint32_t grid, hipStream_t st);
// Visibility of the sensor for the air-path returns of every level (the
// closest-hit traversal bounded by each ray's distance to the sensor); the
// unblocked returns are added to the accumulator.  a.depth must be 0.
hipError_t launch_shadow(const LevelArgs& a, uint32_t grid, bool help, hipStream_t st);
// All bounce levels in one persistent launch (primaries from queue `in`).
hipError_t launch_scan(const LevelArgs& a, uint32_t grid, hipStream_t st);
hipError_t launch_finalize(const DevScan* scans, uint32_t n_scans, const unsigned long long* acc,
                           uint32_t max_cells, hipStream_t st);

// profile counter block (u64): [0] node visits, [1] triangle tests, [2] rays,
// [3] hits, then per bounce level: wave iterations, active lanes, and the
// same two after the level's queue ran dry, and the most loop iterations
// any one ray took
constexpr int kProfIters = 4;
constexpr int kProfActive = kProfIters + 8;
constexpr int kProfTailIters = kProfActive + 8;
constexpr int kProfTailActive = kProfTailIters + 8;
constexpr int kProfMaxVisits = kProfTailActive + 8;
constexpr int kProfPoolMax = kProfMaxVisits + 8;  // fused scan: largest child pool of a wave
constexpr int kProfWords = kProfPoolMax + 1;
constexpr int kBlock = 256;
// shade: lanes per block (one queue reservation per block step); the air-path
// variant holds twice the registers and keeps two blocks per CU with 256
constexpr int kShadeBlock = 512;
constexpr int kShadeBlockAir = 256;
constexpr int shade_block(bool air) { return air ? kShadeBlockAir : kShadeBlock; }
constexpr uint32_t kMaxLevels = 8;   // bounce levels (interactions per path) at most
constexpr uint32_t kLeafRing = 256;  // four-wide trace: leaf entries per wave (power of two)
// a node step appends up to four leaves per lane and runs only while they fit
static_assert(kLeafRing >= 4u * 64u && (kLeafRing & (kLeafRing - 1u)) == 0u, "leaf ring size");
constexpr uint32_t kNodeSteps = 6;   // four-wide trace: node steps per refill/triangle decision at most
constexpr uint32_t kLeafRing8 = 1024;  // eight-wide trace: leaf entries per wave (power of two)
constexpr int kStack8 = 6;              // eight-wide trace: node groups per lane in LDS
constexpr int kTraceBlock = 128;  // trace workgroup (LDS stack of kStack words per lane)

}  // namespace rr
