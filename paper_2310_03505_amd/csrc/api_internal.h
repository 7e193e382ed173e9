// api_internal.h -- library-private state shared by api.cpp and server.cpp.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <string>
#include <vector>

#include "../../include/radarays_hip.h"
#include "bvh.h"
#include "bvh_gpu.h"
#include "kernels.h"
#include "post.h"
#include "rr_internal.h"

struct rr_context {
  int device = 0;
  int n_cu = 256;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  uint32_t* h_ctr = nullptr;  // pinned, for stats
  std::string err;
  // profiling
  uint32_t prof_flags = 0;
  struct EvPair {
    hipEvent_t a, b;
    uint32_t depth;
    int kind;  // 0 raygen, 1 trace, 2 shade, 3 air-path visibility
  };
  std::vector<hipEvent_t> ev_free;
  std::vector<EvPair> ev_used;
  unsigned long long* d_prof = nullptr;
  // tuning
  uint32_t refill_lanes = 8;
  uint32_t trace_waves_per_cu = 24;
  uint32_t pool_rays = 64;
  uint32_t tri_batch = 6;   // queued leaves that start a triangle phase
  uint32_t fused = 0;       // 1: all bounce levels in one persistent launch
  uint32_t shade_batch = 64;  // fused: finished rays that start a shade phase
  uint32_t tail_help = 12;    // rays per trace lane up to which a level uses tail helping
  size_t batch_budget = (size_t)24 << 30;  // workspace bytes per batch group
};

struct rr_scene {
  rr_context* ctx = nullptr;
  std::vector<float> V;
  std::vector<uint32_t> F;
  std::vector<uint16_t> M;
  uint32_t nv = 0, nt = 0;
  uint32_t max_mat = 0;
  bool built = false;
  rr::BuiltBvh bvh;
  void* d_nodes = nullptr;  // rr::Node4 or rr::Node8 array, as bvh.width says
  uint32_t n_nodes = 0;     // nodes in d_nodes
  rr::GpuBvh* gb = nullptr; // state of a tree built on the GPU (kept for refits)
  rr::HostRefit* hr = nullptr;  // refit state of a host-built tree (first refit on)
  bool refitted = false;        // device nodes and triangles differ from `bvh`
  float4* d_tris = nullptr;
  float4* d_aux = nullptr;
  uint64_t dev_bytes = 0;
  // graphs and servers that hold the device copies (their kernel arguments
  // or dispatcher point at them): rebuilding or releasing the scene while
  // any exists would free memory they still read
  mutable std::atomic<uint32_t> holders{0};
};


namespace rr {

#define HIP_TRY(ctx, expr)                                                                    \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return fail(ctx, e_ == hipErrorOutOfMemory ? RR_ENOMEM : RR_EDEVICE, "%s: %s", #expr,   \
                  hipGetErrorString(e_));                                                     \
  } while (0)

// lanes whose traversal stack may spill into the workspace: 256 compute
// units x 32 waves x 64 lanes
constexpr uint32_t kSpillLanes = 256u * 32u * 64u;

// Workspace layout of a set of scans (see api.cpp).
struct Layout {
  size_t off_scans = 0, off_mats = 0, off_ctr = 0, off_acc = 0, off_hits = 0, off_spill = 0, off_wq = 0;
  size_t off_shq[3] = {};  // air-path visibility rays (only when a scan has the flag)
  bool air = false;
  uint64_t shq_cap = 0;    // at most one visibility ray per hit at depth >= 1
  size_t off_q[2][4] = {};
  size_t total = 0;
  uint64_t cap = 0;       // rays per queue
  uint64_t acc_cells = 0;
  uint64_t n_first = 0;
  uint32_t max_b = 0;
  uint32_t spill_entries = 0;  // stack entries per lane in the spill area
  uint32_t spill_lanes = 0;    // lanes the spill area holds
};

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

// fused: add the per-wave child pools and hit rings of the one-launch mode.
// The spill area holds spill_entries stack entries for each of spill_lanes
// lanes; the defaults cover any tree the builders accept and any grid.
void make_layout(const rr_sensor_params* const* ps, uint32_t n, Layout& L, bool fused = false,
                 uint32_t spill_entries = kSpill, uint32_t spill_lanes = kSpillLanes);
// Persistent trace blocks of a launch at the context's tuning (the spill
// area must hold this many blocks' lanes).
uint32_t trace_grid_blocks(const rr_context* ctx);
bool tail_help_on(const rr_context* ctx, uint64_t bound, uint32_t grid_blocks);
// 32-bit spill words a lane may need beyond its LDS stack when tracing this
// scene's tree (from the build's worst-case stack need).
uint32_t scene_spill_need(const rr_scene* sc);
void make_scan(const rr_pose& pose, const rr_sensor_params& p, DevScan& s);
rr_status check_params(rr_context* ctx, const rr_sensor_params* p);
rr_status check_pose(rr_context* ctx, const rr_pose* q);
rr_status check_materials(rr_context* ctx, const rr_material* m, uint32_t n, const rr_scene* sc);
rr_status check_scene(rr_context* ctx, const rr_scene* sc);
rr_status fail(rr_context* ctx, rr_status s, const char* fmt, ...);
// Enqueues the scans on `st` using workspace `ws`; when counters_host is
// non-null the level counters are copied there (stream-ordered, no wait).
rr_status run(rr_context* ctx, const rr_scene* sc, std::vector<DevScan>& scans,
              const rr_sensor_params* const* ps, const rr_material* mats, uint32_t n_mats, char* ws,
              size_t ws_bytes, rr_scan_stats* stats, hipStream_t st, uint64_t* accum_out,
              float beam_width_for_mats, uint32_t* counters_host = nullptr,
              bool upload_tables = true, const PostArgs* post = nullptr,
              uint32_t spill_entries = kSpill);
// Validates an epilogue parameter block and fills the launch arguments
// (blur weights included); the caller sets the image pointers and sizes.
rr_status make_post_args(rr_context* ctx, const rr_post_params* p, PostArgs& a);
// Uploads the scan table (prim_base / acc_base filled) and the material
// table of a set of scans into workspace `ws`.
rr_status upload_tables(rr_context* ctx, std::vector<DevScan>& scans, const rr_sensor_params* const* ps,
                        const rr_material* mats, uint32_t n_mats, char* ws, hipStream_t st,
                        float beam_width_for_mats);
rr_status ensure_ws(rr_context* ctx, size_t bytes);
// Device address of this device's copy of the allocation-free scan's scratch
// array (noalloc.hip), looked up once per device with that device current.
rr_status scratch_setup(int device);

}  // namespace rr
