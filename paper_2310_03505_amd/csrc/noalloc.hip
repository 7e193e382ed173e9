// noalloc.hip -- rr_radar_scan_noalloc: one scan that allocates no memory.
//
// For callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc): the scan
// runs on a fixed device array, `scratch`, that the code object carries,
// instead of the context's workspace.  The kernels are those of
// rr_radar_scan; only the workspace differs, and the spill area of the
// traversal stacks is sized for the resident tree's worst-case stack need
// instead of the largest any tree may have.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <vector>

#include "api_internal.h"

using namespace rr;

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;

// One copy per device, held from the code object's load to the end of the
// process.  In host code `scratch` names a host-side stand-in: the device
// address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
std::vector<void*> g_ptr;  // per device: scratch's device address (nullptr: not set up)

}  // namespace

namespace rr {

// Looks up this device's copy of `scratch` with the device current; called
// by rr_create.  Idempotent per device.
rr_status scratch_setup(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  if ((size_t)device < g_ptr.size() && g_ptr[(size_t)device]) return RR_OK;
  DeviceGuard dg(device);
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return fail(nullptr, RR_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
  if (g_ptr.size() <= (size_t)device) g_ptr.resize((size_t)device + 1, nullptr);
  g_ptr[(size_t)device] = p;
  return RR_OK;
}

}  // namespace rr

extern "C" {

rr_status rr_scratch_bytes(size_t* bytes) {
  if (!bytes) return fail(nullptr, RR_EINVAL, "bytes is NULL");
  *bytes = kScratchBytes;
  return RR_OK;
}

rr_status rr_radar_scan_noalloc(rr_context* ctx, const rr_scene* sc, const rr_pose* pose,
                                const rr_sensor_params* params, const rr_material* mats, uint32_t n_mats,
                                float* image_dev, rr_scan_stats* stats, void* stream) {
  if (!ctx) return fail(nullptr, RR_EINVAL, "context is NULL");
  rr_status s;
  if ((s = check_scene(ctx, sc)) || (s = check_params(ctx, params)) || (s = check_pose(ctx, pose)) ||
      (s = check_materials(ctx, mats, n_mats, sc)))
    return s;
  if (!image_dev) return fail(ctx, RR_EINVAL, "image_dev is NULL");
  if (ctx->fused == 1) return fail(ctx, RR_EINVAL, "the allocation-free scan runs the level-by-level launches");
  if (sc->bvh.width == 8) return fail(ctx, RR_EINVAL, "the allocation-free scan needs a four-wide BVH");
  void* ws = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if ((size_t)ctx->device < g_ptr.size()) ws = g_ptr[(size_t)ctx->device];
  }
  if (!ws) return fail(ctx, RR_ESTATE, "scratch of device %d was not set up", ctx->device);
  const uint32_t spill = scene_spill_need(sc);
  Layout L;
  make_layout(&params, 1, L, false, spill, trace_grid_blocks(ctx) * (uint32_t)kTraceBlock);
  if (L.total > kScratchBytes)
    return fail(ctx, RR_ENOMEM, "the scan needs %zu bytes of workspace, more than the %zu-byte scratch", L.total,
                kScratchBytes);
  DeviceGuard g(ctx->device);
  std::vector<DevScan> scans(1);
  make_scan(*pose, *params, scans[0]);
  scans[0].image = image_dev;
  // no profiling events (they would be created here)
  const uint32_t prof = ctx->prof_flags;
  ctx->prof_flags = 0;
  s = run(ctx, sc, scans, &params, mats, n_mats, static_cast<char*>(ws), kScratchBytes, stats,
          static_cast<hipStream_t>(stream), nullptr, params->beam_width_rad, nullptr, true, nullptr, spill);
  ctx->prof_flags = prof;
  return s;
}

}  // extern "C"
