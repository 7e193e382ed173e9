// graph.cpp -- captured launch sequences (rr_graph_*) and the launch
// parameter autotuner (rr_autotune).
//
// A graph holds the whole per-batch sequence: clear, ray generation, one
// trace and one shade launch per bounce level, finalize.  The scan and
// material tables are the only inputs that change between replays; they are
// uploaded by a small kernel on the caller's stream right before the graph
// is launched there, so the captured nodes never change.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "api_internal.h"

using namespace rr;

struct rr_graph {
  rr_context* ctx = nullptr;
  const rr_scene* scene = nullptr;
  std::vector<rr_sensor_params> params;  // shapes the graph was captured for
  std::vector<rr_material> mats;
  std::vector<bool> masked;  // scans captured with a primary mask
  char* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool holds_scene = false;  // counted in scene->holders
};

namespace {

void graph_free(rr_graph* g) {
  if (!g) return;
  DeviceGuard dg(g->ctx->device);
  (void)hipDeviceSynchronize();
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->cap_stream) (void)hipStreamDestroy(g->cap_stream);
  if (g->ws) (void)hipFree(g->ws);
  if (g->holds_scene) g->scene->holders.fetch_sub(1);
  delete g;
}

rr_status check_descs(rr_context* ctx, const rr_scan_desc* d, uint32_t n) {
  rr_status s;
  for (uint32_t i = 0; i < n; ++i) {
    if ((s = check_params(ctx, &d[i].params)) || (s = check_pose(ctx, &d[i].pose))) return s;
    if (!d[i].image_dev) return fail(ctx, RR_EINVAL, "scan %u: image_dev is NULL", i);
    if (d[i].params.beam_width_rad != d[0].params.beam_width_rad)
      return fail(ctx, RR_EINVAL, "scans of a graph must share the beam width");
  }
  return RR_OK;
}

// Uploads the tables of `d` (n scans) into the graph's workspace on `st`.
rr_status graph_upload(rr_graph* g, const rr_scan_desc* d, hipStream_t st) {
  const uint32_t n = (uint32_t)g->params.size();
  std::vector<const rr_sensor_params*> ps(n);
  std::vector<DevScan> scans(n);
  for (uint32_t i = 0; i < n; ++i) {
    ps[i] = &d[i].params;
    make_scan(d[i].pose, d[i].params, scans[i]);
    scans[i].image = d[i].image_dev;
    scans[i].mask = d[i].primary_mask_dev;
  }
  return upload_tables(g->ctx, scans, ps.data(), g->mats.data(), (uint32_t)g->mats.size(), g->ws, st,
                       d[0].params.beam_width_rad);
}

}  // namespace

extern "C" {

rr_status rr_graph_create(rr_context* ctx, const rr_scene* sc, const rr_scan_desc* descs, uint32_t n,
                          const rr_material* mats, uint32_t n_mats, rr_graph** out) {
  if (!ctx) return fail(nullptr, RR_EINVAL, "context is NULL");
  if (!out) return fail(ctx, RR_EINVAL, "out is NULL");
  *out = nullptr;
  if (!descs || n == 0 || n > 65535) return fail(ctx, RR_EINVAL, "need 1..65535 scans");
  rr_status s;
  if ((s = check_scene(ctx, sc)) || (s = check_materials(ctx, mats, n_mats, sc)) ||
      (s = check_descs(ctx, descs, n)))
    return s;
  DeviceGuard dg(ctx->device);
  rr_graph* g = new rr_graph();
  g->ctx = ctx;
  g->scene = sc;
  sc->holders.fetch_add(1);
  g->holds_scene = true;
  g->mats.assign(mats, mats + n_mats);
  std::vector<const rr_sensor_params*> ps(n);
  std::vector<DevScan> scans(n);
  for (uint32_t i = 0; i < n; ++i) {
    g->params.push_back(descs[i].params);
    make_scan(descs[i].pose, descs[i].params, scans[i]);
    scans[i].image = descs[i].image_dev;
    scans[i].mask = descs[i].primary_mask_dev;
    g->masked.push_back(descs[i].primary_mask_dev != nullptr);
  }
  for (uint32_t i = 0; i < n; ++i) ps[i] = &g->params[i];
  Layout L;
  make_layout(ps.data(), n, L, ctx->fused != 0);
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&g->ws), L.total);
  if (e != hipSuccess) {
    graph_free(g);
    return fail(ctx, RR_ENOMEM, "graph workspace of %zu bytes: %s", L.total, hipGetErrorString(e));
  }
  g->ws_bytes = L.total;
  if ((e = hipStreamCreateWithFlags(&g->cap_stream, hipStreamNonBlocking)) != hipSuccess) {
    graph_free(g);
    return fail(ctx, RR_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
  }
  // tables of the creating scans, so a replay without new scans is valid
  if ((s = graph_upload(g, descs, g->cap_stream)) ||
      ((e = hipStreamSynchronize(g->cap_stream)) != hipSuccess &&
       (s = fail(ctx, RR_EDEVICE, "hipStreamSynchronize: %s", hipGetErrorString(e))))) {
    graph_free(g);
    return s;
  }
  // capture without per-launch events or counters
  const uint32_t prof = ctx->prof_flags;
  ctx->prof_flags = 0;
  e = hipStreamBeginCapture(g->cap_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    ctx->prof_flags = prof;
    graph_free(g);
    return fail(ctx, RR_EDEVICE, "hipStreamBeginCapture: %s", hipGetErrorString(e));
  }
  s = run(ctx, sc, scans, ps.data(), mats, n_mats, g->ws, g->ws_bytes, nullptr, g->cap_stream, nullptr,
          descs[0].params.beam_width_rad, nullptr, /*upload_tables=*/false);
  ctx->prof_flags = prof;
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(g->cap_stream, &graph);
  g->graph = graph;
  if (s) {
    graph_free(g);
    return s;
  }
  if (e != hipSuccess) {
    graph_free(g);
    return fail(ctx, RR_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
  }
  if ((e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0)) != hipSuccess) {
    graph_free(g);
    return fail(ctx, RR_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  *out = g;
  return RR_OK;
}

rr_status rr_graph_launch(rr_graph* g, const rr_scan_desc* descs, void* stream) {
  if (!g) return fail(nullptr, RR_EINVAL, "graph is NULL");
  rr_context* ctx = g->ctx;
  DeviceGuard dg(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  rr_status s;
  if (descs) {
    const uint32_t n = (uint32_t)g->params.size();
    if ((s = check_descs(ctx, descs, n))) return s;
    for (uint32_t i = 0; i < n; ++i) {
      const rr_sensor_params &a = descs[i].params, &b = g->params[i];
      if (a.n_azimuth != b.n_azimuth || a.rays_per_beam != b.rays_per_beam || a.n_bins != b.n_bins ||
          a.max_bounces != b.max_bounces || (a.flags & RR_AIR_PATH) != (b.flags & RR_AIR_PATH))
        return fail(ctx, RR_EINVAL,
                    "scan %u: azimuths, rays per beam, bins, bounces and the air-path flag must match the "
                    "captured scans", i);
      // a masked level 0 is compacted by ray generation, an unmasked one is
      // filled in place: the captured launches differ
      if ((descs[i].primary_mask_dev != nullptr) != g->masked[i])
        return fail(ctx, RR_EINVAL, "scan %u: a primary mask must be given exactly when the captured scan had one", i);
    }
    if ((s = graph_upload(g, descs, st))) return s;
  }
  HIP_TRY(ctx, hipGraphLaunch(g->exec, st));
  return RR_OK;
}

rr_status rr_graph_destroy(rr_graph* g) {
  graph_free(g);
  return RR_OK;
}

}  // extern "C"

// Coordinate descent over the trace launch parameters.  `run_once` enqueues
// the workload on `st`; each candidate is timed over `reps` runs after one
// untimed run; a parameter keeps its new value only when it beats the
// incumbent by more than 1%, and the descent stops after a pass without
// change (at most three passes).  On success the fastest tuning stays set.
template <class Run>
static rr_status tune(rr_context* ctx, hipStream_t st, uint32_t reps, bool one_launch_ok, Run&& run_once,
                      rr_tuning* best, double* best_ms) {
  rr_status s = RR_OK;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(ctx, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(ctx, RR_EDEVICE, "hipEventCreate failed");
  }
  const uint32_t prof = ctx->prof_flags;
  ctx->prof_flags = 0;
  rr_tuning cur{};
  (void)rr_get_tuning(ctx, &cur);
  const rr_tuning orig = cur;
  auto measure = [&](const rr_tuning& t, double& ms) -> rr_status {
    rr_status r = rr_set_tuning(ctx, &t);
    if (r) return r;
    for (uint32_t k = 0; k <= reps; ++k) {
      if (k == 1 && hipEventRecord(e0, st) != hipSuccess) return fail(ctx, RR_EDEVICE, "hipEventRecord failed");
      if ((r = run_once())) return r;
    }
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
      return fail(ctx, RR_EDEVICE, "event wait failed");
    float f = 0.0f;
    if (hipEventElapsedTime(&f, e0, e1) != hipSuccess) return fail(ctx, RR_EDEVICE, "hipEventElapsedTime failed");
    ms = (double)f / reps;
    return RR_OK;
  };
  static const uint32_t kRefill[] = {4, 8, 12, 16, 24, 32, 48};
  static const uint32_t kWaves[] = {8, 12, 16, 20, 24, 32};
  static const uint32_t kPool[] = {64, 128, 256};
  static const uint32_t kTriBatch[] = {4, 6, 8, 16, 32};
  static const uint32_t kFused[] = {1, 2};  // one launch per scan, one per level
  static const uint32_t kShadeBatch[] = {16, 32, 64};
  static const uint32_t kTailHelp[] = {RR_TAIL_HELP_OFF, 4, 12, 32};
  struct Axis {
    const uint32_t* v;
    size_t n;
    uint32_t rr_tuning::*f;
  } axes[] = {{kRefill, 7, &rr_tuning::refill_lanes},
              {kWaves, 6, &rr_tuning::trace_waves_per_cu},
              {kPool, 3, &rr_tuning::pool_rays},
              {kTriBatch, 5, &rr_tuning::tri_batch},
              {kFused, 2, &rr_tuning::fused},
              {kShadeBatch, 3, &rr_tuning::shade_batch},
              {kTailHelp, 4, &rr_tuning::tail_help}};
  if (!one_launch_ok && cur.fused == 1) cur.fused = 2;
  double inc = 0.0;
  s = measure(cur, inc);
  for (int pass = 0; pass < 3 && !s; ++pass) {
    bool changed = false;
    for (const Axis& ax : axes) {
      for (size_t i = 0; i < ax.n && !s; ++i) {
        if (cur.*(ax.f) == ax.v[i]) continue;
        if (ax.f == &rr_tuning::fused && ax.v[i] == 1 && !one_launch_ok) continue;
        rr_tuning t = cur;
        t.*(ax.f) = ax.v[i];
        double ms = 0.0;
        if ((s = measure(t, ms))) break;
        if (ms < inc * 0.99) {
          inc = ms;
          cur = t;
          changed = true;
        }
      }
      if (s) break;
    }
    if (!changed) break;
  }
  ctx->prof_flags = prof;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s) {
    std::string why = ctx->err;
    (void)rr_set_tuning(ctx, &orig);
    ctx->err = why;
    return s;
  }
  if ((s = rr_set_tuning(ctx, &cur))) return s;
  if (best) *best = cur;
  if (best_ms) *best_ms = inc;
  return RR_OK;
}

extern "C" {

rr_status rr_autotune(rr_context* ctx, const rr_scene* sc, const rr_pose* pose, const rr_sensor_params* params,
                      const rr_material* mats, uint32_t n_mats, float* image_dev, uint32_t reps, rr_tuning* best,
                      double* best_ms, void* stream) {
  if (!ctx) return fail(nullptr, RR_EINVAL, "context is NULL");
  if (!image_dev) return fail(ctx, RR_EINVAL, "image_dev is NULL");
  if (reps == 0 || reps > 1000) return fail(ctx, RR_EINVAL, "reps out of [1, 1000]");
  rr_status s;
  if ((s = check_scene(ctx, sc)) || (s = check_params(ctx, params)) || (s = check_pose(ctx, pose)) ||
      (s = check_materials(ctx, mats, n_mats, sc)))
    return s;
  DeviceGuard dg(ctx->device);
  // the one-launch mode traces only plain scans on a four-wide tree; it is
  // no candidate for air-path scans or an eight-wide tree
  const bool one_launch_ok = !(params->flags & RR_AIR_PATH) && sc->bvh.width != 8;
  return tune(ctx, static_cast<hipStream_t>(stream), reps, one_launch_ok,
              [&] { return rr_radar_scan(ctx, sc, pose, params, mats, n_mats, image_dev, nullptr, stream); }, best,
              best_ms);
}

rr_status rr_autotune_batch(rr_context* ctx, const rr_scene* sc, const rr_scan_desc* scans, uint32_t n_scans,
                            const rr_material* mats, uint32_t n_mats, uint32_t reps, rr_tuning* best,
                            double* best_ms, void* stream) {
  if (!ctx) return fail(nullptr, RR_EINVAL, "context is NULL");
  if (!scans || n_scans == 0 || n_scans > 65535) return fail(ctx, RR_EINVAL, "need 1..65535 scans");
  if (reps == 0 || reps > 1000) return fail(ctx, RR_EINVAL, "reps out of [1, 1000]");
  rr_status s;
  if ((s = check_scene(ctx, sc)) || (s = check_materials(ctx, mats, n_mats, sc))) return s;
  bool air = false;
  for (uint32_t i = 0; i < n_scans; ++i) air = air || (scans[i].params.flags & RR_AIR_PATH) != 0;
  DeviceGuard dg(ctx->device);
  const bool one_launch_ok = !air && sc->bvh.width != 8;
  // the batch call validates the scans (and fails the first candidate otherwise)
  return tune(ctx, static_cast<hipStream_t>(stream), reps, one_launch_ok,
              [&] { return rr_radar_scan_batch(ctx, sc, scans, n_scans, mats, n_mats, nullptr, stream); }, best,
              best_ms);
}

}  // extern "C"
