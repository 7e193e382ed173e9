// api.cpp -- the C ABI declared in include/radarays_hip.h.
//
// Host work per scan: validate, derive the per-scan constants (rotation,
// Eq. 2 radius scale, beam-window coefficients of the standard BRDF), lay
// out the workspace, and enqueue: clear -> bounce level 0..B-1 -> finalize,
// all on the caller's stream with no host synchronisation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/radarays_hip.h"
#include "bvh.h"
#include "kernels.h"
#include "rr_internal.h"

using namespace rr;

#include "api_internal.h"

namespace rr {

thread_local std::string g_err;

rr_status fail(rr_context* ctx, rr_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (ctx) ctx->err = buf;
  g_err = buf;
  return s;
}

bool finite3(const float* p) { return std::isfinite(p[0]) && std::isfinite(p[1]) && std::isfinite(p[2]); }

rr_status check_params(rr_context* ctx, const rr_sensor_params* p) {
  if (!p) return fail(ctx, RR_EINVAL, "params is NULL");
  if (p->n_azimuth < 1 || p->n_azimuth > RR_MAX_AZIMUTH)
    return fail(ctx, RR_EINVAL, "n_azimuth %u out of [1, %u]", p->n_azimuth, RR_MAX_AZIMUTH);
  if (p->rays_per_beam < 1 || p->rays_per_beam > RR_MAX_RAYS_PER_BEAM)
    return fail(ctx, RR_EINVAL, "rays_per_beam %u out of range", p->rays_per_beam);
  if (p->max_bounces < 1 || p->max_bounces > RR_MAX_BOUNCES)
    return fail(ctx, RR_EINVAL, "max_bounces %u out of [1, 8]", p->max_bounces);
  if (p->n_bins < 1 || p->n_bins > RR_MAX_BINS)
    return fail(ctx, RR_EINVAL, "n_bins %u out of [1, %u]", p->n_bins, RR_MAX_BINS);
  if ((uint64_t)p->n_azimuth * p->rays_per_beam > RR_MAX_PRIMARIES)
    return fail(ctx, RR_EINVAL, "n_azimuth * rays_per_beam exceeds %u", RR_MAX_PRIMARIES);
  if (!(std::isfinite(p->bin_size_m) && p->bin_size_m > 0.0f))
    return fail(ctx, RR_EINVAL, "bin_size_m must be finite and > 0");
  if (!(p->beam_width_rad >= 0.0f && p->beam_width_rad < (float)M_PI))
    return fail(ctx, RR_EINVAL, "beam_width_rad must be in [0, pi)");
  if (!(p->beam_prob > 0.0f && p->beam_prob < 1.0f))
    return fail(ctx, RR_EINVAL, "beam_prob must be in (0, 1)");
  if (!(std::isfinite(p->energy_cutoff) && p->energy_cutoff >= 0.0f))
    return fail(ctx, RR_EINVAL, "energy_cutoff must be finite and >= 0");
  if (!std::isfinite((float)p->n_bins * p->bin_size_m))
    return fail(ctx, RR_EINVAL, "n_bins * bin_size_m overflows");
  if (p->flags & ~31u) return fail(ctx, RR_EINVAL, "unknown flag bits 0x%x", p->flags);
  if (!(p->beam_stretch_az >= 0.0f && p->beam_stretch_az <= 100.0f && p->beam_stretch_inc >= 0.0f &&
        p->beam_stretch_inc <= 100.0f))
    return fail(ctx, RR_EINVAL, "beam stretch factors must be in [0, 100]");
  return RR_OK;
}

rr_status check_pose(rr_context* ctx, const rr_pose* q) {
  if (!q) return fail(ctx, RR_EINVAL, "pose is NULL");
  if (!finite3(q->position)) return fail(ctx, RR_EINVAL, "pose position not finite");
  double n = 0;
  for (int i = 0; i < 4; ++i) {
    if (!std::isfinite(q->quat_wxyz[i])) return fail(ctx, RR_EINVAL, "pose quaternion not finite");
    n += (double)q->quat_wxyz[i] * q->quat_wxyz[i];
  }
  if (std::fabs(std::sqrt(n) - 1.0) > 1e-3) return fail(ctx, RR_EINVAL, "pose quaternion not unit");
  return RR_OK;
}

rr_status check_materials(rr_context* ctx, const rr_material* m, uint32_t n, const rr_scene* sc) {
  if (n < 1 || n > RR_MAX_MATERIALS || !m) return fail(ctx, RR_EINVAL, "need 1..255 materials");
  for (uint32_t i = 0; i < n; ++i) {
    const rr_material& q = m[i];
    if (q.kind > RR_COOK_TORRANCE) return fail(ctx, RR_EINVAL, "material %u: unknown kind", i);
    if ((q.kind == RR_DIELECTRIC || q.kind == RR_COOK_TORRANCE) && !(std::isfinite(q.n) && q.n > 0.0f))
      return fail(ctx, RR_EINVAL, "material %u: n must be > 0", i);
    if (q.kind == RR_COOK_TORRANCE) {
      if (!(q.reflectance >= 0.0f && q.reflectance <= 1.0f && q.A >= 0.0f && q.A <= 1.0f && q.B >= 1e-4f &&
            q.B <= 1.0f))
        return fail(ctx, RR_EINVAL, "material %u: Cook-Torrance needs A in [0,1], B in [1e-4,1]", i);
      continue;
    }
    if (!(q.reflectance >= 0.0f && q.reflectance <= 1.0f))
      return fail(ctx, RR_EINVAL, "material %u: reflectance out of [0,1]", i);
    if (!(q.A >= 0.0f && q.A <= 1.0f && q.B >= 0.0f && q.B <= 1.0f && q.A + q.B <= 1.0f + 1e-6f))
      return fail(ctx, RR_EINVAL, "material %u: need A, B in [0,1], A + B <= 1", i);
    if (!(std::isfinite(q.C) && q.C >= 0.0f)) return fail(ctx, RR_EINVAL, "material %u: C must be >= 0", i);
  }
  if (sc && sc->nt && sc->max_mat >= n)
    return fail(ctx, RR_EINVAL, "scene uses material %u but only %u given", sc->max_mat, n);
  return RR_OK;
}

// erfinv by Newton's method on erf (erfc near 1), started from Winitzki's
// closed-form approximation (a = 0.147).
double erfinv_newton(double p) {
  const double a = 0.147;
  double ap = std::fabs(p);
  double w = -std::log((1.0 - ap) * (1.0 + ap));  // -ln(1 - p^2)
  double t = 2.0 / (M_PI * a) - w / 2.0;
  double x = std::sqrt(std::max(0.0, std::sqrt(t * t + w / a) - t));
  for (int it = 0; it < 60; ++it) {
    double f = ap < 0.5 ? std::erf(x) - ap : (1.0 - ap) - std::erfc(x);
    double dfdx = 2.0 / std::sqrt(M_PI) * std::exp(-x * x);
    double step = f / dfdx;
    x -= step;
    if (std::fabs(step) <= 2e-16 * std::fabs(x)) break;
  }
  return p < 0 ? -x : x;
}

// Integral of cos^C over [-pi/2, pi/2] via the Beta function.
double lobe_integral(double C) {
  return std::sqrt(M_PI) * std::exp(std::lgamma((C + 1.0) / 2.0) - std::lgamma(C / 2.0 + 1.0));
}

void make_scan(const rr_pose& pose, const rr_sensor_params& p, DevScan& s) {
  std::memset(&s, 0, sizeof s);
  double w = pose.quat_wxyz[0], x = pose.quat_wxyz[1], y = pose.quat_wxyz[2], z = pose.quat_wxyz[3];
  double qn = std::sqrt(w * w + x * x + y * y + z * z);
  w /= qn;
  x /= qn;
  y /= qn;
  z /= qn;
  s.R[0] = 1.0 - 2.0 * (y * y + z * z);
  s.R[1] = 2.0 * (x * y - w * z);
  s.R[2] = 2.0 * (x * z + w * y);
  s.R[3] = 2.0 * (x * y + w * z);
  s.R[4] = 1.0 - 2.0 * (x * x + z * z);
  s.R[5] = 2.0 * (y * z - w * x);
  s.R[6] = 2.0 * (x * z - w * y);
  s.R[7] = 2.0 * (y * z + w * x);
  s.R[8] = 1.0 - 2.0 * (x * x + y * y);
  double b = p.beam_width_rad, P = p.beam_prob;
  s.sigma_r = (b / 2.0) / (std::sqrt(2.0) * erfinv_newton(P));
  for (int a = 0; a < 3; ++a) s.pos[a] = pose.position[a];
  s.e0 = 1.0f / (float)p.rays_per_beam;
  s.bin_size = p.bin_size_m;
  s.r_max = (float)p.n_bins * p.bin_size_m;
  s.e_cut = p.energy_cutoff;
  s.n_az = p.n_azimuth;
  s.n_s = p.rays_per_beam;
  s.max_b = p.max_bounces;
  s.n_bins = p.n_bins;
  s.flags = p.flags;
  s.scan_id = p.scan_id;
  s.seed = p.seed;
  s.stretch_az = p.beam_stretch_az > 0.0f ? p.beam_stretch_az : 1.0f;
  s.stretch_inc = p.beam_stretch_inc > 0.0f ? p.beam_stretch_inc : 1.0f;
  s.n_prim = p.n_azimuth * p.rays_per_beam;
}

// Beam-window coefficients of the standard BRDF (Eq. 5) normalised to unit
// integral over [-pi/2, pi/2] (Eq. 3) and integrated over a window of width
// b around the return angle (Eq. 4); the S lobe uses the midpoint rule.
void make_materials(const rr_material* m, uint32_t n, float beam_width, std::vector<DevMaterial>& out) {
  out.resize(n);
  double b = beam_width;
  for (uint32_t i = 0; i < n; ++i) {
    double A = m[i].A, B = m[i].B, S = 1.0 - A - B;
    double Z = A * M_PI + 2.0 * B + S * lobe_integral(m[i].C);
    DevMaterial& d = out[i];
    std::memset(&d, 0, sizeof d);
    d.kind = m[i].kind;
    d.n = m[i].n;
    d.refl = m[i].reflectance;
    d.C = m[i].C;
    if (m[i].kind == RR_COOK_TORRANCE) {
      // diffuse amount, roughness, and the solid angle of the beam cone
      d.a = m[i].A;
      d.beta = m[i].B;
      d.s = 2.0 * M_PI * (1.0 - std::cos(b / 2.0));
      continue;
    }
    d.a = A * b / Z;
    d.beta = 2.0 * B * std::sin(b / 2.0) / Z;
    d.s = S * b / Z;
  }
}

constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// fused scan: per-wave child pool and hit ring, for every wave a trace grid
// can have (kSpillLanes / 64)
constexpr uint32_t kWqPool = 2048u, kWqHits = 256u;
constexpr size_t kWqBytes = (size_t)(kSpillLanes / 64u) * (kWqPool + kWqHits) * 64u;

// Levels alternate between two queues; level d of a scan has at most
// N_p * 2^d rays, and only scans with B > d have a level d.  The hit buffer
// holds one (t, leaf) pair per ray of the current level.
void make_layout(const rr_sensor_params* const* ps, uint32_t n, Layout& L, bool fused,
                 uint32_t spill_entries, uint32_t spill_lanes) {
  uint64_t level[RR_MAX_BOUNCES] = {};
  L = Layout();
  L.spill_entries = spill_entries;
  L.spill_lanes = spill_lanes;
  for (uint32_t i = 0; i < n; ++i) {
    const rr_sensor_params& p = *ps[i];
    uint64_t np = (uint64_t)p.n_azimuth * p.rays_per_beam;
    L.n_first += np;
    L.acc_cells += (uint64_t)p.n_azimuth * p.n_bins;
    L.max_b = std::max(L.max_b, p.max_bounces);
    L.air = L.air || (p.flags & RR_AIR_PATH) != 0;
    for (uint32_t d = 1; d < p.max_bounces; ++d) level[d] += np << d;
  }
  L.cap = L.n_first;
  for (uint32_t d = 1; d < RR_MAX_BOUNCES; ++d) L.cap = std::max(L.cap, level[d]);
  size_t o = 0;
  L.off_scans = o;
  o += align256(sizeof(DevScan) * n);
  L.off_mats = o;
  o += align256(sizeof(DevMaterial) * RR_MAX_MATERIALS);
  L.off_ctr = o;
  o += align256(sizeof(uint32_t) * kCtrWords);
  L.off_acc = o;
  o += align256(8 * L.acc_cells);
  size_t cap = (size_t)std::max<uint64_t>(L.cap, 1);
  L.off_hits = o;
  o += align256(8 * cap);
  L.off_spill = o;
  o += align256(sizeof(int32_t) * (size_t)spill_entries * spill_lanes);
  L.off_wq = o;
  if (fused) o += align256(kWqBytes);
  if (L.air) {
    // at most one visibility ray per hit at depth >= 1, all levels together
    for (uint32_t d = 1; d < RR_MAX_BOUNCES; ++d) L.shq_cap += level[d];
    const size_t sc = (size_t)std::max<uint64_t>(L.shq_cap, 1);
    L.off_shq[0] = o;
    o += align256(16 * sc);
    L.off_shq[1] = o;
    o += align256(16 * sc);
    L.off_shq[2] = o;
    o += align256(16 * sc);
  }
  for (int q = 0; q < 2; ++q) {
    L.off_q[q][0] = o;
    o += align256(16 * cap);
    L.off_q[q][1] = o;
    o += align256(16 * cap);
    L.off_q[q][2] = o;
    o += align256(16 * cap);
    L.off_q[q][3] = o;
    o += align256(4 * cap);
  }
  L.total = o;
}

QueueView queue_at(char* ws, const Layout& L, int q) {
  return QueueView{reinterpret_cast<float4*>(ws + L.off_q[q][0]), reinterpret_cast<float4*>(ws + L.off_q[q][1]),
                   reinterpret_cast<uint4*>(ws + L.off_q[q][2]), reinterpret_cast<uint32_t*>(ws + L.off_q[q][3])};
}

uint32_t trace_grid_blocks(const rr_context* ctx) {
  uint32_t g = std::max(1u, (uint32_t)ctx->n_cu * ctx->trace_waves_per_cu / (kTraceBlock / 64u));
  return std::min(g, kSpillLanes / (uint32_t)kTraceBlock);
}

// Tail helping (idle lanes walk subtrees of their wave's unfinished rays)
// for a traversal launch whose rays number at most ctx->tail_help per lane
// of its grid (`bound` is the launch's ray bound).  Few rays per lane leave
// the launch waiting on its longest walks, which helpers shorten; with many
// the helpers' bookkeeping costs more than the short tail it saves.
bool tail_help_on(const rr_context* ctx, uint64_t bound, uint32_t grid_blocks) {
  return ctx->tail_help != RR_TAIL_HELP_OFF &&
         bound <= (uint64_t)ctx->tail_help * grid_blocks * (uint64_t)kTraceBlock;
}

uint32_t scene_spill_need(const rr_scene* sc) {
  // in 32-bit words per lane: an eight-wide stack entry (a node group) takes two
  if (sc->bvh.width == 8)
    return sc->bvh.max_stack > (uint32_t)kStack8 ? 2u * (sc->bvh.max_stack - (uint32_t)kStack8) : 0u;
  return sc->bvh.max_stack > (uint32_t)kStack ? sc->bvh.max_stack - (uint32_t)kStack : 0u;
}

rr_status check_scene(rr_context* ctx, const rr_scene* sc) {
  if (!sc) return fail(ctx, RR_EINVAL, "scene is NULL");
  if (!sc->built) return fail(ctx, RR_ESTATE, "scene has no BVH (call rr_bvh_build)");
  if (!sc->d_nodes) return fail(ctx, RR_ESTATE, "scene has no device copy (created without a context)");
  if (sc->ctx != ctx) return fail(ctx, RR_EINVAL, "scene belongs to another context");
  return RR_OK;
}

// Enqueue the scans described by `scans` (prim_base, acc_base filled here).
rr_status run(rr_context* ctx, const rr_scene* sc, std::vector<DevScan>& scans,
              const rr_sensor_params* const* ps, const rr_material* mats, uint32_t n_mats, char* ws,
              size_t ws_bytes, rr_scan_stats* stats, hipStream_t st, uint64_t* accum_out,
              float beam_width_for_mats, uint32_t* counters_host, bool upload, const PostArgs* post,
              uint32_t spill_entries) {
  if (post && scans.size() != 1) return fail(ctx, RR_EINVAL, "the fused epilogue takes one scan");
  // trace: persistent, enough waves to fill every CU
  const uint32_t trace_grid = trace_grid_blocks(ctx);
  Layout L;
  if (spill_entries >= (uint32_t)kSpill)
    make_layout(ps, (uint32_t)scans.size(), L, ctx->fused != 0);
  else
    make_layout(ps, (uint32_t)scans.size(), L, ctx->fused != 0, spill_entries, trace_grid * (uint32_t)kTraceBlock);
  if (scene_spill_need(sc) > L.spill_entries)
    return fail(ctx, RR_EINVAL, "the spill area holds %u stack entries per lane, the tree needs %u",
                L.spill_entries, scene_spill_need(sc));
  if (ws_bytes < L.total)
    return fail(ctx, RR_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, L.total);
  if (L.cap >= (1ull << 31) || L.n_first >= (1ull << 31))
    return fail(ctx, RR_ENOMEM, "ray queues exceed 2^31 entries");
  if (L.acc_cells >= 0xffffffffull) return fail(ctx, RR_ENOMEM, "image cells exceed 2^32 - 1");
  uint32_t max_cells = 0;
  for (size_t i = 0; i < scans.size(); ++i)
    max_cells = std::max<uint32_t>(max_cells, scans[i].n_az * scans[i].n_bins);
  DevScan* d_scans = reinterpret_cast<DevScan*>(ws + L.off_scans);
  DevMaterial* d_mats = reinterpret_cast<DevMaterial*>(ws + L.off_mats);
  uint32_t* d_ctr = reinterpret_cast<uint32_t*>(ws + L.off_ctr);
  auto* d_acc = reinterpret_cast<unsigned long long*>(ws + L.off_acc);
  if (upload) {
    rr_status us = upload_tables(ctx, scans, ps, mats, n_mats, ws, st, beam_width_for_mats);
    if (us) return us;
  }
  bool masked = false;
  for (const DevScan& q : scans) masked = masked || q.mask != nullptr;
  if (L.air) {
    if (sc->bvh.width == 8) return fail(ctx, RR_EINVAL, "air-path returns need a four-wide BVH");
    if (ctx->fused) return fail(ctx, RR_EINVAL, "air-path returns need the level-by-level launches");
  }
  for (size_t i = 0; i < scans.size(); ++i) {
    // record slots (with the air-path outcomes) are 32-bit indices
    const uint64_t stride = (uint64_t)((1u << scans[i].max_b) - 1u) * ((scans[i].flags & RR_AIR_PATH) ? 2u : 1u);
    if (scans[i].records && (uint64_t)scans[i].n_prim * stride > 0xffffffffull)
      return fail(ctx, RR_EINVAL, "records exceed 2^32 entries");
  }
  // without masks every primary has a fixed queue slot and level 0 is full
  HIP_TRY(ctx, launch_clear(d_acc, (size_t)L.acc_cells, d_ctr, masked ? 0u : (uint32_t)L.n_first, st));
  for (size_t i = 0; i < scans.size(); ++i)
    if (scans[i].records)
      HIP_TRY(ctx, launch_fill_i32(scans[i].records,
                                   (size_t)scans[i].n_prim * ((1u << scans[i].max_b) - 1u) *
                                       ((scans[i].flags & RR_AIR_PATH) ? 2u : 1u),
                                   -2, st));
  LevelArgs a{};
  if (sc->bvh.width == 8) {
    if (ctx->fused) return fail(ctx, RR_EINVAL, "the one-launch mode needs a four-wide BVH");
    a.nodes8 = static_cast<const Node8*>(sc->d_nodes);
    a.n_nodes = sc->n_nodes;
  } else {
    a.nodes = static_cast<const Node4*>(sc->d_nodes);
    a.n_nodes = sc->n_nodes;
  }
  a.levels = L.max_b;
  a.tris = sc->d_tris;
  a.aux = sc->d_aux;
  a.scans = d_scans;
  a.n_scans = (uint32_t)scans.size();
  a.cap = (uint32_t)L.cap;
  a.mats = d_mats;
  a.acc = d_acc;
  a.hits = reinterpret_cast<uint2*>(ws + L.off_hits);
  a.n_first = (uint32_t)L.n_first;
  a.masked = masked ? 1u : 0u;
  a.counters = d_ctr;
  a.prof = (ctx->prof_flags & RR_PROFILE_COUNT) ? ctx->d_prof : nullptr;
  const bool timed_all = (ctx->prof_flags & RR_PROFILE_TIME) != 0;
  const bool timed_trace = timed_all || (ctx->prof_flags & RR_PROFILE_TRACE_TIME) != 0;
  a.refill = ctx->refill_lanes;
  a.pool = ctx->pool_rays;
  a.tri_batch = ctx->tri_batch;
  a.spill = reinterpret_cast<int32_t*>(ws + L.off_spill);
  a.wq = reinterpret_cast<float4*>(ws + L.off_wq);
  a.wq_pool = kWqPool;
  a.wq_hits = kWqHits;
  a.shade_batch = ctx->shade_batch;
  a.air = L.air ? 1u : 0u;
  if (L.air) {
    a.shq = ShadowView{reinterpret_cast<float4*>(ws + L.off_shq[0]), reinterpret_cast<float4*>(ws + L.off_shq[1]),
                       reinterpret_cast<uint4*>(ws + L.off_shq[2])};
    if (L.shq_cap >= (1ull << 32)) return fail(ctx, RR_ENOMEM, "visibility rays exceed 2^32");
    a.shq_cap = (uint32_t)L.shq_cap;
    // outcome records exist only for a single scan (the records entry point)
    a.air_rec = (scans.size() == 1 && (scans[0].flags & RR_AIR_PATH)) ? scans[0].records : nullptr;
  }
  const uint32_t flat_cap = (uint32_t)ctx->n_cu * 8u;
  auto timed_launch = [&](int kind, uint32_t depth, auto&& fn) -> rr_status {
    const bool timed = kind == 1 ? timed_trace : timed_all;
    rr_context::EvPair ev{};
    if (timed) {
      for (hipEvent_t* e : {&ev.a, &ev.b}) {
        if (ctx->ev_free.empty()) {
          hipEvent_t ne;
          HIP_TRY(ctx, hipEventCreate(&ne));
          ctx->ev_free.push_back(ne);
        }
        *e = ctx->ev_free.back();
        ctx->ev_free.pop_back();
      }
      ev.depth = depth;
      ev.kind = kind;
      HIP_TRY(ctx, hipEventRecord(ev.a, st));
    }
    HIP_TRY(ctx, fn());
    if (timed) {
      HIP_TRY(ctx, hipEventRecord(ev.b, st));
      ctx->ev_used.push_back(ev);
    }
    return RR_OK;
  };
  rr_status rs;
  a.depth = 0;
  a.out = queue_at(ws, L, 0);
  {
    uint64_t blocks = (L.n_first + kBlock - 1) / kBlock;
    uint32_t grid = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(blocks, 1), flat_cap);
    if ((rs = timed_launch(0, 0, [&] { return launch_raygen(a, grid, st); }))) return rs;
  }
  uint64_t level_bound = L.n_first;
  if (ctx->fused) {
    // every level in one persistent launch; each wave keeps its rays' children
    a.depth = 0;
    a.in = queue_at(ws, L, 0);
    uint64_t tblocks = (L.n_first + kTraceBlock - 1) / kTraceBlock;
    uint32_t tgrid = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(tblocks, 1), trace_grid);
    if ((rs = timed_launch(1, 0, [&] { return launch_scan(a, tgrid, st); }))) return rs;
  }
  for (uint32_t d = 0; d < (ctx->fused ? 0u : L.max_b); ++d) {
    a.depth = d;
    a.in = queue_at(ws, L, d & 1);
    a.out = queue_at(ws, L, (d + 1) & 1);
    uint64_t tblocks = (level_bound + kTraceBlock - 1) / kTraceBlock;
    uint32_t tgrid = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(tblocks, 1), trace_grid);
    const bool help = tail_help_on(ctx, level_bound, tgrid);
    if ((rs = timed_launch(1, d, [&] { return launch_trace(a, tgrid, help, st); }))) return rs;
    // shade grid: 32 x 512 lanes per CU (the air-path variant 24 x 256): many
    // short blocks, so a finishing block hands its CU to the next while the
    // other resident blocks still run
    const uint32_t sb = (uint32_t)shade_block(a.air);
    const uint32_t lanes_per_cu = a.air ? 24u * 256u : 32u * 512u;
    uint64_t sblocks = (level_bound + sb - 1) / sb;
    uint32_t sgrid = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(sblocks, 1), (uint64_t)ctx->n_cu * (lanes_per_cu / sb));
    if ((rs = timed_launch(2, d, [&] { return launch_shade(a, sgrid, st); }))) return rs;
    level_bound = std::min<uint64_t>(level_bound * 2, L.cap);
  }
  if (L.air && L.max_b > 1) {
    // visibility of the sensor for the air-path returns of every level, in one launch
    a.depth = 0;
    uint64_t vblocks = (L.shq_cap + kTraceBlock - 1) / kTraceBlock;
    uint32_t vgrid = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(vblocks, 1), trace_grid);
    // its rays are one per air-path return that can add energy, usually a
    // small share of the bound (one per hit at depth >= 1), and each walk
    // ends at its first blocker: a launch of few rays per lane, so helping
    // applies whenever it is on
    const bool help = ctx->tail_help != RR_TAIL_HELP_OFF;
    if ((rs = timed_launch(3, 0, [&] { return launch_shadow(a, vgrid, help, st); }))) return rs;
  }
  if (post) {
    // finalize and epilogue in one launch
    PostArgs pa = *post;
    pa.img = nullptr;
    pa.acc = d_acc;
    pa.image = scans[0].image;
    pa.n_az = scans[0].n_az;
    pa.n_bins = scans[0].n_bins;
    pa.n_images = 1;
    HIP_TRY(ctx, launch_post(pa, st));
  } else {
    HIP_TRY(ctx, launch_finalize(d_scans, (uint32_t)scans.size(), d_acc, max_cells, st));
  }
  if (accum_out)
    HIP_TRY(ctx, hipMemcpyAsync(accum_out, d_acc, 8 * L.acc_cells, hipMemcpyDeviceToDevice, st));
  if (counters_host)
    HIP_TRY(ctx, hipMemcpyAsync(counters_host, d_ctr, 4 * kCtrHostWords, hipMemcpyDeviceToHost, st));
  if (stats) {
    HIP_TRY(ctx, hipMemcpyAsync(ctx->h_ctr, d_ctr, 4 * kCtrHostWords, hipMemcpyDeviceToHost, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
    std::memset(stats, 0, sizeof *stats);
    for (uint32_t d = 0; d < RR_MAX_BOUNCES; ++d) {
      uint64_t c = d < L.max_b ? ctx->h_ctr[kCtrCount + d] : 0;
      stats->rays_per_depth[d] = c;
      stats->segments += c;
    }
    stats->overflow = ctx->h_ctr[kCtrOverflow];
    stats->air_rays = ctx->h_ctr[kCtrShadow];
    if (stats->overflow & kOverflowSteps)
      return fail(ctx, RR_EOVERFLOW, "a traversal launch reached its iteration bound");
    if (stats->overflow) return fail(ctx, RR_EOVERFLOW, "ray queue overflow");
  }
  return RR_OK;
}

rr_status make_post_args(rr_context* ctx, const rr_post_params* p, PostArgs& a) {
  if (!p) return fail(ctx, RR_EINVAL, "post parameters are NULL");
  a = PostArgs{};
  const double sigma = p->blur_sigma_bins;
  if (!(sigma >= 0.0 && sigma <= 16.0)) return fail(ctx, RR_EINVAL, "blur_sigma_bins must be in [0, 16]");
  if (!(p->uniform_amp >= 0.0f && std::isfinite(p->uniform_amp)))
    return fail(ctx, RR_EINVAL, "uniform_amp must be finite and >= 0");
  if (!(p->perlin_amp >= 0.0f && std::isfinite(p->perlin_amp)))
    return fail(ctx, RR_EINVAL, "perlin_amp must be finite and >= 0");
  if (p->perlin_amp > 0.0f && !(p->perlin_cell_az >= 1.0f && p->perlin_cell_bins >= 1.0f &&
                                std::isfinite(p->perlin_cell_az) && std::isfinite(p->perlin_cell_bins)))
    return fail(ctx, RR_EINVAL, "perlin cell sizes must be finite and >= 1");
  if (!(p->db_floor < 0.0f && std::isfinite(p->db_floor)))
    return fail(ctx, RR_EINVAL, "db_floor must be finite and < 0");
  if (p->max_value < 1 || p->max_value > 255) return fail(ctx, RR_EINVAL, "max_value must be in 1..255");
  if (p->reserved0 || p->reserved1) return fail(ctx, RR_EINVAL, "reserved fields must be 0");
  // blur taps m = -R..R, weights exp(-m^2 / (2 sigma^2)) normalised to sum 1
  const int R = sigma > 0.0 ? (int)std::ceil(3.0 * sigma) : 0;
  double wsum = 0.0;
  for (int m = -R; m <= R; ++m) {
    a.w[m + R] = R ? std::exp(-((double)m * (double)m) / (2.0 * sigma * sigma)) : 1.0;
    wsum += a.w[m + R];
  }
  for (int m = -R; m <= R; ++m) a.w[m + R] = a.w[m + R] / wsum;
  a.R = R;
  a.uamp = p->uniform_amp;
  a.pamp = p->perlin_amp;
  a.cell_az = p->perlin_amp > 0.0f ? p->perlin_cell_az : 1.0;
  a.cell_bins = p->perlin_amp > 0.0f ? p->perlin_cell_bins : 1.0;
  a.db_floor = p->db_floor;
  a.max_value = (double)p->max_value;
  a.px_scale = a.max_value / (0.0 - a.db_floor);
  // lattice rows one 1024-bin tile can touch: floor(1023 / cell) + 2, plus
  // two for the rounding of the quotients
  a.gcap = p->perlin_amp > 0.0f
               ? (uint32_t)std::min(std::floor(1023.0 / a.cell_bins) + 4.0, (double)kPostTile + 4.0)
               : 0u;
  a.seed = p->seed;
  a.scan_id = p->scan_id;
  return RR_OK;
}

rr_status upload_tables(rr_context* ctx, std::vector<DevScan>& scans, const rr_sensor_params* const* ps,
                        const rr_material* mats, uint32_t n_mats, char* ws, hipStream_t st,
                        float beam_width_for_mats) {
  Layout L;
  make_layout(ps, (uint32_t)scans.size(), L);
  uint64_t pb = 0, ab = 0;
  for (size_t i = 0; i < scans.size(); ++i) {
    scans[i].prim_base = (uint32_t)pb;
    scans[i].acc_base = ab;
    pb += scans[i].n_prim;
    ab += (uint64_t)scans[i].n_az * scans[i].n_bins;
  }
  std::vector<DevMaterial> dm;
  make_materials(mats, n_mats, beam_width_for_mats, dm);
  HIP_TRY(ctx, put_blob(ws + L.off_scans, scans.data(), sizeof(DevScan) * scans.size(), st));
  HIP_TRY(ctx, put_blob(ws + L.off_mats, dm.data(), sizeof(DevMaterial) * dm.size(), st));
  return RR_OK;
}

rr_status ensure_ws(rr_context* ctx, size_t bytes) {
  if (ctx->ws_bytes >= bytes) return RR_OK;
  if (ctx->ws) {
    HIP_TRY(ctx, hipDeviceSynchronize());
    HIP_TRY(ctx, hipFree(ctx->ws));
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) return fail(ctx, RR_ENOMEM, "workspace of %zu bytes: %s", bytes, hipGetErrorString(e));
  ctx->ws = p;
  ctx->ws_bytes = bytes;
  return RR_OK;
}


}  // namespace rr

// ====================================================================== ABI
extern "C" {

const char* rr_status_str(rr_status s) {
  switch (s) {
    case RR_OK: return "ok";
    case RR_EINVAL: return "invalid argument";
    case RR_ENOMEM: return "out of memory";
    case RR_EDEVICE: return "device error";
    case RR_ESTATE: return "invalid state";
    case RR_EOVERFLOW: return "queue overflow";
    default: return "unknown status";
  }
}

const char* rr_last_error(const rr_context* ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

rr_status rr_create(int device, rr_context** out) {
  if (!out) return fail(nullptr, RR_EINVAL, "out is NULL");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n <= 0) return fail(nullptr, RR_EDEVICE, "no HIP device available");
  if (device < 0 || device >= n) return fail(nullptr, RR_EINVAL, "device %d out of [0, %d)", device, n);
  auto* c = new rr_context();
  c->device = device;
  DeviceGuard g(device);
  int cu = 0;
  if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cu > 0)
    c->n_cu = cu;
  void* p = nullptr;
  e = hipHostMalloc(&p, 4 * kCtrHostWords, hipHostMallocDefault);
  if (e != hipSuccess) {
    delete c;
    return fail(nullptr, RR_ENOMEM, "pinned host buffer: %s", hipGetErrorString(e));
  }
  c->h_ctr = static_cast<uint32_t*>(p);
  rr_status ss = scratch_setup(device);
  if (ss) {
    (void)hipHostFree(p);
    delete c;
    return ss;
  }
  *out = c;
  return RR_OK;
}

rr_status rr_destroy(rr_context* ctx) {
  if (!ctx) return RR_OK;
  {
    DeviceGuard g(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->h_ctr) (void)hipHostFree(ctx->h_ctr);
    if (ctx->d_prof) (void)hipFree(ctx->d_prof);
    for (auto& p : ctx->ev_used) {
      (void)hipEventDestroy(p.a);
      (void)hipEventDestroy(p.b);
    }
    for (auto e : ctx->ev_free) (void)hipEventDestroy(e);
  }
  delete ctx;
  return RR_OK;
}

rr_status rr_scene_upload(rr_context* ctx, const float* V, uint32_t nv, const uint32_t* F, uint32_t nt,
                          const uint16_t* M, rr_scene** out) {
  if (!out) return fail(ctx, RR_EINVAL, "out is NULL");
  *out = nullptr;
  if (nt && (!V || !F || !M)) return fail(ctx, RR_EINVAL, "NULL mesh array");
  for (uint32_t i = 0; i < nv; ++i) {
    const float* p = V + 3 * (size_t)i;
    if (!finite3(p)) return fail(ctx, RR_EINVAL, "vertex %u not finite", i);
    for (int a = 0; a < 3; ++a)
      if (std::fabs(p[a]) > 1e7f) return fail(ctx, RR_EINVAL, "vertex %u beyond 1e7", i);
  }
  uint32_t mm = 0;
  for (uint32_t j = 0; j < nt; ++j) {
    for (int a = 0; a < 3; ++a)
      if (F[3 * (size_t)j + a] >= nv) return fail(ctx, RR_EINVAL, "triangle %u: index out of range", j);
    mm = std::max<uint32_t>(mm, M[j]);
  }
  auto* s = new rr_scene();
  s->ctx = ctx;
  s->nv = nv;
  s->nt = nt;
  s->max_mat = mm;
  s->V.assign(V, V + 3 * (size_t)nv);
  s->F.assign(F, F + 3 * (size_t)nt);
  s->M.assign(M, M + nt);
  *out = s;
  return RR_OK;
}

namespace {

void free_scene_device(rr_scene* sc) {
  if (sc->d_nodes) (void)hipFree(sc->d_nodes);
  if (sc->d_tris) (void)hipFree(sc->d_tris);
  if (sc->d_aux) (void)hipFree(sc->d_aux);
  sc->d_nodes = nullptr;
  sc->d_tris = nullptr;
  sc->d_aux = nullptr;
  if (sc->gb) {
    rr::gpu_bvh_free(*sc->gb);
    delete sc->gb;
    sc->gb = nullptr;
  }
  if (sc->hr) {
    rr::host_refit_free(*sc->hr);
    delete sc->hr;
    sc->hr = nullptr;
  }
  sc->refitted = false;
}

// Linear BVH built on the GPU from the scene's mesh (uploaded here).
rr_status build_on_gpu(rr_context* ctx, rr_scene* sc, uint32_t max_leaf) {
  using namespace rr;
  if (!ctx) return fail(ctx, RR_EINVAL, "the GPU builder needs a context");
  if (sc->nt >= kMaxLeafTris) return fail(ctx, RR_EINVAL, "scene has %u triangles, more than 2^27", sc->nt);
  DeviceGuard dg(ctx->device);
  auto t0 = std::chrono::steady_clock::now();
  free_scene_device(sc);
  sc->gb = new GpuBvh();
  GpuBvh& g = *sc->gb;
  g.nv = sc->nv;
  g.nt = sc->nt;
  g.max_leaf = max_leaf;
  const size_t nt = std::max<uint32_t>(sc->nt, 1), nv = std::max<uint32_t>(sc->nv, 1);
  struct Alloc {
    void** p;
    size_t bytes;
  } allocs[] = {
      {reinterpret_cast<void**>(&g.V), 12 * nv},          {reinterpret_cast<void**>(&g.F), 12 * nt},
      {reinterpret_cast<void**>(&g.M), 2 * nt},           {reinterpret_cast<void**>(&g.sorted), 4 * nt},
      {reinterpret_cast<void**>(&g.child), 8 * nt},       {reinterpret_cast<void**>(&g.parent), 8 * nt},
      {reinterpret_cast<void**>(&g.range), 8 * nt},       {reinterpret_cast<void**>(&g.head), 4 * nt},
      {reinterpret_cast<void**>(&g.box), 48 * nt},        {reinterpret_cast<void**>(&g.flag), 4 * nt},
      {reinterpret_cast<void**>(&g.misc), 64},            {reinterpret_cast<void**>(&g.keys), 8 * nt},
      {reinterpret_cast<void**>(&g.ids), 4 * nt},         {reinterpret_cast<void**>(&sc->d_nodes), 64 * nt},
      {reinterpret_cast<void**>(&g.depth), 4 * nt},       {reinterpret_cast<void**>(&g.order), 4 * nt},
      {reinterpret_cast<void**>(&g.level), 8 * kMaxTreeDepth},
      {reinterpret_cast<void**>(&sc->d_tris), 48 * nt},   {reinterpret_cast<void**>(&sc->d_aux), 16 * nt},
  };
  size_t total = 0;
  for (const Alloc& a : allocs) {
    HIP_TRY(ctx, hipMalloc(a.p, a.bytes));
    total += a.bytes;
  }
  // scratch of the sort and the scan (rocPRIM reports the sizes)
  {
    size_t sb = 0, cb = 0;
    HIP_TRY(ctx, rocprim_sizes(nt, &sb, &cb));
    g.temp_bytes = std::max<size_t>(std::max(sb, cb), 256);
    HIP_TRY(ctx, hipMalloc(&g.temp, g.temp_bytes));
  }
  if (sc->nv) HIP_TRY(ctx, hipMemcpy(g.V, sc->V.data(), 12 * (size_t)sc->nv, hipMemcpyHostToDevice));
  if (sc->nt) {
    HIP_TRY(ctx, hipMemcpy(g.F, sc->F.data(), 12 * (size_t)sc->nt, hipMemcpyHostToDevice));
    HIP_TRY(ctx, hipMemcpy(g.M, sc->M.data(), 2 * (size_t)sc->nt, hipMemcpyHostToDevice));
  }
  HIP_TRY(ctx, gpu_bvh_build(g, static_cast<Node4*>(sc->d_nodes), sc->d_tris, sc->d_aux, nullptr));
  auto t1 = std::chrono::steady_clock::now();
  BuiltBvh& b = sc->bvh;
  b = BuiltBvh();
  b.width = 4;
  b.n_tris = sc->nt;
  b.n_hittable = g.m;
  b.n_refs = g.m;
  b.n_leaves = g.n_leaves;
  b.max_depth = g.max_depth;
  b.max_stack = g.max_stack;
  b.pad = g.pad;
  b.build_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  sc->n_nodes = g.n_nodes;
  sc->dev_bytes = 64 * (size_t)g.n_nodes + 48 * (size_t)std::max<uint32_t>(g.m, 1) + 16 * nt;
  if (b.max_stack > (uint32_t)(kStack + kSpill))
    return fail(ctx, RR_EOVERFLOW, "BVH needs %u stack entries, more than %u", b.max_stack, kStack + kSpill);
  sc->built = true;
  (void)total;
  return RR_OK;
}

}  // namespace

rr_status rr_bvh_build(rr_context* ctx, rr_scene* sc, const rr_bvh_options* opt) {
  if (!sc) return fail(ctx, RR_EINVAL, "scene is NULL");
  if (sc->ctx != ctx) return fail(ctx, RR_EINVAL, "scene belongs to another context");
  if (sc->holders.load())
    return fail(ctx, RR_ESTATE, "%u graph(s) or server(s) still use this scene's BVH", sc->holders.load());
  BvhBuildOptions o;
  if (opt && opt->builder > 1) return fail(ctx, RR_EINVAL, "builder must be 0 (host) or 1 (GPU)");
  if (opt && opt->builder == 1) {
    const uint32_t leaf = opt->max_leaf_size ? opt->max_leaf_size : 2u;
    if (leaf > 16) return fail(ctx, RR_EINVAL, "max_leaf_size out of [1, 16]");
    if (opt->width && opt->width != 4) return fail(ctx, RR_EINVAL, "the GPU builder makes four-wide trees");
    if (opt->split_pct || opt->spatial_pct > 0) return fail(ctx, RR_EINVAL, "the GPU builder does not split triangles");
    sc->built = false;
    return build_on_gpu(ctx, sc, leaf);
  }
  if (opt) {
    if (opt->max_leaf_size) o.max_leaf = opt->max_leaf_size;
    if (opt->sah_bins) o.bins = opt->sah_bins;
    o.threads = opt->n_threads;
    o.split_pct = opt->split_pct;
    if (opt->spatial_pct < -1 || opt->spatial_pct > 200) return fail(ctx, RR_EINVAL, "spatial_pct out of [-1, 200]");
    if (opt->spatial_pct) o.spatial_pct = opt->spatial_pct < 0 ? 0u : (uint32_t)opt->spatial_pct;
    o.width = opt->width ? opt->width : 4u;
    if (opt->merge_leaves > 2) return fail(ctx, RR_EINVAL, "merge_leaves out of [0, 2]");
    o.merge_leaves = opt->merge_leaves != 2;
    if (opt->collapse > 2) return fail(ctx, RR_EINVAL, "collapse out of [0, 2]");
    o.collapse = opt->collapse == 1 ? 1u : 0u;
  }
  if (o.width != 4 && o.width != 8) return fail(ctx, RR_EINVAL, "width must be 4 or 8");
  if (o.width == 8 && o.max_leaf > 4) return fail(ctx, RR_EINVAL, "an eight-wide BVH takes leaves of at most 4 triangles");
  if (o.split_pct > 200) return fail(ctx, RR_EINVAL, "split_pct out of [0, 200]");
  if (o.max_leaf < 1 || o.max_leaf > 16) return fail(ctx, RR_EINVAL, "max_leaf_size out of [1, 16]");
  if (o.bins < 4 || o.bins > 64) return fail(ctx, RR_EINVAL, "sah_bins out of [4, 64]");
  try {
    build_bvh(sc->V.data(), sc->F.data(), sc->nt, sc->M.data(), o, sc->bvh);
  } catch (const std::bad_alloc&) {
    return fail(ctx, RR_ENOMEM, "host memory for the BVH");
  }
  if (sc->bvh.n_hittable >= kMaxLeafTris)
    return fail(ctx, RR_EINVAL, "scene has %u triangles, more than 2^27", sc->bvh.n_hittable);
  const uint32_t stack_cap = sc->bvh.width == 8 ? (uint32_t)(kStack8 + kSpill / 2) : (uint32_t)(kStack + kSpill);
  if (sc->bvh.max_stack > stack_cap)
    return fail(ctx, RR_EOVERFLOW, "BVH needs %u stack entries, more than %u", sc->bvh.max_stack, stack_cap);
  if (sc->bvh.width == 8 && sc->bvh.tris.size() / 3 >= kMaxTris8)
    return fail(ctx, RR_EINVAL, "an eight-wide BVH addresses fewer than 2^24 triangle references");
  sc->built = true;
  sc->n_nodes = (uint32_t)(sc->bvh.width == 8 ? sc->bvh.nodes8.size() : sc->bvh.nodes.size());
  if (!ctx) return RR_OK;
  DeviceGuard g(ctx->device);
  free_scene_device(sc);
  size_t bn = sc->bvh.width == 8 ? sizeof(Node8) * sc->bvh.nodes8.size() : sizeof(Node4) * sc->bvh.nodes.size();
  size_t bt = sizeof(float4) * std::max<size_t>(sc->bvh.tris.size(), 3);
  size_t ba = sizeof(float4) * std::max<size_t>(sc->bvh.aux.size(), 1);
  HIP_TRY(ctx, hipMalloc(reinterpret_cast<void**>(&sc->d_nodes), bn));
  HIP_TRY(ctx, hipMalloc(reinterpret_cast<void**>(&sc->d_tris), bt));
  HIP_TRY(ctx, hipMalloc(reinterpret_cast<void**>(&sc->d_aux), ba));
  if (sc->bvh.width == 8)
    HIP_TRY(ctx, hipMemcpy(sc->d_nodes, sc->bvh.nodes8.data(), bn, hipMemcpyHostToDevice));
  else
    HIP_TRY(ctx, hipMemcpy(sc->d_nodes, sc->bvh.nodes.data(), bn, hipMemcpyHostToDevice));
  if (!sc->bvh.tris.empty())
    HIP_TRY(ctx, hipMemcpy(sc->d_tris, sc->bvh.tris.data(), sizeof(float4) * sc->bvh.tris.size(),
                           hipMemcpyHostToDevice));
  if (!sc->bvh.aux.empty())
    HIP_TRY(ctx, hipMemcpy(sc->d_aux, sc->bvh.aux.data(), sizeof(float4) * sc->bvh.aux.size(),
                           hipMemcpyHostToDevice));
  sc->dev_bytes = bn + bt + ba;
  return RR_OK;
}

rr_status rr_bvh_get_info(const rr_scene* sc, rr_bvh_info* out) {
  if (!sc || !out) return fail(nullptr, RR_EINVAL, "NULL argument");
  if (!sc->built) return fail(nullptr, RR_ESTATE, "scene has no BVH");
  std::memset(out, 0, sizeof *out);
  out->n_tris = sc->bvh.n_tris;
  out->n_hittable = sc->bvh.n_hittable;
  out->n_nodes = sc->n_nodes;
  out->n_leaves = sc->bvh.n_leaves;
  out->max_depth = sc->bvh.max_depth;
  out->max_stack = sc->bvh.max_stack;
  out->device_bytes = sc->dev_bytes;
  out->sah_cost = sc->bvh.sah_cost;
  out->build_ms = sc->bvh.build_ms;
  return RR_OK;
}

rr_status rr_bvh_selfcheck(const rr_scene* sc, uint32_t n_rays, uint64_t seed, uint64_t* mismatches) {
  if (!sc || !mismatches) return fail(nullptr, RR_EINVAL, "NULL argument");
  if (!sc->built) return fail(nullptr, RR_ESTATE, "scene has no BVH");
  if (!sc->gb && !sc->refitted) {
    *mismatches = bvh_selfcheck(sc->bvh, n_rays, seed);
    return RR_OK;
  }
  if (!sc->gb) {
    // a refitted host tree: check the device copy (same structure, moved
    // triangles) against brute force over its own leaf triangles
    DeviceGuard dg(sc->ctx->device);
    rr::BuiltBvh b;
    b.width = 4;
    b.n_tris = sc->bvh.n_tris;
    b.nodes.resize(sc->bvh.nodes.size());
    b.tris.resize(sc->bvh.tris.size());
    b.aux.resize(sc->bvh.aux.size());
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(b.nodes.data(), sc->d_nodes, sizeof(rr::Node4) * b.nodes.size(), hipMemcpyDeviceToHost) != hipSuccess ||
        (!b.tris.empty() &&
         hipMemcpy(b.tris.data(), sc->d_tris, sizeof(float4) * b.tris.size(), hipMemcpyDeviceToHost) != hipSuccess) ||
        (!b.aux.empty() &&
         hipMemcpy(b.aux.data(), sc->d_aux, sizeof(float4) * b.aux.size(), hipMemcpyDeviceToHost) != hipSuccess))
      return fail(sc->ctx, RR_EDEVICE, "download of the refitted tree failed");
    for (int k = 0; k < 3; ++k) {
      b.lo[k] = INFINITY;
      b.hi[k] = -INFINITY;
    }
    for (size_t p = 0; p < b.tris.size() / 3; ++p) {
      const float4* t = &b.tris[3 * p];
      for (int k = 0; k < 3; ++k) {
        const float v0 = (&t[0].x)[k];
        for (float x : {v0, v0 + (&t[1].x)[k], v0 + (&t[2].x)[k]}) {
          b.lo[k] = std::min(b.lo[k], x);
          b.hi[k] = std::max(b.hi[k], x);
        }
      }
    }
    for (int k = 0; k < 3; ++k)
      if (!(b.lo[k] <= b.hi[k])) b.lo[k] = b.hi[k] = 0.0f;
    *mismatches = rr::bvh_selfcheck(b, n_rays, seed);
    return RR_OK;
  }
  // a tree built on the GPU: download it and check it on the host, plus
  // that its leaves hold every hittable triangle of the current vertices
  // exactly once
  const rr::GpuBvh& g = *sc->gb;
  DeviceGuard dg(sc->ctx->device);
  rr::BuiltBvh b;
  b.width = 4;
  b.n_tris = g.nt;
  b.nodes.resize(sc->n_nodes);
  b.tris.resize(3 * (size_t)g.m);
  b.aux.resize(g.nt);
  std::vector<float> V(3 * (size_t)g.nv);
  if (hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(b.nodes.data(), sc->d_nodes, sizeof(rr::Node4) * b.nodes.size(), hipMemcpyDeviceToHost) != hipSuccess ||
      (g.m && hipMemcpy(b.tris.data(), sc->d_tris, sizeof(float4) * b.tris.size(), hipMemcpyDeviceToHost) != hipSuccess) ||
      (g.nt && hipMemcpy(b.aux.data(), sc->d_aux, sizeof(float4) * b.aux.size(), hipMemcpyDeviceToHost) != hipSuccess) ||
      (g.nv && hipMemcpy(V.data(), g.V, 4 * V.size(), hipMemcpyDeviceToHost) != hipSuccess))
    return fail(sc->ctx, RR_EDEVICE, "download of the GPU-built tree failed");
  bool first = true;
  for (uint32_t p = 0; p < g.m; ++p) {
    const float4* t = &b.tris[3 * (size_t)p];
    const float v0[3] = {t[0].x, t[0].y, t[0].z};
    for (int k = 0; k < 3; ++k) {
      const float q[3] = {v0[k], v0[k] + (&t[1].x)[k], v0[k] + (&t[2].x)[k]};
      for (float x : q) {
        b.lo[k] = first ? x : std::min(b.lo[k], x);
        b.hi[k] = first ? x : std::max(b.hi[k], x);
      }
    }
    first = false;
  }
  uint64_t bad = rr::bvh_selfcheck(b, n_rays, seed);
  std::vector<uint8_t> seen(g.nt, 0);
  for (uint32_t p = 0; p < g.m; ++p) {
    uint32_t id;
    std::memcpy(&id, &b.tris[3 * (size_t)p].w, 4);
    if (id >= g.nt || seen[id]++) ++bad;
  }
  for (uint32_t j = 0; j < g.nt; ++j) {
    const float* p0 = &V[3 * (size_t)sc->F[3 * (size_t)j + 0]];
    const float* p1 = &V[3 * (size_t)sc->F[3 * (size_t)j + 1]];
    const float* p2 = &V[3 * (size_t)sc->F[3 * (size_t)j + 2]];
    float e1[3], e2[3];
    for (int a = 0; a < 3; ++a) {
      e1[a] = p1[a] - p0[a];
      e2[a] = p2[a] - p0[a];
    }
    const float n0 = e1[1] * e2[2] - e1[2] * e2[1], n1 = e1[2] * e2[0] - e1[0] * e2[2];
    const float n2 = e1[0] * e2[1] - e1[1] * e2[0];
    // every hittable triangle sits in exactly one leaf; a triangle that a
    // refit made degenerate stays in its leaf (zero edges, never hit)
    const bool hittable = rr::dot3(n0, n1, n2, n0, n1, n2) > 0.0f;
    if (hittable ? seen[j] != 1 : seen[j] > 1) ++bad;
  }
  *mismatches = bad;
  return RR_OK;
}

rr_status rr_bvh_refit(rr_context* ctx, rr_scene* sc, const float* vertices_dev, uint32_t nv, void* stream) {
  if (!sc || !vertices_dev) return fail(ctx, RR_EINVAL, "NULL argument");
  if (sc->ctx != ctx || !ctx) return fail(ctx, RR_EINVAL, "scene belongs to another context");
  if (!sc->built || !sc->d_nodes) return fail(ctx, RR_ESTATE, "scene has no BVH on the device");
  if (nv != sc->nv) return fail(ctx, RR_EINVAL, "refit takes %u vertices, got %u", sc->nv, nv);
  DeviceGuard dg(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (sc->gb) {
    if (nv) HIP_TRY(ctx, hipMemcpyAsync(sc->gb->V, vertices_dev, 12 * (size_t)nv, hipMemcpyDeviceToDevice, st));
    HIP_TRY(ctx, rr::gpu_bvh_refit(*sc->gb, static_cast<rr::Node4*>(sc->d_nodes), sc->d_tris, sc->d_aux, st));
    return RR_OK;
  }
  if (sc->bvh.width != 4) return fail(ctx, RR_EINVAL, "refit of an eight-wide BVH is not supported");
  if (!sc->hr) {
    // first refit of this tree: its depth order, indices and materials
    sc->hr = new rr::HostRefit();
    const hipError_t e = rr::host_refit_setup(*sc->hr, sc->bvh.nodes.data(), (uint32_t)sc->bvh.nodes.size(),
                                              (uint32_t)(sc->bvh.tris.size() / 3), sc->F.data(), sc->M.data(),
                                              sc->nt);
    if (e != hipSuccess) {
      rr::host_refit_free(*sc->hr);
      delete sc->hr;
      sc->hr = nullptr;
      return fail(ctx, e == hipErrorOutOfMemory ? RR_ENOMEM : RR_EDEVICE, "refit set-up: %s", hipGetErrorString(e));
    }
  }
  sc->refitted = true;
  HIP_TRY(ctx, rr::host_refit(*sc->hr, vertices_dev, nv, static_cast<rr::Node4*>(sc->d_nodes), sc->d_tris,
                              sc->d_aux, st));
  return RR_OK;
}

rr_status rr_scene_release(rr_context* ctx, rr_scene* sc) {
  if (!sc) return RR_OK;
  if (sc->ctx != ctx) return fail(ctx, RR_EINVAL, "scene belongs to another context");
  if (sc->holders.load())
    return fail(ctx, RR_ESTATE, "%u graph(s) or server(s) still use this scene", sc->holders.load());
  if (ctx) {
    DeviceGuard g(ctx->device);
    free_scene_device(sc);
  }
  delete sc;
  return RR_OK;
}

rr_status rr_workspace_query(const rr_sensor_params* params, size_t* bytes) {
  if (!bytes) return fail(nullptr, RR_EINVAL, "bytes is NULL");
  rr_status s = check_params(nullptr, params);
  if (s) return s;
  Layout L;
  make_layout(&params, 1, L);
  *bytes = L.total;
  return RR_OK;
}

rr_status rr_batch_workspace_query(const rr_scan_desc* scans, uint32_t n, size_t* bytes) {
  if (!bytes || !scans || n == 0 || n > 65535) return fail(nullptr, RR_EINVAL, "need 1..65535 scans");
  std::vector<const rr_sensor_params*> ps(n);
  for (uint32_t i = 0; i < n; ++i) {
    rr_status s = check_params(nullptr, &scans[i].params);
    if (s) return s;
    ps[i] = &scans[i].params;
  }
  Layout L;
  make_layout(ps.data(), n, L);
  *bytes = L.total;
  return RR_OK;
}

static rr_status scan_common(rr_context* ctx, const rr_scene* sc, const rr_pose* pose,
                             const rr_sensor_params* params, const rr_material* mats, uint32_t n_mats,
                             const uint8_t* mask, float* image, int32_t* records, uint64_t* accum,
                             void* ws, size_t ws_bytes, rr_scan_stats* stats, void* stream,
                             const rr_post_params* post = nullptr, float* db = nullptr,
                             uint8_t* u8 = nullptr) {
  if (!ctx) return fail(nullptr, RR_EINVAL, "context is NULL");
  rr_status s;
  if ((s = check_scene(ctx, sc)) || (s = check_params(ctx, params)) || (s = check_pose(ctx, pose)) ||
      (s = check_materials(ctx, mats, n_mats, sc)))
    return s;
  PostArgs pa{};
  if (post) {
    if ((s = make_post_args(ctx, post, pa))) return s;
    if (!image && !db && !u8) return fail(ctx, RR_EINVAL, "image_dev, db_dev and u8_dev are all NULL");
    pa.db = db;
    pa.u8 = u8;
  } else if (!image) {
    return fail(ctx, RR_EINVAL, "image_dev is NULL");
  }
  DeviceGuard g(ctx->device);
  Layout L;
  make_layout(&params, 1, L, ctx->fused != 0);
  if (!ws) {
    if ((s = ensure_ws(ctx, L.total))) return s;
    ws = ctx->ws;
    ws_bytes = ctx->ws_bytes;
  }
  std::vector<DevScan> scans(1);
  make_scan(*pose, *params, scans[0]);
  scans[0].image = image;
  scans[0].records = records;
  scans[0].mask = mask;
  return run(ctx, sc, scans, &params, mats, n_mats, static_cast<char*>(ws), ws_bytes, stats,
             static_cast<hipStream_t>(stream), accum, params->beam_width_rad, nullptr, true,
             post ? &pa : nullptr);
}

rr_status rr_radar_scan(rr_context* ctx, const rr_scene* sc, const rr_pose* pose,
                        const rr_sensor_params* params, const rr_material* mats, uint32_t n_mats,
                        float* image_dev, rr_scan_stats* stats, void* stream) {
  return scan_common(ctx, sc, pose, params, mats, n_mats, nullptr, image_dev, nullptr, nullptr, nullptr, 0,
                     stats, stream);
}

rr_status rr_radar_scan_ws(rr_context* ctx, const rr_scene* sc, const rr_pose* pose,
                           const rr_sensor_params* params, const rr_material* mats, uint32_t n_mats,
                           float* image_dev, void* ws, size_t ws_bytes, rr_scan_stats* stats, void* stream) {
  if (!ws) return fail(ctx, RR_EINVAL, "workspace_dev is NULL");
  if (reinterpret_cast<uintptr_t>(ws) & 255u) return fail(ctx, RR_EINVAL, "workspace not 256-byte aligned");
  return scan_common(ctx, sc, pose, params, mats, n_mats, nullptr, image_dev, nullptr, nullptr, ws, ws_bytes,
                     stats, stream);
}

rr_status rr_radar_scan_records(rr_context* ctx, const rr_scene* sc, const rr_pose* pose,
                                const rr_sensor_params* params, const rr_material* mats, uint32_t n_mats,
                                const uint8_t* mask, float* image_dev, int32_t* records_dev,
                                uint64_t* accum_dev, rr_scan_stats* stats, void* stream) {
  return scan_common(ctx, sc, pose, params, mats, n_mats, mask, image_dev, records_dev, accum_dev, nullptr,
                     0, stats, stream);
}

rr_status rr_radar_scan_post(rr_context* ctx, const rr_scene* sc, const rr_pose* pose,
                             const rr_sensor_params* params, const rr_material* mats, uint32_t n_mats,
                             const rr_post_params* post, float* image_dev, float* db_dev, uint8_t* u8_dev,
                             rr_scan_stats* stats, void* stream) {
  if (!post) return fail(ctx, RR_EINVAL, "post parameters are NULL");
  return scan_common(ctx, sc, pose, params, mats, n_mats, nullptr, image_dev, nullptr, nullptr, nullptr, 0,
                     stats, stream, post, db_dev, u8_dev);
}

rr_status rr_postprocess(rr_context* ctx, const float* images, uint32_t n_images, uint32_t n_az,
                         uint32_t n_bins, const rr_post_params* post, float* db, uint8_t* u8, void* stream) {
  PostArgs a;
  rr_status s;
  if ((s = make_post_args(ctx, post, a))) return s;
  if (!ctx) return fail(nullptr, RR_EINVAL, "context is NULL");
  if (n_images > 65535 || n_az > 65535 || n_bins > 65535)
    return fail(ctx, RR_EINVAL, "n_images, n_azimuth and n_bins must be <= 65535");
  if (n_images == 0 || n_az == 0 || n_bins == 0) return RR_OK;
  if (!images) return fail(ctx, RR_EINVAL, "images_dev is NULL");
  if (!db && !u8) return fail(ctx, RR_EINVAL, "db_dev and u8_dev are both NULL");
  const size_t n = (size_t)n_images * n_az * n_bins;
  auto overlaps = [&](const void* p, size_t bytes) {
    uintptr_t a0 = reinterpret_cast<uintptr_t>(images), a1 = a0 + 4 * n;
    uintptr_t b0 = reinterpret_cast<uintptr_t>(p), b1 = b0 + bytes;
    return p && a0 < b1 && b0 < a1;
  };
  if (overlaps(db, 4 * n) || overlaps(u8, n)) return fail(ctx, RR_EINVAL, "an output overlaps the input");
  a.img = images;
  a.db = db;
  a.u8 = u8;
  a.n_az = n_az;
  a.n_bins = n_bins;
  a.n_images = n_images;
  DeviceGuard g(ctx->device);
  HIP_TRY(ctx, launch_post(a, static_cast<hipStream_t>(stream)));
  return RR_OK;
}

rr_status rr_radar_scan_batch(rr_context* ctx, const rr_scene* sc, const rr_scan_desc* descs, uint32_t n,
                              const rr_material* mats, uint32_t n_mats, rr_scan_stats* stats, void* stream) {
  if (!ctx) return fail(nullptr, RR_EINVAL, "context is NULL");
  if (!descs || n == 0 || n > 65535) return fail(ctx, RR_EINVAL, "need 1..65535 scans");
  rr_status s;
  if ((s = check_scene(ctx, sc)) || (s = check_materials(ctx, mats, n_mats, sc))) return s;
  for (uint32_t i = 0; i < n; ++i) {
    if ((s = check_params(ctx, &descs[i].params)) || (s = check_pose(ctx, &descs[i].pose))) return s;
    if (!descs[i].image_dev) return fail(ctx, RR_EINVAL, "scan %u: image_dev is NULL", i);
    if (descs[i].params.beam_width_rad != descs[0].params.beam_width_rad)
      return fail(ctx, RR_EINVAL, "scans of a batch must share the beam width");
  }
  DeviceGuard g(ctx->device);
  // consecutive groups whose workspace stays within the context's budget
  // (a single scan larger than the budget forms a group of its own)
  std::vector<std::pair<uint32_t, uint32_t>> groups;
  for (uint32_t i = 0; i < n;) {
    uint32_t j = i + 1;
    std::vector<const rr_sensor_params*> ps{&descs[i].params};
    while (j < n) {
      ps.push_back(&descs[j].params);
      Layout L;
      make_layout(ps.data(), (uint32_t)ps.size(), L, ctx->fused != 0);
      if (L.total > ctx->batch_budget) break;
      ++j;
    }
    groups.emplace_back(i, j);
    i = j;
  }
  size_t need = 0;
  for (auto& gr : groups) {
    std::vector<const rr_sensor_params*> ps;
    for (uint32_t i = gr.first; i < gr.second; ++i) ps.push_back(&descs[i].params);
    Layout L;
    make_layout(ps.data(), (uint32_t)ps.size(), L, ctx->fused != 0);
    need = std::max(need, L.total);
  }
  if ((s = ensure_ws(ctx, need))) return s;
  rr_scan_stats total{};
  for (auto& gr : groups) {
    std::vector<const rr_sensor_params*> ps;
    std::vector<DevScan> scans;
    for (uint32_t i = gr.first; i < gr.second; ++i) {
      ps.push_back(&descs[i].params);
      scans.emplace_back();
      make_scan(descs[i].pose, descs[i].params, scans.back());
      scans.back().image = descs[i].image_dev;
      scans.back().mask = descs[i].primary_mask_dev;
    }
    rr_scan_stats st{};
    s = run(ctx, sc, scans, ps.data(), mats, n_mats, static_cast<char*>(ctx->ws), ctx->ws_bytes,
            stats ? &st : nullptr, static_cast<hipStream_t>(stream), nullptr, descs[0].params.beam_width_rad);
    if (s) return s;
    if (stats) {
      total.segments += st.segments;
      for (uint32_t d = 0; d < RR_MAX_BOUNCES; ++d) total.rays_per_depth[d] += st.rays_per_depth[d];
      total.overflow |= st.overflow;
      total.air_rays += st.air_rays;
    }
  }
  if (stats) *stats = total;
  return RR_OK;
}

rr_status rr_set_tuning(rr_context* ctx, const rr_tuning* t) {
  if (!ctx || !t) return fail(ctx, RR_EINVAL, "NULL argument");
  // every field is checked before any is applied: a refused call changes nothing
  const uint32_t rl = t->refill_lanes ? t->refill_lanes : 8u;
  const uint32_t wc = t->trace_waves_per_cu ? t->trace_waves_per_cu : 24u;
  const uint32_t pr = t->pool_rays ? t->pool_rays : 64u;
  if (rl > 64) return fail(ctx, RR_EINVAL, "refill_lanes out of [1, 64]");
  if (wc > 32) return fail(ctx, RR_EINVAL, "trace_waves_per_cu out of [1, 32]");
  if (pr < 64 || pr > 4096) return fail(ctx, RR_EINVAL, "pool_rays out of [64, 4096]");
  if (t->batch_budget_mb && t->batch_budget_mb < 64) return fail(ctx, RR_EINVAL, "batch_budget_mb below 64");
  if (t->tri_batch > 64) return fail(ctx, RR_EINVAL, "tri_batch out of [1, 64]");
  if (t->fused > 2) return fail(ctx, RR_EINVAL, "fused out of [0, 2]");
  if (t->shade_batch > 64) return fail(ctx, RR_EINVAL, "shade_batch out of [1, 64]");
  if (t->tail_help > 1024 && t->tail_help != RR_TAIL_HELP_OFF)
    return fail(ctx, RR_EINVAL, "tail_help out of [1, 1024] (or RR_TAIL_HELP_OFF)");
  ctx->batch_budget = t->batch_budget_mb ? (size_t)t->batch_budget_mb << 20 : (size_t)24 << 30;
  ctx->refill_lanes = rl;
  ctx->trace_waves_per_cu = wc;
  ctx->pool_rays = pr;
  ctx->fused = t->fused == 1 ? 1u : 0u;
  ctx->shade_batch = t->shade_batch ? t->shade_batch : 64u;
  ctx->tri_batch = t->tri_batch ? t->tri_batch : 6u;
  ctx->tail_help = t->tail_help ? t->tail_help : 12u;
  return RR_OK;
}

rr_status rr_get_tuning(const rr_context* ctx, rr_tuning* out) {
  if (!ctx || !out) return fail(nullptr, RR_EINVAL, "NULL argument");
  std::memset(out, 0, sizeof *out);
  out->refill_lanes = ctx->refill_lanes;
  out->trace_waves_per_cu = ctx->trace_waves_per_cu;
  out->pool_rays = ctx->pool_rays;
  out->tri_batch = ctx->tri_batch;
  out->fused = ctx->fused ? 1u : 2u;
  out->shade_batch = ctx->shade_batch;
  out->tail_help = ctx->tail_help;
  out->batch_budget_mb = (uint32_t)(ctx->batch_budget >> 20);
  return RR_OK;
}

rr_status rr_profile_enable(rr_context* ctx, uint32_t flags) {
  if (!ctx) return fail(nullptr, RR_EINVAL, "context is NULL");
  if (flags & ~(RR_PROFILE_TIME | RR_PROFILE_COUNT | RR_PROFILE_TRACE_TIME))
    return fail(ctx, RR_EINVAL, "unknown profile flags");
  DeviceGuard g(ctx->device);
  if ((flags & RR_PROFILE_COUNT) && !ctx->d_prof) {
    HIP_TRY(ctx, hipMalloc(reinterpret_cast<void**>(&ctx->d_prof), kProfWords * sizeof(unsigned long long)));
    HIP_TRY(ctx, hipMemset(ctx->d_prof, 0, kProfWords * sizeof(unsigned long long)));
  }
  ctx->prof_flags = flags;
  return RR_OK;
}

rr_status rr_measure_gather(rr_context* ctx, uint64_t ws_bytes, uint32_t reads_mb, double* gbs) {
  if (!ctx || !gbs) return fail(ctx, RR_EINVAL, "NULL argument");
  if (ws_bytes < (64u << 10) || ws_bytes > (16ull << 30)) return fail(ctx, RR_EINVAL, "working set out of range");
  if (reads_mb == 0 || reads_mb > (1u << 20)) return fail(ctx, RR_EINVAL, "reads_mb out of range");
  DeviceGuard g(ctx->device);
  const uint32_t threads = (uint32_t)ctx->n_cu * 2048u;  // 32 waves per CU
  const uint64_t n_rows64 = ws_bytes / 64u;
  if (n_rows64 >= (1ull << 32)) return fail(ctx, RR_EINVAL, "working set out of range");
  const uint32_t n_rows = (uint32_t)n_rows64;
  const uint32_t steps = std::max<uint32_t>(1u, (uint32_t)(((uint64_t)reads_mb << 20) / (16ull * threads)));
  void* buf = nullptr;
  void* out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  rr_status s = RR_OK;
  auto bail = [&](rr_status st) {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (buf) (void)hipFree(buf);
    if (out) (void)hipFree(out);
    return st;
  };
  hipError_t e;
  if ((e = hipMalloc(&buf, (size_t)n_rows * 64u)) != hipSuccess ||
      (e = hipMalloc(&out, sizeof(float) * threads)) != hipSuccess)
    return bail(fail(ctx, RR_ENOMEM, "gather probe buffers: %s", hipGetErrorString(e)));
  if ((e = hipMemset(buf, 0, (size_t)n_rows * 64u)) != hipSuccess || (e = hipEventCreate(&e0)) != hipSuccess ||
      (e = hipEventCreate(&e1)) != hipSuccess)
    return bail(fail(ctx, RR_EDEVICE, "gather probe: %s", hipGetErrorString(e)));
  const float4* b4 = static_cast<const float4*>(buf);
  float* o = static_cast<float*>(out);
  // one warm pass, then the timed one
  if ((e = launch_gather(b4, n_rows, steps, o, threads, nullptr)) != hipSuccess ||
      (e = hipEventRecord(e0, nullptr)) != hipSuccess ||
      (e = launch_gather(b4, n_rows, steps, o, threads, nullptr)) != hipSuccess ||
      (e = hipEventRecord(e1, nullptr)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess)
    return bail(fail(ctx, RR_EDEVICE, "gather probe: %s", hipGetErrorString(e)));
  float ms = 0.0f;
  if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess)
    return bail(fail(ctx, RR_EDEVICE, "gather probe: %s", hipGetErrorString(e)));
  *gbs = 16.0 * threads * (double)steps / (ms * 1e-3) / 1e9;
  return bail(s);
}

rr_status rr_profile_read(rr_context* ctx, rr_profile* out) {
  if (!ctx || !out) return fail(ctx, RR_EINVAL, "NULL argument");
  DeviceGuard g(ctx->device);
  std::memset(out, 0, sizeof *out);
  for (auto& p : ctx->ev_used) {
    HIP_TRY(ctx, hipEventSynchronize(p.b));
    float ms = 0.0f;
    HIP_TRY(ctx, hipEventElapsedTime(&ms, p.a, p.b));
    if (p.kind == 1) {
      out->trace_ms += ms;
      if (p.depth < RR_MAX_BOUNCES) out->trace_level_ms[p.depth] += ms;
      out->trace_launches++;
    } else if (p.kind == 2) {
      out->shade_ms += ms;
    } else if (p.kind == 3) {
      out->shadow_ms += ms;
    } else {
      out->raygen_ms += ms;
    }
    ctx->ev_free.push_back(p.a);
    ctx->ev_free.push_back(p.b);
  }
  ctx->ev_used.clear();
  if (ctx->d_prof) {
    unsigned long long h[kProfWords] = {};
    HIP_TRY(ctx, hipDeviceSynchronize());
    HIP_TRY(ctx, hipMemcpy(h, ctx->d_prof, sizeof h, hipMemcpyDeviceToHost));
    HIP_TRY(ctx, hipMemset(ctx->d_prof, 0, sizeof h));
    out->node_visits = h[0];
    out->tri_tests = h[1];
    out->rays = h[2];
    out->hits = h[3];
    for (int d = 0; d < RR_MAX_BOUNCES; ++d) {
      out->wave_iters[d] = h[kProfIters + d];
      out->active_lanes[d] = h[kProfActive + d];
      out->tail_wave_iters[d] = h[kProfTailIters + d];
      out->tail_active_lanes[d] = h[kProfTailActive + d];
      out->max_ray_iters[d] = h[kProfMaxVisits + d];
    }
  }
  return RR_OK;
}

}  // extern "C"
