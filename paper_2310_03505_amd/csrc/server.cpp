// server.cpp -- continuous-batching scan server (rr_server_* in the C ABI).
//
// One dispatcher thread owns the context.  Requests wait in a FIFO; when a
// slot (stream + workspace) is free the dispatcher admits the oldest
// requests whose combined workspace fits the slot's budget, enqueues them as
// one batch, and appends a host callback to the slot's stream that records
// completion times and frees the slot.  Slots run concurrently.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "api_internal.h"

using namespace rr;
using Clock = std::chrono::steady_clock;

namespace {

struct Req {
  uint64_t ticket;
  rr_pose pose;
  rr_sensor_params params;
  float* image;
  Clock::time_point t_submit;
};

struct Result {
  bool done = false;
  rr_status status = RR_OK;
  double latency_ms = 0.0;
};

}  // namespace

struct rr_server;

namespace {
struct Slot {
  rr_server* srv = nullptr;
  hipStream_t stream = nullptr;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  bool busy = false;
  std::vector<Req> batch;
  uint32_t* h_ctr = nullptr;  // pinned copy of the level counters
};
}  // namespace

struct rr_server {
  rr_context* ctx = nullptr;
  const rr_scene* scene = nullptr;
  std::vector<rr_material> mats;
  uint32_t n_slots = 2, max_batch = 256;
  size_t slot_budget = 0;
  std::vector<Slot> slots;
  std::deque<Req> pending;
  std::unordered_map<uint64_t, Result> results;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::thread worker;
  bool stop = false;
  uint64_t next_ticket = 1;
  // statistics since the last reset
  std::vector<double> lat;
  uint64_t submitted = 0, completed = 0, rejected = 0, batches = 0, segments = 0;
  bool have_first = false;
  Clock::time_point t_first, t_last;
  rr_status launch_error = RR_OK;
};

namespace {

size_t layout_bytes(const std::vector<const rr_sensor_params*>& ps, bool fused) {
  Layout L;
  make_layout(ps.data(), (uint32_t)ps.size(), L, fused);
  return L.total;
}

void on_batch_done(void* arg) {
  Slot* sl = static_cast<Slot*>(arg);
  rr_server* s = sl->srv;
  auto now = Clock::now();
  std::lock_guard<std::mutex> lk(s->mu);
  uint64_t segs = 0;
  for (uint32_t d = 0; d < RR_MAX_BOUNCES; ++d) segs += sl->h_ctr[kCtrCount + d];
  for (const Req& r : sl->batch) {
    Result& res = s->results[r.ticket];
    res.done = true;
    res.latency_ms = std::chrono::duration<double, std::milli>(now - r.t_submit).count();
    s->lat.push_back(res.latency_ms);
    s->completed++;
  }
  s->segments += segs;
  s->batches++;
  s->t_last = now;
  sl->batch.clear();
  sl->busy = false;
  s->cv_work.notify_all();
  s->cv_done.notify_all();
}

void dispatcher(rr_server* s) {
  DeviceGuard g(s->ctx->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    auto free_slot = [&]() -> int {
      for (uint32_t i = 0; i < s->n_slots; ++i)
        if (!s->slots[i].busy) return (int)i;
      return -1;
    };
    s->cv_work.wait(lk, [&] { return (s->stop && s->pending.empty()) || (!s->pending.empty() && free_slot() >= 0); });
    if (s->pending.empty()) break;  // stopping and drained
    Slot& sl = s->slots[(size_t)free_slot()];
    // admission: oldest first while the batch's workspace fits the budget
    std::vector<const rr_sensor_params*> ps;
    sl.batch.clear();
    float bw = s->pending.front().params.beam_width_rad;
    while (!s->pending.empty() && sl.batch.size() < s->max_batch) {
      const Req& cand = s->pending.front();
      if (cand.params.beam_width_rad != bw) break;
      ps.push_back(&cand.params);
      if (!sl.batch.empty() && layout_bytes(ps, s->ctx->fused != 0) > s->slot_budget) {
        ps.pop_back();
        break;
      }
      sl.batch.push_back(cand);
      s->pending.pop_front();
    }
    sl.busy = true;
    lk.unlock();
    // launch outside the lock; pointers into sl.batch stay valid (no resize)
    std::vector<const rr_sensor_params*> bp;
    std::vector<DevScan> scans(sl.batch.size());
    for (size_t i = 0; i < sl.batch.size(); ++i) {
      bp.push_back(&sl.batch[i].params);
      make_scan(sl.batch[i].pose, sl.batch[i].params, scans[i]);
      scans[i].image = sl.batch[i].image;
    }
    rr_status st = RR_OK;
    size_t need = layout_bytes(bp, s->ctx->fused != 0);
    if (sl.ws_bytes < need) {
      if (sl.ws) (void)hipFree(sl.ws);  // the slot's stream is idle
      sl.ws = nullptr;
      sl.ws_bytes = 0;
      if (hipMalloc(&sl.ws, need) != hipSuccess) {
        sl.ws = nullptr;
        st = RR_ENOMEM;
      } else {
        sl.ws_bytes = need;
      }
    }
    if (st == RR_OK)
      st = run(s->ctx, s->scene, scans, bp.data(), s->mats.data(), (uint32_t)s->mats.size(),
               static_cast<char*>(sl.ws), sl.ws_bytes, nullptr, sl.stream, nullptr, bw, sl.h_ctr);
    if (st == RR_OK && hipLaunchHostFunc(sl.stream, on_batch_done, &sl) != hipSuccess) st = RR_EDEVICE;
    // no callback is pending on this slot when the launch failed; wait for
    // what was enqueued before taking the lock again
    if (st != RR_OK) (void)hipStreamSynchronize(sl.stream);
    lk.lock();
    if (st != RR_OK) {
      // nothing (more) will complete on this slot for this batch: fail its requests
      for (const Req& r : sl.batch) {
        Result& res = s->results[r.ticket];
        res.done = true;
        res.status = st;
      }
      s->launch_error = st;
      sl.batch.clear();
      sl.busy = false;
      s->cv_done.notify_all();
    }
  }
  // drain: wait for the slots in flight
  s->cv_work.wait(lk, [&] {
    for (auto& q : s->slots)
      if (q.busy) return false;
    return true;
  });
}

}  // namespace

extern "C" {

rr_status rr_server_create(rr_context* ctx, const rr_scene* scene, const rr_material* mats, uint32_t n_mats,
                           const rr_server_options* opt, rr_server** out) {
  if (!out) return fail(ctx, RR_EINVAL, "out is NULL");
  *out = nullptr;
  if (!ctx) return fail(nullptr, RR_EINVAL, "context is NULL");
  rr_status st;
  if ((st = check_scene(ctx, scene)) || (st = check_materials(ctx, mats, n_mats, scene))) return st;
  auto* s = new rr_server();
  s->ctx = ctx;
  s->scene = scene;
  s->mats.assign(mats, mats + n_mats);
  uint64_t budget = (uint64_t)32 << 30;
  if (opt) {
    if (opt->n_slots) s->n_slots = opt->n_slots;
    if (opt->max_batch_scans) s->max_batch = opt->max_batch_scans;
    if (opt->memory_budget) budget = opt->memory_budget;
  }
  if (s->n_slots < 1 || s->n_slots > 8 || s->max_batch < 1 || s->max_batch > 65535) {
    delete s;
    return fail(ctx, RR_EINVAL, "n_slots must be 1..8 and max_batch_scans 1..65535");
  }
  s->slot_budget = (size_t)(budget / s->n_slots);
  DeviceGuard g(ctx->device);
  s->slots.resize(s->n_slots);
  for (auto& sl : s->slots) {
    sl.srv = s;
    void* p = nullptr;
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipHostMalloc(&p, 4 * kCtrHostWords, hipHostMallocDefault) != hipSuccess) {
      for (auto& q : s->slots) {
        if (q.stream) (void)hipStreamDestroy(q.stream);
        if (q.h_ctr) (void)hipHostFree(q.h_ctr);
      }
      delete s;
      return fail(ctx, RR_EDEVICE, "server streams / pinned buffers");
    }
    sl.h_ctr = static_cast<uint32_t*>(p);
    std::memset(sl.h_ctr, 0, 4 * kCtrHostWords);
  }
  scene->holders.fetch_add(1);
  s->worker = std::thread(dispatcher, s);
  *out = s;
  return RR_OK;
}

rr_status rr_server_submit(rr_server* s, const rr_pose* pose, const rr_sensor_params* params, float* image,
                           uint64_t* ticket) {
  if (!s || !ticket) return fail(nullptr, RR_EINVAL, "NULL argument");
  rr_status st;
  if ((st = check_params(nullptr, params)) || (st = check_pose(nullptr, pose))) return st;
  if (!image) return fail(nullptr, RR_EINVAL, "image_dev is NULL");
  std::vector<const rr_sensor_params*> ps{params};
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return fail(nullptr, RR_ESTATE, "server is stopping");
  if (layout_bytes(ps, s->ctx->fused != 0) > s->slot_budget) {
    s->rejected++;
    return fail(nullptr, RR_ENOMEM, "request needs more workspace than a slot's budget");
  }
  Req r;
  r.ticket = s->next_ticket++;
  r.pose = *pose;
  r.params = *params;
  r.image = image;
  r.t_submit = Clock::now();
  if (!s->have_first) {
    s->have_first = true;
    s->t_first = r.t_submit;
  }
  s->submitted++;
  s->results[r.ticket] = Result();
  s->pending.push_back(r);
  *ticket = r.ticket;
  s->cv_work.notify_all();
  return RR_OK;
}

rr_status rr_server_wait(rr_server* s, uint64_t ticket, double* latency_ms) {
  if (!s) return fail(nullptr, RR_EINVAL, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->results.find(ticket);
  if (it == s->results.end()) return fail(nullptr, RR_EINVAL, "unknown ticket");
  s->cv_done.wait(lk, [&] { return s->results[ticket].done; });
  Result r = s->results[ticket];
  s->results.erase(ticket);
  if (latency_ms) *latency_ms = r.latency_ms;
  if (r.status) return fail(nullptr, r.status, "request failed");
  return RR_OK;
}

rr_status rr_server_poll(rr_server* s, uint64_t ticket, int* done, double* latency_ms) {
  if (!s || !done) return fail(nullptr, RR_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->results.find(ticket);
  if (it == s->results.end()) return fail(nullptr, RR_EINVAL, "unknown ticket");
  *done = it->second.done ? 1 : 0;
  if (it->second.done) {
    Result r = it->second;
    s->results.erase(it);
    if (latency_ms) *latency_ms = r.latency_ms;
    if (r.status) return fail(nullptr, r.status, "request failed");
  }
  return RR_OK;
}

rr_status rr_server_get_stats(rr_server* s, rr_server_stats* out) {
  if (!s || !out) return fail(nullptr, RR_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  std::memset(out, 0, sizeof *out);
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->rejected = s->rejected;
  out->batches = s->batches;
  out->segments = s->segments;
  if (!s->lat.empty()) {
    std::vector<double> v = s->lat;
    std::sort(v.begin(), v.end());
    auto pct = [&](double q) {
      size_t i = (size_t)std::min<double>(v.size() - 1, std::ceil(q * v.size()) - 1);
      return v[i];
    };
    out->latency_p50_ms = pct(0.50);
    out->latency_p99_ms = pct(0.99);
    double sum = 0;
    for (double x : v) sum += x;
    out->latency_mean_ms = sum / v.size();
    out->latency_max_ms = v.back();
  }
  if (s->have_first && s->completed) {
    out->wall_s = std::chrono::duration<double>(s->t_last - s->t_first).count();
    if (out->wall_s > 0) {
      out->scans_per_s = s->completed / out->wall_s;
      out->mseg_per_s = s->segments / out->wall_s / 1e6;
    }
  }
  return RR_OK;
}

rr_status rr_server_reset_stats(rr_server* s) {
  if (!s) return fail(nullptr, RR_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  s->lat.clear();
  s->submitted = s->completed = s->rejected = s->batches = s->segments = 0;
  s->have_first = false;
  return RR_OK;
}

rr_status rr_server_destroy(rr_server* s) {
  if (!s) return RR_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv_work.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  {
    DeviceGuard g(s->ctx->device);
    for (auto& sl : s->slots) {
      if (sl.stream) {
        (void)hipStreamSynchronize(sl.stream);
        (void)hipStreamDestroy(sl.stream);
      }
      if (sl.ws) (void)hipFree(sl.ws);
      if (sl.h_ctr) (void)hipHostFree(sl.h_ctr);
    }
  }
  s->scene->holders.fetch_sub(1);
  delete s;
  return RR_OK;
}

}  // extern "C"
