// Serving: continuous batching of render requests over resident scenes.
//
// Threads (all on the device current at creation):
//  - n slot threads, each with its own HIP stream and workspace: a slot takes
//    the next admitted request, runs Preprocess through the tile order
//    (render_prepare, one host wait for the pair count) on its stream, records
//    an event, and hands the frame to the batcher;
//  - the batcher: whenever frames are ready (and fewer than kMaxInFlight
//    batches are running) it makes its blend stream wait for their events,
//    uploads one job descriptor per frame and launches render_batch_kernel
//    over all their (frame, tile) items, then each frame's load sums and
//    copies (render_finish), and records the batch's event;
//  - the retirer: waits for batches in launch order and completes their
//    requests, which frees their slots and returns their arenas to the pool.
// Admission (in arrival order) happens when a request is submitted and when
// a request completes: the head of the queue is admitted when a slot is free
// and its footprint fits the memory budget (or nothing is admitted at all).
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "adr_internal.h"

using namespace adr;

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

constexpr int kMaxJobs = 64;       // frames per batch (max_batch <= this)
constexpr int kRing = 4;           // job-descriptor buffers (> kMaxInFlight)
constexpr int kMaxInFlight = 2;    // batched blends enqueued and not yet finished
constexpr size_t kPoolGrain = (size_t)2 << 20;

// Device blocks kept for reuse: a block handed back is reused for any later
// request (the server returns arenas only when nothing uses them any more).
struct Pool {
  std::mutex mu;
  std::multimap<size_t, void*> free_blocks;
  std::unordered_map<void*, size_t> size_of;
  size_t held = 0;

  void* take(size_t bytes) {
    bytes = (bytes + kPoolGrain - 1) / kPoolGrain * kPoolGrain;
    {
      std::lock_guard<std::mutex> lk(mu);
      auto it = free_blocks.lower_bound(bytes);
      if (it != free_blocks.end() && it->first <= 2 * bytes) {
        void* p = it->second;
        free_blocks.erase(it);
        return p;
      }
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    std::lock_guard<std::mutex> lk(mu);
    size_of[p] = bytes;
    held += bytes;
    return p;
  }
  void give(void* p) {
    std::lock_guard<std::mutex> lk(mu);
    auto it = size_of.find(p);
    if (it != size_of.end()) free_blocks.emplace(it->second, p);
  }
  void release_all() {
    for (auto& kv : size_of) (void)hipFree(kv.first);
    size_of.clear();
    free_blocks.clear();
    held = 0;
  }
};

void* pool_alloc(size_t bytes, void* /*stream*/, void* ctx) { return static_cast<Pool*>(ctx)->take(bytes); }
void pool_free(void* p, size_t /*bytes*/, void* /*stream*/, void* ctx) { static_cast<Pool*>(ctx)->give(p); }

struct Slot;

struct Request {
  uint64_t ticket = 0;
  const adr_scene* scene = nullptr;
  adr_camera cam{};
  adr_render_params params{};
  adr_frame frame{};
  int64_t footprint = 0;
  uint64_t history_key = 0;
  double arrival_s = 0, submit_s = 0, start_s = 0, done_s = 0;
  int32_t status = ADR_OK;
  int32_t batch_size = 0;
  int64_t batch_id = -1;
  std::string error;
  bool finished = false;
  FramePlan plan;
  Slot* slot = nullptr;
};

struct Slot {
  int index = 0;
  hipStream_t stream = nullptr;
  hipEvent_t prepared = nullptr;
  adr_workspace* ws = nullptr;
  std::shared_ptr<Request> req;  // the admitted request, until it completes
  std::thread thread;
};

struct Batch {
  int64_t id = 0;
  int ring = 0;
  hipEvent_t done = nullptr;
  std::vector<std::shared_ptr<Request>> reqs;
  int32_t status = ADR_OK;
  std::string error;
};

}  // namespace

struct adr_server {
  int device = 0;
  adr_server_config cfg{};
  Pool pool;
  adr_allocator pool_alloc{};
  std::vector<std::unique_ptr<Slot>> slots;
  hipStream_t blend_stream = nullptr;
  BlendJob* jobs_host[kRing] = {};
  BlendJob* jobs_dev[kRing] = {};
  hipEvent_t batch_done[kRing] = {};
  bool ring_busy[kRing] = {};
  std::thread batcher, retirer;

  std::mutex mu;
  std::condition_variable cv;  // every state change below
  std::deque<std::shared_ptr<Request>> queue;                      // submitted, not admitted
  std::vector<std::shared_ptr<Request>> ready;                     // prepared, waiting for a blend
  std::deque<Batch> in_flight;                                     // launched, not retired
  std::unordered_map<uint64_t, std::shared_ptr<Request>> requests;  // not yet waited for
  std::unordered_map<uint64_t, int64_t> pairs_seen;                // (scene, size, cull) -> pairs
  uint64_t next_ticket = 1;
  int64_t next_batch = 0;
  int64_t reserved = 0;
  int64_t n_admitted = 0;
  adr_server_stats stats{};
  bool stopping = false;
  bool batcher_done = false;
};

namespace {

uint64_t history_key(const adr_scene* s, const adr_camera& c, const adr_render_params& p) {
  uint64_t h = s->uid * 0x9e3779b97f4a7c15ull;
  h ^= ((uint64_t)(uint32_t)c.width << 32 | (uint32_t)c.height) + 0x7f4a7c159e3779b9ull + (h << 6) + (h >> 2);
  h ^= (uint64_t)p.cull + 0x94d049bb133111ebull + (h << 6) + (h >> 2);
  return h;
}

// Footprint of a request at admission: its workspace for the scene, the
// camera's tiles and the estimated pairs (+25% margin).
int64_t footprint(adr_server* sv, const Request& r) {
  const int64_t n = r.scene->d.n;
  const int64_t tiles = (int64_t)((r.cam.width + kTile - 1) / kTile) * ((r.cam.height + kTile - 1) / kTile);
  auto it = sv->pairs_seen.find(r.history_key);
  const int64_t pairs = it != sv->pairs_seen.end() ? it->second : 4 * n;
  return adr_workspace_bytes(n, pairs + pairs / 4, tiles);
}

// Admits queued requests in arrival order; call with sv->mu held.
void admit_locked(adr_server* sv) {
  while (!sv->queue.empty()) {
    Slot* free_slot = nullptr;
    for (auto& s : sv->slots)
      if (!s->req) {
        free_slot = s.get();
        break;
      }
    if (!free_slot) return;
    std::shared_ptr<Request> r = sv->queue.front();
    r->footprint = footprint(sv, *r);
    const bool none_running = sv->reserved == 0;
    if (!none_running && sv->reserved + r->footprint > sv->cfg.memory_budget) return;
    sv->queue.pop_front();
    sv->reserved += r->footprint;
    sv->stats.reserved_bytes_peak = std::max<int64_t>(sv->stats.reserved_bytes_peak, sv->reserved);
    r->start_s = now_s();
    r->slot = free_slot;
    free_slot->req = r;
    sv->n_admitted += 1;
  }
}

// A request is done (with r->status set): frees its slot and reservation.
void complete_locked(adr_server* sv, const std::shared_ptr<Request>& r) {
  r->done_s = now_s();
  r->finished = true;
  sv->reserved -= r->footprint;
  if (r->status == ADR_OK) sv->pairs_seen[r->history_key] = r->frame.n_pairs;
  sv->stats.requests_done += 1;
}

void slot_loop(adr_server* sv, Slot* slot) {
  (void)hipSetDevice(sv->device);
  for (;;) {
    std::shared_ptr<Request> r;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      sv->cv.wait(lk, [&] { return sv->stopping || slot->req; });
      if (!slot->req) return;  // stopping (every request was finished first)
      r = slot->req;
    }
    adr_status st = render_prepare(r->scene, &r->cam, &r->params, &r->frame, slot->ws, slot->stream, r->plan);
    std::string err = st == ADR_OK ? std::string() : std::string(adr_last_error());
    if (st == ADR_OK) {
      const hipError_t e = hipEventRecord(slot->prepared, slot->stream);
      if (e != hipSuccess) {
        st = hip_fail(e, "adr_server: hipEventRecord");
        err = adr_last_error();
      }
    }
    if (st != ADR_OK) {  // nothing of this frame may still run when its arenas go back
      (void)hipStreamSynchronize(slot->stream);
      (void)hipGetLastError();
    }
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      if (st == ADR_OK) {
        sv->ready.push_back(r);
      } else {
        r->status = st;
        r->error = err;
        complete_locked(sv, r);
      }
      sv->cv.notify_all();
      // wait until the frame is done, then hand the slot back
      sv->cv.wait(lk, [&] { return r->finished; });
    }
    workspace_release_frame_arenas(slot->ws);
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      slot->req.reset();
      admit_locked(sv);
    }
    sv->cv.notify_all();
  }
}

void batcher_loop(adr_server* sv) {
  (void)hipSetDevice(sv->device);
  for (;;) {
    std::vector<std::shared_ptr<Request>> take;
    int ring = -1;
    int64_t id = 0;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      sv->cv.wait(lk, [&] {
        return (sv->stopping && sv->ready.empty()) ||
               (!sv->ready.empty() && (int)sv->in_flight.size() < kMaxInFlight);
      });
      if (sv->ready.empty()) return;  // stopping and drained
      for (int k = 0; k < kRing; ++k)
        if (!sv->ring_busy[k]) {
          ring = k;
          break;
        }
      const size_t n = std::min<size_t>(sv->ready.size(), (size_t)sv->cfg.max_batch);
      take.assign(sv->ready.begin(), sv->ready.begin() + n);
      sv->ready.erase(sv->ready.begin(), sv->ready.begin() + n);
      sv->ring_busy[ring] = true;
      id = sv->next_batch++;
    }
    // larger frames first: their heaviest tiles start before the small frames' tiles
    std::stable_sort(take.begin(), take.end(), [](const std::shared_ptr<Request>& a, const std::shared_ptr<Request>& b) {
      return a->plan.n_tiles > b->plan.n_tiles;
    });
    Batch bt;
    bt.id = id;
    bt.ring = ring;
    bt.done = sv->batch_done[ring];
    bt.reqs = take;
    hipError_t e = hipSuccess;
    int64_t blocks = 0;
    bool any_cap = false;
    int n_jobs = 0;
    for (auto& r : take) {
      if (e == hipSuccess) e = hipStreamWaitEvent(sv->blend_stream, r->slot->prepared, 0);
      adr_workspace* ws = r->slot->ws;
      BlendJob j = make_blend_job(ws, ws->rec, ws->exact, r->plan.vals, r->plan.cam, r->plan.blend, r->plan.n_pairs,
                                  r->scene->d.n, &r->frame, r->plan.want_load);
      j.block_base = (int32_t)blocks;
      blocks += j.n_tiles;
      any_cap = any_cap || r->params.lb_cap > 0;
      sv->jobs_host[ring][n_jobs++] = j;
    }
    if (e == hipSuccess)
      e = hipMemcpyAsync(sv->jobs_dev[ring], sv->jobs_host[ring], n_jobs * sizeof(BlendJob), hipMemcpyHostToDevice,
                         sv->blend_stream);
    if (e == hipSuccess) e = launch_render_batch(sv->jobs_dev[ring], n_jobs, blocks, any_cap, sv->blend_stream);
    if (e != hipSuccess) {
      bt.status = hip_fail(e, "adr_server: batched blend");
      bt.error = adr_last_error();
    }
    for (auto& r : take) {
      if (bt.status != ADR_OK) break;
      const adr_status st =
          render_finish(r->scene, &r->cam, &r->params, &r->frame, r->slot->ws, sv->blend_stream, r->plan, true);
      if (st != ADR_OK) {
        r->status = st;
        r->error = adr_last_error();
      }
    }
    if (hipEventRecord(bt.done, sv->blend_stream) != hipSuccess && bt.status == ADR_OK) {
      bt.status = hip_fail(hipGetLastError(), "adr_server: hipEventRecord");
      bt.error = adr_last_error();
    }
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      for (auto& r : take) {
        r->batch_id = id;
        r->batch_size = (int32_t)take.size();
      }
      sv->stats.batches += 1;
      sv->stats.max_batch_seen = std::max<int32_t>(sv->stats.max_batch_seen, (int32_t)take.size());
      sv->in_flight.push_back(std::move(bt));
    }
    sv->cv.notify_all();
  }
}

void retirer_loop(adr_server* sv) {
  (void)hipSetDevice(sv->device);
  for (;;) {
    Batch bt;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      sv->cv.wait(lk, [&] { return !sv->in_flight.empty() || (sv->stopping && sv->batcher_done); });
      if (sv->in_flight.empty()) return;
      bt = sv->in_flight.front();
    }
    hipError_t e = hipEventSynchronize(bt.done);
    if (e != hipSuccess && bt.status == ADR_OK) {
      bt.status = hip_fail(e, "adr_server: batch");
      bt.error = adr_last_error();
    }
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      sv->in_flight.pop_front();
      sv->ring_busy[bt.ring] = false;
      for (auto& r : bt.reqs) {
        if (bt.status != ADR_OK && r->status == ADR_OK) {
          r->status = bt.status;
          r->error = bt.error;
        }
        complete_locked(sv, r);
      }
    }
    sv->cv.notify_all();
  }
}

void stop_and_free(adr_server* sv) {
  {
    // every queued and running request finishes first
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->cv.wait(lk, [&] {
      if (!sv->queue.empty() || !sv->ready.empty() || !sv->in_flight.empty()) return false;
      for (auto& s : sv->slots)
        if (s->req) return false;
      return true;
    });
    sv->stopping = true;
  }
  sv->cv.notify_all();
  for (auto& s : sv->slots)
    if (s->thread.joinable()) s->thread.join();
  if (sv->batcher.joinable()) sv->batcher.join();
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->batcher_done = true;
  }
  sv->cv.notify_all();
  if (sv->retirer.joinable()) sv->retirer.join();
  (void)hipDeviceSynchronize();
  for (auto& s : sv->slots) {
    if (s->ws) adr_workspace_destroy(s->ws);
    if (s->prepared) (void)hipEventDestroy(s->prepared);
    if (s->stream) (void)hipStreamDestroy(s->stream);
  }
  sv->slots.clear();
  for (int k = 0; k < kRing; ++k) {
    if (sv->jobs_host[k]) (void)hipHostFree(sv->jobs_host[k]);
    if (sv->jobs_dev[k]) (void)hipFree(sv->jobs_dev[k]);
    if (sv->batch_done[k]) (void)hipEventDestroy(sv->batch_done[k]);
  }
  if (sv->blend_stream) (void)hipStreamDestroy(sv->blend_stream);
  sv->pool.release_all();
}

}  // namespace

extern "C" double adr_clock_s(void) { return now_s(); }

extern "C" adr_status adr_server_create(const adr_server_config* config, adr_server** out) {
  if (!out || !config || config->n_slots < 1 || config->n_slots > 64 || config->max_batch < 1 ||
      config->max_batch > kMaxJobs || config->memory_budget <= 0) {
    set_error("adr_server_create: NULL argument, or n_slots / max_batch outside 1..64, or memory_budget <= 0");
    return ADR_E_INVALID;
  }
  *out = nullptr;
  auto* sv = new (std::nothrow) adr_server();
  if (!sv) {
    set_error("adr_server_create: host allocation failed");
    return ADR_E_OOM;
  }
  sv->cfg = *config;
  if (hipGetDevice(&sv->device) != hipSuccess) {
    (void)hipGetLastError();
    delete sv;
    set_error("adr_server_create: no current HIP device");
    return ADR_E_HIP;
  }
  sv->pool_alloc.alloc = pool_alloc;
  sv->pool_alloc.free = pool_free;
  sv->pool_alloc.ctx = &sv->pool;
  adr_status st = ADR_OK;
  if (hipStreamCreateWithFlags(&sv->blend_stream, hipStreamNonBlocking) != hipSuccess) st = ADR_E_HIP;
  for (int k = 0; k < kRing && st == ADR_OK; ++k) {
    if (hipHostMalloc((void**)&sv->jobs_host[k], kMaxJobs * sizeof(BlendJob), hipHostMallocDefault) != hipSuccess ||
        hipMalloc((void**)&sv->jobs_dev[k], kMaxJobs * sizeof(BlendJob)) != hipSuccess)
      st = ADR_E_OOM;
    else if (hipEventCreateWithFlags(&sv->batch_done[k], hipEventDisableTiming) != hipSuccess)
      st = ADR_E_HIP;
  }
  for (int i = 0; i < config->n_slots && st == ADR_OK; ++i) {
    auto s = std::make_unique<Slot>();
    s->index = i;
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&s->prepared, hipEventDisableTiming) != hipSuccess) {
      st = ADR_E_HIP;
    } else {
      st = workspace_create(&sv->pool_alloc, false, &s->ws);
      if (st == ADR_OK) s->ws->headroom = false;  // arenas sized to the frame: the pool keeps them
    }
    sv->slots.push_back(std::move(s));
  }
  if (st != ADR_OK) {
    (void)hipGetLastError();
    const std::string msg = "adr_server_create: could not create a stream, event, workspace or staging buffer";
    stop_and_free(sv);
    delete sv;
    set_error(msg);
    return st;
  }
  for (auto& s : sv->slots) s->thread = std::thread(slot_loop, sv, s.get());
  sv->batcher = std::thread(batcher_loop, sv);
  sv->retirer = std::thread(retirer_loop, sv);
  *out = sv;
  return ADR_OK;
}

extern "C" void adr_server_destroy(adr_server* server) {
  if (!server) return;
  stop_and_free(server);
  delete server;
}

extern "C" adr_status adr_server_submit(adr_server* server, const adr_scene* scene, const adr_camera* cam,
                                        const adr_render_params* params, const adr_frame* frame, double arrival_s,
                                        uint64_t* ticket) {
  if (!server || !ticket) {
    set_error("adr_server_submit: NULL server or ticket");
    return ADR_E_INVALID;
  }
  const adr_status vs = validate_render_args(scene, cam, params, frame);
  if (vs != ADR_OK) return vs;
  auto req = std::make_shared<Request>();
  req->scene = scene;
  req->cam = *cam;
  req->params = *params;
  req->params.flags &= ~ADR_FLAG_TIMING;  // stage events are per workspace, not per request
  req->frame = *frame;
  req->submit_s = now_s();
  req->arrival_s = arrival_s > 0 ? arrival_s : req->submit_s;
  req->history_key = history_key(scene, *cam, *params);
  {
    std::lock_guard<std::mutex> lk(server->mu);
    if (server->stopping) {
      set_error("adr_server_submit: server is shutting down");
      return ADR_E_INVALID;
    }
    req->ticket = server->next_ticket++;
    server->requests.emplace(req->ticket, req);
    server->queue.push_back(req);
    admit_locked(server);
  }
  server->cv.notify_all();
  *ticket = req->ticket;
  return ADR_OK;
}

extern "C" adr_status adr_server_wait(adr_server* server, uint64_t ticket, adr_request_info* info) {
  if (!server) {
    set_error("adr_server_wait: NULL server");
    return ADR_E_INVALID;
  }
  std::shared_ptr<Request> req;
  {
    std::unique_lock<std::mutex> lk(server->mu);
    auto it = server->requests.find(ticket);
    if (it == server->requests.end()) {
      set_error("adr_server_wait: unknown or already retired ticket");
      return ADR_E_INVALID;
    }
    req = it->second;
    server->cv.wait(lk, [&] { return req->finished; });
    server->requests.erase(ticket);
  }
  if (info) {
    info->status = req->status;
    info->batch_size = req->batch_size;
    info->n_pairs = req->frame.n_pairs;
    info->batch_id = req->batch_id;
    info->footprint = req->footprint;
    info->arrival_s = req->arrival_s;
    info->submit_s = req->submit_s;
    info->start_s = req->start_s;
    info->done_s = req->done_s;
  }
  if (req->status != ADR_OK) set_error(req->error);
  return ADR_OK;
}

extern "C" adr_status adr_server_stats_get(adr_server* server, adr_server_stats* out) {
  if (!server || !out) {
    set_error("adr_server_stats_get: NULL argument");
    return ADR_E_INVALID;
  }
  std::lock_guard<std::mutex> lk(server->mu);
  *out = server->stats;
  {
    std::lock_guard<std::mutex> pk(server->pool.mu);
    out->pool_bytes = (int64_t)server->pool.held;
  }
  return ADR_OK;
}
