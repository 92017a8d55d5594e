// Serving: a fixed set of render slots (host thread + HIP stream +
// workspace) consuming a FIFO of frame requests over resident scenes. Each
// slot renders with adr_render on its own stream, so frames of different
// requests overlap on the device; a request's results do not depend on what
// else runs, because every frame's state lives in its slot's workspace.
#include <chrono>
#include <condition_variable>
#include <deque>
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

struct Request {
  uint64_t ticket = 0;
  const adr_scene* scene = nullptr;
  adr_camera cam{};
  adr_render_params params{};
  adr_frame frame{};
  double submit_s = 0, start_s = 0, done_s = 0;
  int32_t status = ADR_OK;
  std::string error;
  bool finished = false;
};

struct Slot {
  hipStream_t stream = nullptr;
  adr_workspace* ws = nullptr;
  std::thread thread;
};

}  // namespace

struct adr_server {
  int device = 0;
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Request>> queue;
  std::unordered_map<uint64_t, std::shared_ptr<Request>> requests;
  uint64_t next_ticket = 1;
  bool stopping = false;
};

namespace {

void slot_loop(adr_server* sv, Slot* slot) {
  (void)hipSetDevice(sv->device);
  for (;;) {
    std::shared_ptr<Request> req;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      sv->cv_work.wait(lk, [&] { return sv->stopping || !sv->queue.empty(); });
      if (sv->queue.empty()) return;  // stopping and drained
      req = sv->queue.front();
      sv->queue.pop_front();
    }
    req->start_s = now_s();
    adr_status st = adr_render(req->scene, &req->cam, &req->params, &req->frame, slot->ws, slot->stream);
    std::string err = st == ADR_OK ? std::string() : std::string(adr_last_error());
    const hipError_t e = hipStreamSynchronize(slot->stream);
    if (e != hipSuccess && st == ADR_OK) {
      st = ADR_E_HIP;
      err = std::string("adr_server: stream synchronize failed: ") + hipGetErrorString(e);
      (void)hipGetLastError();
    }
    req->done_s = now_s();
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      req->status = st;
      req->error = std::move(err);
      req->finished = true;
    }
    sv->cv_done.notify_all();
  }
}

void stop_and_free(adr_server* sv) {
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stopping = true;
  }
  sv->cv_work.notify_all();
  for (Slot& s : sv->slots)
    if (s.thread.joinable()) s.thread.join();
  for (Slot& s : sv->slots) {
    if (s.ws) adr_workspace_destroy(s.ws);
    if (s.stream) (void)hipStreamDestroy(s.stream);
  }
  sv->slots.clear();
}

}  // namespace

extern "C" double adr_clock_s(void) { return now_s(); }

// Switched off: the first GPU run of the serving test ended with a GPU
// memory fault whose cause has not been found (no out-of-bounds access or
// lifetime error has been identified in this file or in the render path it
// drives). Until one is, creating a server reports ADR_E_UNSUPPORTED.
static constexpr bool kServingEnabled = false;

extern "C" adr_status adr_server_create(int32_t n_slots, adr_server** out) {
  if (!out || n_slots < 1 || n_slots > 64) {
    set_error("adr_server_create: NULL out or n_slots outside 1..64");
    return ADR_E_INVALID;
  }
  *out = nullptr;
  if (!kServingEnabled) {
    set_error("adr_server_create: serving is switched off in this build (a GPU fault in its first test is "
              "not yet explained)");
    return ADR_E_UNSUPPORTED;
  }
  auto* sv = new (std::nothrow) adr_server();
  if (!sv) {
    set_error("adr_server_create: host allocation failed");
    return ADR_E_OOM;
  }
  if (hipGetDevice(&sv->device) != hipSuccess) {
    (void)hipGetLastError();
    delete sv;
    set_error("adr_server_create: no current HIP device");
    return ADR_E_HIP;
  }
  sv->slots.resize((size_t)n_slots);
  for (Slot& s : sv->slots) {
    adr_status st = ADR_OK;
    if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      s.stream = nullptr;
      set_error("adr_server_create: hipStreamCreateWithFlags failed");
      st = ADR_E_HIP;
    } else {
      st = adr_workspace_create(&s.ws);
    }
    if (st != ADR_OK) {
      stop_and_free(sv);
      delete sv;
      return st;
    }
  }
  for (Slot& s : sv->slots) s.thread = std::thread(slot_loop, sv, &s);
  *out = sv;
  return ADR_OK;
}

extern "C" void adr_server_destroy(adr_server* server) {
  if (!server) return;
  stop_and_free(server);
  delete server;
}

extern "C" adr_status adr_server_submit(adr_server* server, const adr_scene* scene, const adr_camera* cam,
                                        const adr_render_params* params, const adr_frame* frame,
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
  req->frame = *frame;
  req->submit_s = now_s();
  {
    std::lock_guard<std::mutex> lk(server->mu);
    if (server->stopping) {
      set_error("adr_server_submit: server is shutting down");
      return ADR_E_INVALID;
    }
    req->ticket = server->next_ticket++;
    server->requests.emplace(req->ticket, req);
    server->queue.push_back(req);
  }
  server->cv_work.notify_one();
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
    server->cv_done.wait(lk, [&] { return req->finished; });
    server->requests.erase(ticket);  // (the iterator may be stale after the wait)
  }
  if (info) {
    info->status = req->status;
    info->n_pairs = req->frame.n_pairs;
    info->submit_s = req->submit_s;
    info->start_s = req->start_s;
    info->done_s = req->done_s;
  }
  if (req->status != ADR_OK) set_error(req->error);
  return ADR_OK;
}
