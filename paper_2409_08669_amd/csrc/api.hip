// C ABI: workspace management and the per-frame orchestration of the six
// stages of Sec. 3.2 on the caller's stream.
//
// A workspace is four device arenas (per Gaussian, per pair, per tile, and a
// few fixed words), each one allocation carved into 256-byte aligned arrays.
// When a frame needs a larger arena the new one is allocated before the old
// one is released: through the caller's allocator (a stream-ordered release),
// or with hipMalloc while the old arena is kept until the next reserve or
// destroy. No hipFree runs inside a render.
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "adr_internal.h"

namespace adr {

namespace {
thread_local std::string g_error;
}  // namespace

void set_error(const std::string& msg) { g_error = msg; }

adr_status hip_fail(hipError_t e, const char* what) {
  g_error = std::string(what) + ": " + hipGetErrorString(e);
  (void)hipGetLastError();
  return ADR_E_HIP;
}

namespace {

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Carves consecutive 256-byte aligned arrays out of one arena (or only adds
// up their sizes when base is null).
struct Carver {
  uint8_t* base;
  size_t off = 0;
  template <class T>
  T* take(int64_t count) {
    off = align256(off);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += (size_t)(count > 0 ? count : 0) * sizeof(T);
    return p;
  }
  size_t bytes() const { return align256(off); }
};

}  // namespace

size_t carve_gauss_arena(uint8_t* base, int64_t n, adr_workspace* ws) {
  Carver c{base};
  auto* rec = c.take<RenderRecord>(n);
  auto* exact = c.take<ExactRecord>(n);
  auto* rect = c.take<uint2>(n);
  auto* touched = c.take<uint32_t>(n);
  auto* offsets = c.take<uint32_t>(n);
  auto* touched_sorted = c.take<uint32_t>(n);
  auto* dk0 = c.take<uint32_t>(n);
  auto* dk1 = c.take<uint32_t>(n);
  auto* dv0 = c.take<uint32_t>(n);
  auto* dv1 = c.take<uint32_t>(n);
  auto* scan_partials = c.take<uint32_t>(inclusive_sum_partials(n) + 1);
  auto* block_parts = c.take<ulonglong4>(preprocess_blocks(n));
  auto* scratch = c.take<uint32_t>(sort_scratch_entries(n));
  if (ws) {
    ws->rec = rec;
    ws->exact = exact;
    ws->tile_rect = rect;
    ws->touched = touched;
    ws->offsets = offsets;
    ws->touched_sorted = touched_sorted;
    ws->depth.keys[0] = dk0;
    ws->depth.keys[1] = dk1;
    ws->depth.vals[0] = dv0;
    ws->depth.vals[1] = dv1;
    ws->scan_partials = scan_partials;
    ws->block_parts = block_parts;
    ws->depth_scratch = scratch;
  }
  return c.bytes();
}

size_t carve_pair_arena(uint8_t* base, int64_t n_pairs, adr_workspace* ws) {
  Carver c{base};
  auto* k0 = c.take<uint32_t>(n_pairs);
  auto* k1 = c.take<uint32_t>(n_pairs);
  auto* v0 = c.take<uint32_t>(n_pairs);
  auto* v1 = c.take<uint32_t>(n_pairs);
  auto* dup_first = c.take<uint32_t>(duplicate_blocks(n_pairs) + 1);
  auto* scratch = c.take<uint32_t>(sort_scratch_entries(n_pairs));
  if (ws) {
    ws->pairs.keys[0] = k0;
    ws->pairs.keys[1] = k1;
    ws->pairs.vals[0] = v0;
    ws->pairs.vals[1] = v1;
    ws->dup_first = dup_first;
    ws->pair_scratch = scratch;
  }
  return c.bytes();
}

size_t carve_tile_arena(uint8_t* base, int64_t n_tiles, adr_workspace* ws) {
  Carver c{base};
  auto* ranges = c.take<uint32_t>(2 * n_tiles);
  auto* order = c.take<uint32_t>(n_tiles);
  auto* counts = c.take<uint32_t>(tile_order_scratch((int)n_tiles));
  auto* wave_sums = c.take<unsigned long long>(16 * n_tiles);  // 4 waves x 4 sums per tile
  if (ws) {
    ws->ranges = ranges;
    ws->tile_order = order;
    ws->order_counts = counts;
    ws->wave_sums = wave_sums;
  }
  return c.bytes();
}

size_t carve_fixed_arena(uint8_t* base, adr_workspace* ws) {
  Carver c{base};
  auto* counters = c.take<unsigned long long>(kCounterSlots);
  auto* hists = c.take<uint32_t>(2 * kHistWords);
  auto* load_acc = c.take<unsigned long long>(kLoadAccWords);
  auto* notify = c.take<unsigned long long>(kNotifySlots);
  if (ws) {
    ws->dev_counters = counters;
    ws->hists = hists;
    ws->load_acc = load_acc;
    ws->notify_slot = notify;
  }
  return c.bytes();
}

namespace {

size_t carve_grad_arena(uint8_t* base, int64_t n, adr_workspace* ws) {
  Carver c{base};
  auto* g = c.take<float>((int64_t)kGrad2d * n);
  if (ws) ws->grad2d = g;
  return c.bytes();
}

void* acquire(adr_workspace* ws, size_t bytes, hipStream_t stream) {
  if (ws->growth == Growth::kAllocator) return ws->alloc.alloc(bytes, (void*)stream, ws->alloc.ctx);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

// in_render: called while a frame may still use the arena on `stream`
void release(adr_workspace* ws, Arena& a, hipStream_t stream, bool in_render) {
  if (!a.base) return;
  if (ws->growth == Growth::kAllocator) {
    ws->alloc.free(a.base, a.bytes, (void*)stream, ws->alloc.ctx);
  } else if (ws->growth == Growth::kDefault) {
    if (in_render)
      ws->retired.push_back(a);
    else
      (void)hipFree(a.base);
  }
  a = Arena{};
}

void free_retired(adr_workspace* ws) {
  for (Arena& a : ws->retired) (void)hipFree(a.base);
  ws->retired.clear();
}

using CarveFn = size_t (*)(uint8_t*, int64_t, adr_workspace*);

adr_status grow_arena(adr_workspace* ws, Arena& arena, int64_t& cap, int64_t need, CarveFn carve, bool headroom,
                      bool in_render, hipStream_t stream, const char* what) {
  if (need <= cap && arena.base) return ADR_OK;
  if (ws->growth == Growth::kNone) {
    set_error(std::string("workspace of fixed size too small for the frame's ") + what);
    return ADR_E_WORKSPACE;
  }
  int64_t n = need < 1 ? 1 : need;
  if (headroom) n += n / 4;  // frame-to-frame jitter does not regrow
  const size_t bytes = carve(nullptr, n, nullptr);
  auto* p = static_cast<uint8_t*>(acquire(ws, bytes, stream));
  if (!p) {
    set_error(std::string("workspace allocation failed: ") + what);
    return ADR_E_OOM;
  }
  release(ws, arena, stream, in_render);
  arena.base = p;
  arena.bytes = bytes;
  cap = n;
  carve(p, n, ws);
  return ADR_OK;
}

int bits_for(int64_t v) {
  int b = 0;
  while (((int64_t)1 << b) < v) ++b;
  return b;
}

}  // namespace

adr_status ensure_capacity(adr_workspace* ws, int64_t n_gauss, int64_t n_pairs, int64_t n_tiles, hipStream_t stream) {
  adr_status st;
  const bool h = ws->headroom;
  if ((st = grow_arena(ws, ws->gauss_arena, ws->gauss_capacity, n_gauss, carve_gauss_arena, h, true, stream,
                       "Gaussians")) != ADR_OK)
    return st;
  if ((st = grow_arena(ws, ws->pair_arena, ws->pair_capacity, n_pairs, carve_pair_arena, h, true, stream,
                       "pairs")) != ADR_OK)
    return st;
  return grow_arena(ws, ws->tile_arena, ws->tile_capacity, n_tiles, carve_tile_arena, h, true, stream, "tiles");
}

void workspace_release_frame_arenas(adr_workspace* ws) {
  release(ws, ws->gauss_arena, nullptr, false);
  release(ws, ws->pair_arena, nullptr, false);
  release(ws, ws->tile_arena, nullptr, false);
  ws->gauss_capacity = ws->pair_capacity = ws->tile_capacity = 0;
}

}  // namespace adr

using namespace adr;

static void free_workspace(adr_workspace* ws) {
  if (ws->slots[0] == ws)
    for (int i = 1; i < adr_workspace::kFrameSlots; ++i)
      if (ws->slots[i]) free_workspace(ws->slots[i]);
  Arena* arenas[] = {&ws->gauss_arena, &ws->pair_arena, &ws->tile_arena, &ws->fixed_arena, &ws->grad_arena};
  for (Arena* a : arenas) release(ws, *a, nullptr, false);
  free_retired(ws);
  if (ws->host_counters) (void)hipHostFree(ws->host_counters);
  if (ws->notify_host) (void)hipHostFree(ws->notify_host);
  for (auto& e : ws->ev)
    if (e) (void)hipEventDestroy(e);
  if (ws->prep_done) (void)hipEventDestroy(ws->prep_done);
  if (ws->slot_free) (void)hipEventDestroy(ws->slot_free);
  if (ws->side) (void)hipStreamDestroy(ws->side);
  delete ws;
}

extern "C" const char* adr_last_error(void) { return g_error.c_str(); }

extern "C" const char* adr_version(void) { return "adr-gfx950 0.2"; }

namespace adr {
adr_status workspace_create(const adr_allocator* allocator, bool pipelined, adr_workspace** out) {
  if (!out) {
    set_error("adr_workspace_create: NULL argument");
    return ADR_E_INVALID;
  }
  *out = nullptr;
  if (allocator && (!allocator->alloc || !allocator->free)) {
    set_error("adr_workspace_create: an allocator needs both alloc and free");
    return ADR_E_INVALID;
  }
  adr_workspace* ws = new (std::nothrow) adr_workspace();
  if (!ws) {
    set_error("adr_workspace_create: host allocation failed");
    return ADR_E_OOM;
  }
  if (allocator) {
    ws->growth = Growth::kAllocator;
    ws->alloc = *allocator;
  }
  bool ok = hipHostMalloc(&ws->host_counters, kCounterSlots * sizeof(unsigned long long), hipHostMallocDefault) ==
                hipSuccess &&
            hipHostMalloc(&ws->notify_host, kNotifySlots * sizeof(unsigned long long),
                          hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess;
  if (ok) {
    std::memset(ws->host_counters, 0, kCounterSlots * sizeof(unsigned long long));
    std::memset(ws->notify_host, 0, kNotifySlots * sizeof(unsigned long long));
    ok = hipHostGetDevicePointer((void**)&ws->notify_dev, ws->notify_host, 0) == hipSuccess;
  }
  if (ok) {
    const size_t bytes = carve_fixed_arena(nullptr, nullptr);
    auto* p = static_cast<uint8_t*>(acquire(ws, bytes, nullptr));
    ok = p != nullptr;
    if (ok) {
      ws->fixed_arena = Arena{p, bytes};
      carve_fixed_arena(p, ws);
    }
  }
  if (!ok) {
    (void)hipGetLastError();
    free_workspace(ws);
    set_error("adr_workspace_create: allocation failed");
    return ADR_E_OOM;
  }
  for (int i = 0; i < adr_workspace::kEvents; ++i) {
    if (hipEventCreate(&ws->ev[i]) != hipSuccess) {
      (void)hipGetLastError();
      ws->ev[i] = nullptr;
      free_workspace(ws);
      set_error("adr_workspace_create: hipEventCreate failed");
      return ADR_E_HIP;
    }
  }
  if (pipelined) {
    ws->slots[0] = ws;
    for (int i = 1; i < adr_workspace::kFrameSlots; ++i) {
      adr_status st = workspace_create(allocator, false, &ws->slots[i]);
      if (st != ADR_OK) {
        free_workspace(ws);
        return st;
      }
    }
    bool ok2 = true;
    for (adr_workspace* s : ws->slots)  // default priority: every slot's early stages
      ok2 = ok2 && hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&s->prep_done, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&s->slot_free, hipEventDisableTiming) == hipSuccess;
    if (!ok2) {
      (void)hipGetLastError();
      free_workspace(ws);
      set_error("adr_workspace_create: could not create the side streams or their events");
      return ADR_E_HIP;
    }
  }
  *out = ws;
  return ADR_OK;
}
}  // namespace adr

extern "C" adr_status adr_workspace_create(const adr_allocator* allocator, adr_workspace** out) {
  return workspace_create(allocator, true, out);
}

extern "C" void adr_workspace_destroy(adr_workspace* ws) {
  if (!ws) return;
  (void)hipDeviceSynchronize();
  free_workspace(ws);
}

extern "C" int64_t adr_workspace_bytes(int64_t n_gauss, int64_t n_pairs, int64_t n_tiles) {
  if (n_gauss < 0 || n_pairs < 0 || n_tiles < 0) return -1;
  return (int64_t)(carve_gauss_arena(nullptr, n_gauss, nullptr) + carve_pair_arena(nullptr, n_pairs, nullptr) +
                   carve_tile_arena(nullptr, n_tiles, nullptr) + carve_fixed_arena(nullptr, nullptr));
}

extern "C" int64_t adr_workspace_capacity_bytes(const adr_workspace* ws) {
  if (!ws) return -1;
  size_t b = ws->gauss_arena.bytes + ws->pair_arena.bytes + ws->tile_arena.bytes + ws->fixed_arena.bytes +
             ws->grad_arena.bytes;
  for (const Arena& a : ws->retired) b += a.bytes;
  if (ws->slots[0] == ws)
    for (int i = 1; i < adr_workspace::kFrameSlots; ++i) b += (size_t)adr_workspace_capacity_bytes(ws->slots[i]);
  return (int64_t)b;
}

extern "C" adr_status adr_workspace_reserve(adr_workspace* ws, int64_t n_gauss, int64_t n_pairs, int64_t n_tiles) {
  if (!ws || n_gauss < 0 || n_pairs < 0 || n_tiles < 0) {
    set_error("adr_workspace_reserve: NULL workspace or negative size");
    return ADR_E_INVALID;
  }
  if (ws->growth == Growth::kNone) {
    set_error("adr_workspace_reserve: fixed-size workspace");
    return ADR_E_INVALID;
  }
  if (hipDeviceSynchronize() != hipSuccess) return hip_fail(hipGetLastError(), "adr_workspace_reserve");
  free_retired(ws);
  adr_status st;
  if ((st = grow_arena(ws, ws->gauss_arena, ws->gauss_capacity, n_gauss, carve_gauss_arena, false, false, nullptr,
                       "Gaussians")) != ADR_OK)
    return st;
  if ((st = grow_arena(ws, ws->pair_arena, ws->pair_capacity, n_pairs, carve_pair_arena, false, false, nullptr,
                       "pairs")) != ADR_OK)
    return st;
  if ((st = grow_arena(ws, ws->tile_arena, ws->tile_capacity, n_tiles, carve_tile_arena, false, false, nullptr,
                       "tiles")) != ADR_OK)
    return st;
  if (ws->slots[0] == ws)
    for (int i = 1; i < adr_workspace::kFrameSlots; ++i)
      if ((st = adr_workspace_reserve(ws->slots[i], n_gauss, n_pairs, n_tiles)) != ADR_OK) return st;
  return ADR_OK;
}

namespace adr {
adr_status validate_render_args(const adr_scene* scene, const adr_camera* cam, const adr_render_params* p,
                                const adr_frame* out) {
  if (!scene || !cam || !p || !out) {
    set_error("adr_render: NULL argument");
    return ADR_E_INVALID;
  }
  if (!out->image) {
    set_error("adr_render: frame.image is required");
    return ADR_E_INVALID;
  }
  if (cam->width < 1 || cam->height < 1 || cam->width > 65535 || cam->height > 65535) {
    set_error("adr_render: width and height must be in 1..65535");
    return ADR_E_INVALID;
  }
  if (!(cam->fx > 0) || !(cam->fy > 0) || !std::isfinite(cam->cx) || !std::isfinite(cam->cy) ||
      !(cam->near_z >= 0)) {
    set_error("adr_render: fx, fy must be > 0, cx, cy finite and near_z >= 0");
    return ADR_E_INVALID;
  }
  for (double v : cam->world_to_cam)
    if (!std::isfinite(v)) {
      set_error("adr_render: world_to_cam must be finite");
      return ADR_E_INVALID;
    }
  if (p->cull < ADR_CULL_3SIGMA || p->cull > ADR_CULL_AABB) {
    set_error("adr_render: unknown cull mode");
    return ADR_E_INVALID;
  }
  if (!(p->alpha_low > 0 && p->alpha_low < 1) || !(p->alpha_max > 0 && p->alpha_max < 1) ||
      !(p->alpha_low <= p->alpha_max) || !(p->t_min > 0 && p->t_min < 1) || !(p->lowpass >= 0) ||
      !(p->ewa_clamp > 0) || p->lb_cap < 0) {
    set_error("adr_render: parameter out of range (0<alpha_low<=alpha_max<1, 0<t_min<1, lowpass>=0, "
              "ewa_clamp>0, lb_cap>=0)");
    return ADR_E_INVALID;
  }
  if ((out->keys || out->values) && out->pair_capacity < 0) {
    set_error("adr_render: negative pair_capacity");
    return ADR_E_INVALID;
  }
  return ADR_OK;
}
}  // namespace adr

static adr_status validate(const adr_scene* scene, const adr_camera* cam, const adr_render_params* p,
                           const adr_frame* out, const adr_workspace* ws) {
  if (!ws) {
    set_error("adr_render: NULL argument");
    return ADR_E_INVALID;
  }
  return validate_render_args(scene, cam, p, out);
}

namespace {

CamArgs camera_args(const adr_camera* cam, const adr_render_params* p) {
  const int W = cam->width, H = cam->height;
  CamArgs ca{};
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) ca.r[3 * i + j] = cam->world_to_cam[4 * i + j];
    ca.t[i] = cam->world_to_cam[4 * i + 3];
  }
  for (int j = 0; j < 3; ++j)  // camera centre -R^T t
    ca.cam_pos[j] = -(ca.r[j] * ca.t[0] + ca.r[3 + j] * ca.t[1] + ca.r[6 + j] * ca.t[2]);
  ca.fx = cam->fx;
  ca.fy = cam->fy;
  ca.cx = cam->cx;
  ca.cy = cam->cy;
  ca.near_z = cam->near_z;
  ca.lim_x = p->ewa_clamp * (W / 2.0) / cam->fx;
  ca.lim_y = p->ewa_clamp * (H / 2.0) / cam->fy;
  ca.width = W;
  ca.height = H;
  ca.tiles_x = (W + kTile - 1) / kTile;
  ca.tiles_y = (H + kTile - 1) / kTile;
  return ca;
}

BlendArgs blend_args(const adr_render_params* p) {
  BlendArgs bl{};
  bl.alpha_max = (float)p->alpha_max;
  bl.t_min = (float)p->t_min;
  bl.q_low = (float)std::log2(p->alpha_low);
  // FP64 bands: each Gaussian's exponent band is its error bound plus 2^-19
  // (the rounding of log2(alpha_low) to float and of the comparison); the
  // transmittance band follows a running error bound per pixel.
  bl.exact = (p->flags & ADR_FLAG_NO_EXACT_BAND) ? 0 : 1;
  bl.band_floor = bl.exact ? 0x1p-19f : 0.f;
  bl.t_err_scale = bl.exact ? 1.5f : 0.f;  // margin over first-order terms left out of D
  bl.t_err_floor = bl.exact ? bl.t_min * 0x1p-21f : 0.f;  // t_min's rounding to float and the subtraction's
  bl.alpha_low_d = p->alpha_low;
  bl.alpha_max_d = p->alpha_max;
  bl.t_min_d = p->t_min;
  for (int c = 0; c < 3; ++c) bl.bg[c] = p->background[c];
  bl.lb_cap = p->lb_cap;
  return bl;
}

// Waits for the pair count, visible count and depth-key range of frame
// ws->frame_seq: spins on mapped host memory, or (fixed-memory workspace)
// copies the device words back and waits for the stream.
adr_status wait_notify(adr_workspace* ws, hipStream_t stream, unsigned long long v[kNotifySlots]) {
  if (ws->notify_host) {
    volatile unsigned long long* nf = ws->notify_host;
    const auto t0 = std::chrono::steady_clock::now();
    while (nf[2] != ws->frame_seq) {
      if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(200)) {
        // slow frame or a failed launch: fall back to the stream's status
        ADR_HIP(hipStreamSynchronize(stream));
        if (nf[2] != ws->frame_seq) {
          set_error("adr_render: Preprocess did not report the pair count");
          return ADR_E_HIP;
        }
        break;
      }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    for (int i = 0; i < kNotifySlots; ++i) v[i] = nf[i];
    return ADR_OK;
  }
  ADR_HIP(hipMemcpyAsync(v, ws->notify_slot, kNotifySlots * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                         stream));
  ADR_HIP(hipStreamSynchronize(stream));
  if (v[2] != ws->frame_seq) {
    set_error("adr_render: Preprocess did not report the pair count");
    return ADR_E_HIP;
  }
  return ADR_OK;
}

}  // namespace

namespace adr {

adr_status render_prepare(const adr_scene* scene, const adr_camera* cam, const adr_render_params* p,
                          adr_frame* out, adr_workspace* ws, hipStream_t stream, FramePlan& plan) {
  adr_status st;
  ws->last_vals = nullptr;  // no frame to differentiate until this one is enqueued whole
  const DeviceScene& s = scene->d;
  plan.cam = camera_args(cam, p);
  plan.n_tiles = (int64_t)plan.cam.tiles_x * plan.cam.tiles_y;
  plan.cull = CullArgs{};
  plan.cull.mode = p->cull;
  plan.cull.quad_cull = (p->flags & ADR_FLAG_NO_QUAD_CULL) ? 0 : 1;
  plan.cull.alpha_low = p->alpha_low;
  plan.cull.q_low = std::log2(p->alpha_low);
  plan.cull.lowpass = p->lowpass;
  plan.blend = blend_args(p);
  plan.want_load = out->load_sums != nullptr || out->load_stats != nullptr;
  const CamArgs& ca = plan.cam;
  const int64_t n_tiles = plan.n_tiles;

  if ((st = ensure_capacity(ws, s.n, 0, n_tiles, stream)) != ADR_OK) return st;
  const bool timing = (p->flags & ADR_FLAG_TIMING) != 0 && ws->ev[0] != nullptr;
  ws->timing_valid = false;
  ws->last_stream = stream;
  if (timing) ADR_HIP(hipEventRecord(ws->ev[0], stream));

  // Clear the frame's counters, load accumulators and tile ranges: in the
  // kernel that follows Preprocess when there is one and the ranges are small
  // enough, else with a launch of their own.
  const bool clear_in_notify = s.n > 0 && 2 * n_tiles <= kNotifyClearMax;
  if (!clear_in_notify) ADR_HIP(launch_frame_init(ws, n_tiles, stream));
  // Stage 1: Preprocess (+ pair total and visible count)
  ws->frame_seq += 1;
  ADR_HIP(launch_preprocess(s, ca, plan.cull, ws, clear_in_notify ? 2 * n_tiles : 0, stream));
  if (timing) ADR_HIP(hipEventRecord(ws->ev[1], stream));
  // The pair count sizes everything after this point.
  unsigned long long nv[kNotifySlots] = {};
  if (s.n > 0 && (st = wait_notify(ws, stream, nv)) != ADR_OK) return st;
  const unsigned long long n_pairs_u = nv[0], n_vis_u = nv[1], dmin = nv[3], dmax = nv[4];
  const int64_t n_vis = (int64_t)n_vis_u;
  if (timing) ADR_HIP(hipEventRecord(ws->ev[2], stream));
  if (n_pairs_u >= (1ull << 32)) {
    set_error("adr_render: 2^32 or more Gaussian-tile pairs in one frame");
    out->n_pairs = (int64_t)n_pairs_u;
    return ADR_E_UNSUPPORTED;
  }
  const int64_t n_pairs = (int64_t)n_pairs_u;
  out->n_pairs = n_pairs;
  plan.n_pairs = n_pairs;
  ws->last_pairs = n_pairs;
  if ((st = ensure_capacity(ws, s.n, n_pairs, n_tiles, stream)) != ADR_OK) return st;

  // Stage 4a: every Gaussian by its 32-bit depth key (ties keep id order);
  // the visible ones come first. Only the bits that vary over the visible
  // keys are sorted: key - dmin, with every larger key (the invisible ones'
  // all-ones key) clamped to lim, which is above every visible key.
  int dsorted = 0;  // which of the two buffers holds the result
  ws->last_depth_bits = 0;
  if (n_vis > 0) {
    if (dmax < dmin || dmax > 0xffffffffull || n_vis > s.n) {
      set_error("adr_render: inconsistent visible count or depth-key range from Preprocess");
      return ADR_E_HIP;
    }
    int dbits = bits_for((int64_t)(dmax - dmin) + 2);
    if (dbits > 32) dbits = 32;
    ws->last_depth_bits = dbits;
    const uint32_t lim = dbits >= 32 ? 0xffffffffu : (uint32_t)((1ull << dbits) - 1);
    // the last pass also lays tiles_touched out in depth order for the scan
    ADR_HIP(launch_radix_sort(ws->depth.keys, ws->depth.vals, s.n, dbits, (uint32_t)dmin, lim, ws->depth_scratch,
                              ws->hists, &dsorted, stream, ws->dev_counters + kCntBadIndex, ws->touched,
                              ws->touched_sorted, s.n));
    if (s.n == 1)  // nothing to sort: the one Gaussian is its own order
      ADR_HIP(hipMemcpyAsync(ws->touched_sorted, ws->touched, sizeof(uint32_t), hipMemcpyDeviceToDevice, stream));
  }
  const uint32_t* order = ws->depth.vals[dsorted];
  if (timing) ADR_HIP(hipEventRecord(ws->ev[3], stream));
  // Stage 2: InclusiveSum of tiles_touched over the Gaussians in depth order
  ADR_HIP(launch_inclusive_sum(ws->touched_sorted, ws->offsets, n_vis, ws->scan_partials, ws->dup_first, stream));
  if (timing) ADR_HIP(hipEventRecord(ws->ev[4], stream));
  // Stage 3: DuplicateWithKeys, in depth order, keyed by tile id
  ADR_HIP(launch_duplicate(ws->offsets, ws->dup_first, order, ws->tile_rect, n_vis, s.n, n_pairs, ca.tiles_x,
                           ws->pairs.keys[0], ws->pairs.vals[0], stream));
  if (timing) ADR_HIP(hipEventRecord(ws->ev[5], stream));
  // Stage 4b: stable sort by tile id; equal tiles keep the depth order
  int psorted = 0;
  ADR_HIP(launch_radix_sort(ws->pairs.keys, ws->pairs.vals, n_pairs, bits_for(n_tiles), 0u, 0xffffffffu,
                            ws->pair_scratch, ws->hists + kHistWords, &psorted, stream,
                            ws->dev_counters + kCntBadIndex));
  plan.tiles = ws->pairs.keys[psorted];
  plan.vals = ws->pairs.vals[psorted];
  if (timing) ADR_HIP(hipEventRecord(ws->ev[6], stream));
  // Stage 5: IdentifyTileRanges
  ADR_HIP(launch_tile_ranges(plan.tiles, n_pairs, ws->ranges, (int32_t)n_tiles, stream));
  if (timing) ADR_HIP(hipEventRecord(ws->ev[7], stream));
  // Stage 6, first part: the tiles' render order
  ADR_HIP(launch_tile_order(ws->ranges, n_pairs, plan.cam.tiles_x, plan.cam.tiles_y, ws->tile_order, ws->order_counts,
                            stream));
  if (timing) ADR_HIP(hipEventRecord(ws->ev[8], stream));
  return ADR_OK;
}

adr_status render_finish(const adr_scene* scene, const adr_camera* cam, const adr_render_params* p,
                         adr_frame* out, adr_workspace* ws, hipStream_t stream, const FramePlan& plan,
                         bool blend_launched) {
  const DeviceScene& s = scene->d;
  const bool timing = (p->flags & ADR_FLAG_TIMING) != 0 && ws->ev[0] != nullptr;
  if (timing) ADR_HIP(hipEventRecord(ws->ev[11], stream));
  if (!blend_launched)
    ADR_HIP(launch_render(ws->rec, ws->exact, plan.vals, ws->ranges, ws->tile_order, plan.n_pairs, s.n, plan.cam,
                          plan.blend, out, plan.want_load, ws, stream));
  ws->last_scene = scene;
  ws->last_scene_uid = scene->uid;
  ws->last_cam = *cam;
  ws->last_params = *p;
  ws->last_vals = plan.vals;
  if (timing) ADR_HIP(hipEventRecord(ws->ev[9], stream));
  if (plan.want_load)
    ADR_HIP(launch_load_sums(ws, (int)plan.n_tiles, (int64_t)cam->width * cam->height, out->load_sums,
                             out->load_stats, stream));
  if (timing) {
    ADR_HIP(hipEventRecord(ws->ev[10], stream));
    ws->timing_valid = true;
  }

  // Optional intermediate outputs.
  if (out->tiles_touched && s.n > 0)
    ADR_HIP(hipMemcpyAsync(out->tiles_touched, ws->touched, (size_t)s.n * sizeof(uint32_t),
                           hipMemcpyDeviceToDevice, stream));
  if (out->ranges)
    ADR_HIP(hipMemcpyAsync(out->ranges, ws->ranges, (size_t)plan.n_tiles * 2 * sizeof(uint32_t),
                           hipMemcpyDeviceToDevice, stream));
  if (out->keys || out->values) {
    if (plan.n_pairs > out->pair_capacity) {
      set_error("adr_render: pair_capacity smaller than the frame's pair count (see n_pairs)");
      return ADR_E_WORKSPACE;
    }
    if (out->keys) ADR_HIP(launch_compose_keys(plan.tiles, plan.vals, ws->rec, plan.n_pairs, s.n, out->keys, stream));
    if (out->values && plan.n_pairs > 0)
      ADR_HIP(hipMemcpyAsync(out->values, plan.vals, (size_t)plan.n_pairs * sizeof(uint32_t),
                             hipMemcpyDeviceToDevice, stream));
  }
  return ADR_OK;
}

}  // namespace adr

extern "C" adr_status adr_render(const adr_scene* scene, const adr_camera* cam, const adr_render_params* p,
                                 adr_frame* out, adr_workspace* ws, void* stream_ptr) {
  adr_status st = validate(scene, cam, p, out, ws);
  if (st != ADR_OK) return st;
  hipStream_t stream = (hipStream_t)stream_ptr;
  FramePlan plan;
  if (ws->slots[0] != ws) {
    ws->last_slot = ws;
    if ((st = render_prepare(scene, cam, p, out, ws, stream, plan)) != ADR_OK) return st;
    return render_finish(scene, cam, p, out, ws, stream, plan, false);
  }
  // Pipelined: the frame takes the next slot, and its stages up to the tile
  // order go to that slot's side stream when they depend on nothing the
  // caller's stream may still be changing (an owned scene: immutable; the
  // slot: free once its previous frame is done), so they overlap the early
  // stages and the blends of the frames before it. A borrowed scene (the
  // caller's arrays, which the caller may change between frames) runs every
  // stage on the caller's stream.
  adr_workspace* slot = ws->slots[ws->next_slot];
  ws->next_slot = (ws->next_slot + 1) % adr_workspace::kFrameSlots;
  ws->last_slot = slot;
  const bool overlap = !scene->d.borrowed;
  hipStream_t early = overlap ? slot->side : stream;
  ADR_HIP(hipStreamWaitEvent(early, slot->slot_free, 0));
  st = render_prepare(scene, cam, p, out, slot, early, plan);
  if (overlap) {  // the caller's stream takes over after the side stream's part (also after a failure)
    ADR_HIP(hipEventRecord(slot->prep_done, early));
    ADR_HIP(hipStreamWaitEvent(stream, slot->prep_done, 0));
  }
  if (st == ADR_OK) st = render_finish(scene, cam, p, out, slot, stream, plan, false);
  slot->last_stream = stream;  // where the frame's last work (and its counters) are
  // the slot is free again once everything enqueued for this frame is done
  ADR_HIP(hipEventRecord(slot->slot_free, stream));
  return st;
}

namespace {

bool same_camera(const adr_camera& a, const adr_camera& b) {
  for (int i = 0; i < 12; ++i)
    if (a.world_to_cam[i] != b.world_to_cam[i]) return false;
  return a.fx == b.fx && a.fy == b.fy && a.cx == b.cx && a.cy == b.cy && a.width == b.width &&
         a.height == b.height && a.near_z == b.near_z;
}

bool same_params(const adr_render_params& a, const adr_render_params& b) {
  return a.cull == b.cull && a.lb_cap == b.lb_cap && a.alpha_low == b.alpha_low && a.alpha_max == b.alpha_max &&
         a.t_min == b.t_min && a.lowpass == b.lowpass && a.ewa_clamp == b.ewa_clamp &&
         a.background[0] == b.background[0] && a.background[1] == b.background[1] &&
         a.background[2] == b.background[2] &&
         (a.flags & ADR_FLAG_NO_EXACT_BAND) == (b.flags & ADR_FLAG_NO_EXACT_BAND);
}

}  // namespace

extern "C" adr_status adr_render_backward_load(const adr_scene* scene, const adr_camera* cam,
                                               const adr_render_params* p, const adr_frame* fwd,
                                               const float* dl_dimage, const float* dl_dload,
                                               adr_scene_grads* grads, adr_workspace* ws, void* stream_ptr) {
  adr_status st = validate(scene, cam, p, fwd, ws);
  if (st != ADR_OK) return st;
  if (!dl_dimage || !grads || !fwd->final_t || !fwd->l_iter) {
    set_error("adr_render_backward: dl_dimage, grads, and the forward frame's final_t and l_iter are required");
    return ADR_E_INVALID;
  }
  adr_workspace* const handle = ws;
  if (ws->last_slot) ws = ws->last_slot;  // the frame slot of the last adr_render
  if (ws->last_scene != scene || ws->last_scene_uid != scene->uid || !same_camera(ws->last_cam, *cam) ||
      !same_params(ws->last_params, *p) || !ws->last_vals) {
    set_error("adr_render_backward: the last adr_render on this workspace was not this scene, camera and params");
    return ADR_E_INVALID;
  }
  hipStream_t stream = (hipStream_t)stream_ptr;
  const DeviceScene& s = scene->d;
  if (s.n == 0) return ADR_OK;
  if ((st = grow_arena(ws, ws->grad_arena, ws->grad_capacity, s.n, carve_grad_arena, true, true, stream,
                       "screen-space gradients")) != ADR_OK)
    return st;
  ADR_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(ws->grad2d), 0u, (int64_t)kGrad2d * s.n, stream));
  CamArgs ca = camera_args(cam, p);
  BlendArgs bl = blend_args(p);
  ADR_HIP(launch_render_backward(ws->rec, ws->exact, ws->last_vals, ws->ranges, ws->last_pairs, s.n, ca, bl,
                                 fwd->final_t, fwd->l_iter, dl_dimage, dl_dload, ws->grad2d, stream));
  ADR_HIP(launch_preprocess_backward(s, ca, p->lowpass, ws->grad2d, *grads, stream));
  if (handle->slots[0] == handle) ADR_HIP(hipEventRecord(ws->slot_free, stream));  // the slot's next frame waits for this
  return ADR_OK;
}

extern "C" adr_status adr_render_backward(const adr_scene* scene, const adr_camera* cam, const adr_render_params* p,
                                          const adr_frame* fwd, const float* dl_dimage, adr_scene_grads* grads,
                                          adr_workspace* ws, void* stream) {
  return adr_render_backward_load(scene, cam, p, fwd, dl_dimage, nullptr, grads, ws, stream);
}

extern "C" int32_t adr_workspace_stage_times(adr_workspace* ws, float* ms, int32_t n) {
  if (ws && ws->last_slot) ws = ws->last_slot;
  if (!ws || !ms || n <= 0 || !ws->timing_valid) return 0;
  if (hipEventSynchronize(ws->ev[10]) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  int32_t k = 0;
  for (; k < 10 && k < n; ++k) {
    float t = 0.f;
    // the blend from its own start: in a pipelined workspace it may wait for
    // the blend of the frame before after its tile order is ready
    const hipEvent_t from = k == 8 ? ws->ev[11] : ws->ev[k];
    if (hipEventElapsedTime(&t, from, ws->ev[k + 1]) != hipSuccess) {
      (void)hipGetLastError();
      t = -1.f;
    }
    ms[k] = t;
  }
  return k;
}

extern "C" int32_t adr_workspace_counters(adr_workspace* ws, int64_t* out, int32_t n) {
  if (ws && ws->last_slot) ws = ws->last_slot;
  if (!ws || !out || n <= 0 || !ws->dev_counters) return 0;
  if (hipStreamSynchronize(ws->last_stream) != hipSuccess ||
      hipMemcpy(ws->host_counters, ws->dev_counters, kCounterSlots * sizeof(unsigned long long),
                hipMemcpyDeviceToHost) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  const int idx[6] = {kCntPairs, kCntVisible, kCntBand, kCntReplay, -1, kCntBadIndex};
  int32_t k = 0;
  for (; k < 6 && k < n; ++k) out[k] = idx[k] >= 0 ? (int64_t)ws->host_counters[idx[k]] : ws->last_depth_bits;
  return k;
}
