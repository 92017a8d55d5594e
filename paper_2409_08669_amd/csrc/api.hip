// C ABI: workspace management and the per-frame orchestration of the six
// stages of Sec. 3.2 on the caller's stream.
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

template <typename T>
adr_status grow(T*& p, int64_t& cap, int64_t need, const char* what) {
  if (need <= cap && p) return ADR_OK;
  int64_t n = need < 1 ? 1 : need;
  n = n + n / 4;  // headroom so that frame-to-frame jitter does not reallocate
  if (p) (void)hipFree(p);
  p = nullptr;
  cap = 0;
  if (hipMalloc(&p, (size_t)n * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    set_error(std::string("workspace allocation failed: ") + what);
    return ADR_E_OOM;
  }
  cap = n;
  return ADR_OK;
}

adr_status ensure_sort_buffers(SortBuffers& sb, int64_t n, const char* what) {
  if (n <= sb.capacity && sb.keys[0]) return ADR_OK;
  int64_t c[4] = {sb.capacity, sb.capacity, sb.capacity, sb.capacity};
  adr_status st;
  if ((st = grow(sb.keys[0], c[0], n, what)) != ADR_OK) return st;
  if ((st = grow(sb.keys[1], c[1], n, what)) != ADR_OK) return st;
  if ((st = grow(sb.vals[0], c[2], n, what)) != ADR_OK) return st;
  if ((st = grow(sb.vals[1], c[3], n, what)) != ADR_OK) return st;
  int64_t m = c[0];
  for (int i = 1; i < 4; ++i) m = c[i] < m ? c[i] : m;
  sb.capacity = m;
  return ADR_OK;
}

adr_status ensure_gauss(adr_workspace* ws, int64_t n) {
  adr_status st;
  if (n > ws->gauss_capacity || !ws->rec) {
    int64_t c[4] = {ws->gauss_capacity, ws->gauss_capacity, ws->gauss_capacity, ws->gauss_capacity};
    int64_t c5 = ws->gauss_capacity;
    if ((st = grow(ws->rec, c[0], n, "records")) != ADR_OK) return st;
    if ((st = grow(ws->exact, c[1], n, "exact records")) != ADR_OK) return st;
    if ((st = grow(ws->tile_rect, c[2], n, "tile rects")) != ADR_OK) return st;
    if ((st = grow(ws->touched, c[3], n, "tiles_touched")) != ADR_OK) return st;
    if ((st = grow(ws->offsets, c5, n, "offsets")) != ADR_OK) return st;
    int64_t c6 = ws->gauss_capacity;
    if ((st = grow(ws->touched_sorted, c6, n, "tiles_touched in depth order")) != ADR_OK) return st;
    int64_t m = c5 < c6 ? c5 : c6;
    for (int i = 0; i < 4; ++i) m = c[i] < m ? c[i] : m;
    ws->gauss_capacity = m;
  }
  if ((st = ensure_sort_buffers(ws->depth, n, "depth sort")) != ADR_OK) return st;
  if ((st = grow(ws->sort_scratch, ws->sort_scratch_capacity, sort_scratch_entries(n), "sort scratch")) != ADR_OK)
    return st;
  if ((st = grow(ws->block_parts, ws->block_parts_capacity, preprocess_blocks(n), "preprocess partials")) != ADR_OK)
    return st;
  return grow(ws->scan_partials, ws->scan_partials_capacity, inclusive_sum_partials(n) + 1, "scan partials");
}

adr_status ensure_pairs(adr_workspace* ws, int64_t p) {
  adr_status st;
  if ((st = ensure_sort_buffers(ws->pairs, p, "pair sort")) != ADR_OK) return st;
  if ((st = grow(ws->dup_first, ws->dup_first_capacity, duplicate_blocks(p) + 1, "pair chunk starts")) != ADR_OK)
    return st;
  return grow(ws->sort_scratch, ws->sort_scratch_capacity, sort_scratch_entries(p), "sort scratch");
}

int bits_for(int64_t v) {
  int b = 0;
  while (((int64_t)1 << b) < v) ++b;
  return b;
}

}  // namespace
}  // namespace adr

using namespace adr;

static void free_workspace_buffers(adr_workspace* ws) {
  void* bufs[] = {ws->rec, ws->exact, ws->tile_rect, ws->touched, ws->offsets, ws->touched_sorted, ws->depth.keys[0],
                  ws->depth.keys[1], ws->depth.vals[0], ws->depth.vals[1], ws->scan_partials, ws->pairs.keys[0],
                  ws->pairs.keys[1], ws->pairs.vals[0], ws->pairs.vals[1], ws->dup_first, ws->sort_scratch, ws->ranges,
                  ws->tile_order, ws->order_counts, ws->wave_sums, ws->dev_counters, ws->hists, ws->block_parts};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  if (ws->host_counters) (void)hipHostFree(ws->host_counters);
  if (ws->notify_host) (void)hipHostFree(ws->notify_host);
}

extern "C" const char* adr_last_error(void) { return g_error.c_str(); }

extern "C" const char* adr_version(void) { return "adr-gfx950 0.1"; }

extern "C" adr_status adr_workspace_create(adr_workspace** out) {
  if (!out) {
    set_error("adr_workspace_create: NULL argument");
    return ADR_E_INVALID;
  }
  *out = nullptr;
  adr_workspace* ws = new (std::nothrow) adr_workspace();
  if (!ws) {
    set_error("adr_workspace_create: host allocation failed");
    return ADR_E_OOM;
  }
  bool ok = hipMalloc(&ws->dev_counters, kCounterSlots * sizeof(unsigned long long)) == hipSuccess &&
            hipMalloc(&ws->hists, 2 * kHistWords * sizeof(uint32_t)) == hipSuccess &&
            hipHostMalloc(&ws->host_counters, kCounterSlots * sizeof(unsigned long long), hipHostMallocDefault) ==
                hipSuccess &&
            hipHostMalloc(&ws->notify_host, kNotifySlots * sizeof(unsigned long long),
                          hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess;
  if (ok) {
    std::memset(ws->host_counters, 0, kCounterSlots * sizeof(unsigned long long));
    std::memset(ws->notify_host, 0, kNotifySlots * sizeof(unsigned long long));
    ok = hipHostGetDevicePointer((void**)&ws->notify_dev, ws->notify_host, 0) == hipSuccess;
  }
  if (!ok) {
    (void)hipGetLastError();
    free_workspace_buffers(ws);
    delete ws;
    set_error("adr_workspace_create: allocation failed");
    return ADR_E_OOM;
  }
  for (int i = 0; i < adr_workspace::kEvents; ++i) {
    if (hipEventCreate(&ws->ev[i]) != hipSuccess) {
      (void)hipGetLastError();
      set_error("adr_workspace_create: hipEventCreate failed");
      for (int k = 0; k < i; ++k) (void)hipEventDestroy(ws->ev[k]);
      free_workspace_buffers(ws);
      delete ws;
      return ADR_E_HIP;
    }
  }
  *out = ws;
  return ADR_OK;
}

extern "C" void adr_workspace_destroy(adr_workspace* ws) {
  if (!ws) return;
  (void)hipDeviceSynchronize();
  free_workspace_buffers(ws);
  for (auto& e : ws->ev)
    if (e) (void)hipEventDestroy(e);
  delete ws;
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

}  // namespace

extern "C" adr_status adr_render(const adr_scene* scene, const adr_camera* cam, const adr_render_params* p,
                                 adr_frame* out, adr_workspace* ws, void* stream_ptr) {
  adr_status st = validate(scene, cam, p, out, ws);
  if (st != ADR_OK) return st;
  ws->last_vals = nullptr;  // no frame to differentiate until this one is enqueued whole
  hipStream_t stream = (hipStream_t)stream_ptr;
  const DeviceScene& s = scene->d;
  const int W = cam->width, H = cam->height;

  CamArgs ca = camera_args(cam, p);
  const int64_t n_tiles = (int64_t)ca.tiles_x * ca.tiles_y;

  CullArgs cu{};
  cu.mode = p->cull;
  cu.quad_cull = (p->flags & ADR_FLAG_NO_QUAD_CULL) ? 0 : 1;
  cu.alpha_low = p->alpha_low;
  cu.q_low = std::log2(p->alpha_low);
  cu.lowpass = p->lowpass;

  BlendArgs bl = blend_args(p);

  if ((st = ensure_gauss(ws, s.n)) != ADR_OK) return st;
  if ((st = grow(ws->ranges, ws->ranges_capacity, 2 * n_tiles, "ranges")) != ADR_OK) return st;
  if ((st = grow(ws->tile_order, ws->tile_order_capacity, n_tiles, "tile order")) != ADR_OK) return st;
  if ((st = grow(ws->order_counts, ws->order_counts_capacity, tile_order_scratch((int)n_tiles), "tile order counts")) !=
      ADR_OK)
    return st;
  if ((st = grow(ws->wave_sums, ws->wave_sums_capacity, 16 * n_tiles, "load-sum partials")) != ADR_OK) return st;
  const bool timing = (p->flags & ADR_FLAG_TIMING) != 0;
  ws->timing_valid = false;
  ws->last_stream = stream;
  if (timing) ADR_HIP(hipEventRecord(ws->ev[0], stream));

  // Clear the frame's counters, load sums and tile ranges: in the kernel that
  // follows Preprocess when there is one and the ranges are small enough,
  // else with a launch of their own.
  const bool clear_in_notify = s.n > 0 && 2 * n_tiles <= kNotifyClearMax;
  if (!clear_in_notify) ADR_HIP(launch_frame_init(ws, n_tiles, out->load_sums, stream));
  // Stage 1: Preprocess (+ pair total and visible count)
  ws->frame_seq += 1;
  ADR_HIP(launch_preprocess(s, ca, cu, ws, clear_in_notify ? 2 * n_tiles : 0, out->load_sums, stream));
  if (timing) ADR_HIP(hipEventRecord(ws->ev[1], stream));
  // The pair count sizes everything after this point. The last Preprocess
  // workgroup writes it to mapped host memory; wait for this frame's number.
  unsigned long long n_pairs_u = 0, n_vis_u = 0, dmin = 0, dmax = 0;
  if (s.n > 0) {
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
    n_pairs_u = nf[0];
    n_vis_u = nf[1];
    dmin = nf[3];
    dmax = nf[4];
  }
  const int64_t n_vis = (int64_t)n_vis_u;
  if (timing) ADR_HIP(hipEventRecord(ws->ev[2], stream));
  if (n_pairs_u >= (1ull << 32)) {
    set_error("adr_render: 2^32 or more Gaussian-tile pairs in one frame");
    out->n_pairs = (int64_t)n_pairs_u;
    return ADR_E_UNSUPPORTED;
  }
  const int64_t n_pairs = (int64_t)n_pairs_u;
  out->n_pairs = n_pairs;
  ws->last_pairs = n_pairs;
  if ((st = ensure_pairs(ws, n_pairs)) != ADR_OK) return st;

  // Stage 4a: every Gaussian by its 32-bit depth key (ties keep id order);
  // the visible ones come first. Only the bits that vary over the visible
  // keys are sorted: key - dmin, with every larger key (the invisible ones'
  // all-ones key) clamped to lim, which is above every visible key.
  int dsorted = 0;  // which of the two buffers holds the result
  ws->last_depth_bits = 0;
  if (n_vis > 0) {
    if (dmax < dmin || dmax > 0xffffffffull) {
      set_error("adr_render: inconsistent depth-key range from Preprocess");
      return ADR_E_HIP;
    }
    int dbits = bits_for((int64_t)(dmax - dmin) + 2);
    if (dbits > 32) dbits = 32;
    ws->last_depth_bits = dbits;
    const uint32_t lim = dbits >= 32 ? 0xffffffffu : (uint32_t)((1ull << dbits) - 1);
    // the last pass also lays tiles_touched out in depth order for the scan
    ADR_HIP(launch_radix_sort(ws->depth.keys, ws->depth.vals, s.n, dbits, (uint32_t)dmin, lim, ws->sort_scratch,
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
                            ws->sort_scratch, ws->hists + kHistWords, &psorted, stream,
                            ws->dev_counters + kCntBadIndex));
  const uint32_t* tiles = ws->pairs.keys[psorted];
  const uint32_t* vals = ws->pairs.vals[psorted];
  if (timing) ADR_HIP(hipEventRecord(ws->ev[6], stream));
  // Stage 5: IdentifyTileRanges
  ADR_HIP(launch_tile_ranges(tiles, n_pairs, ws->ranges, (int32_t)n_tiles, stream));
  if (timing) ADR_HIP(hipEventRecord(ws->ev[7], stream));
  // Stage 6: Render (tile order, blend, load sums)
  ADR_HIP(launch_tile_order(ws->ranges, n_pairs, (int)n_tiles, ws->tile_order, ws->order_counts, stream));
  if (timing) ADR_HIP(hipEventRecord(ws->ev[8], stream));
  ADR_HIP(launch_render(ws->rec, ws->exact, vals, ws->ranges, ws->tile_order, n_pairs, s.n, ca, bl, out, ws,
                        stream));
  ws->last_scene = scene;
  ws->last_scene_uid = scene->uid;
  ws->last_cam = *cam;
  ws->last_params = *p;
  ws->last_vals = vals;
  if (timing) ADR_HIP(hipEventRecord(ws->ev[9], stream));
  ADR_HIP(launch_load_sums(ws, (int)n_tiles, out->load_sums, stream));
  if (timing) {
    ADR_HIP(hipEventRecord(ws->ev[10], stream));
    ws->timing_valid = true;
  }

  // Optional intermediate outputs.
  if (out->tiles_touched && s.n > 0)
    ADR_HIP(hipMemcpyAsync(out->tiles_touched, ws->touched, (size_t)s.n * sizeof(uint32_t),
                           hipMemcpyDeviceToDevice, stream));
  if (out->ranges)
    ADR_HIP(hipMemcpyAsync(out->ranges, ws->ranges, (size_t)n_tiles * 2 * sizeof(uint32_t),
                           hipMemcpyDeviceToDevice, stream));
  if (out->keys || out->values) {
    if (n_pairs > out->pair_capacity) {
      set_error("adr_render: pair_capacity smaller than the frame's pair count (see n_pairs)");
      return ADR_E_WORKSPACE;
    }
    if (out->keys) ADR_HIP(launch_compose_keys(tiles, vals, ws->rec, n_pairs, s.n, out->keys, stream));
    if (out->values && n_pairs > 0)
      ADR_HIP(hipMemcpyAsync(out->values, vals, (size_t)n_pairs * sizeof(uint32_t), hipMemcpyDeviceToDevice,
                             stream));
  }
  return ADR_OK;
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
  if (ws->last_scene != scene || ws->last_scene_uid != scene->uid || !same_camera(ws->last_cam, *cam) ||
      !same_params(ws->last_params, *p) ||
      !ws->last_vals) {
    set_error("adr_render_backward: the last adr_render on this workspace was not this scene, camera and params");
    return ADR_E_INVALID;
  }
  hipStream_t stream = (hipStream_t)stream_ptr;
  const DeviceScene& s = scene->d;
  if (s.n == 0) return ADR_OK;
  if ((st = grow(ws->grad2d, ws->grad2d_capacity, (int64_t)kGrad2d * s.n, "screen-space gradients")) != ADR_OK)
    return st;
  ADR_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(ws->grad2d), 0u, (int64_t)kGrad2d * s.n, stream));
  CamArgs ca = camera_args(cam, p);
  BlendArgs bl = blend_args(p);
  ADR_HIP(launch_render_backward(ws->rec, ws->exact, ws->last_vals, ws->ranges, ws->last_pairs, s.n, ca, bl,
                                 fwd->final_t, fwd->l_iter, dl_dimage, dl_dload, ws->grad2d, stream));
  ADR_HIP(launch_preprocess_backward(s, ca, p->lowpass, ws->grad2d, *grads, stream));
  return ADR_OK;
}

extern "C" adr_status adr_render_backward(const adr_scene* scene, const adr_camera* cam, const adr_render_params* p,
                                          const adr_frame* fwd, const float* dl_dimage, adr_scene_grads* grads,
                                          adr_workspace* ws, void* stream) {
  return adr_render_backward_load(scene, cam, p, fwd, dl_dimage, nullptr, grads, ws, stream);
}

extern "C" int32_t adr_workspace_stage_times(adr_workspace* ws, float* ms, int32_t n) {
  if (!ws || !ms || n <= 0 || !ws->timing_valid) return 0;
  if (hipEventSynchronize(ws->ev[adr_workspace::kEvents - 1]) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  int32_t k = 0;
  for (; k < adr_workspace::kEvents - 1 && k < n; ++k) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, ws->ev[k], ws->ev[k + 1]) != hipSuccess) {
      (void)hipGetLastError();
      t = -1.f;
    }
    ms[k] = t;
  }
  return k;
}

extern "C" int32_t adr_workspace_counters(adr_workspace* ws, int64_t* out, int32_t n) {
  if (!ws || !out || n <= 0) return 0;
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
