// Internal declarations of the gfx950 rasterizer library: device layouts,
// launch helpers and the host-side objects behind the opaque C handles.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/adr.h"

namespace adr {

constexpr int kTile = 16;     // 16 x 16 pixel tiles (Sec. 3.2)
constexpr int kDupPairs = 2048;  // pairs emitted per DuplicateWithKeys workgroup
constexpr int kQuad = 8;      // each wave of a tile's workgroup owns an 8 x 8 quadrant
constexpr int kWave = 64;     // CDNA wavefront

// ---------------------------------------------------------------------------
// Scene in device memory (structure of arrays, coalesced per Gaussian index)
// ---------------------------------------------------------------------------
struct DeviceScene {
  int64_t n = 0;
  int32_t sh_degree = 0;
  int32_t n_coeff = 1;       // (degree+1)^2
  float4* geo_a = nullptr;   // (mean.x, mean.y, mean.z, opacity logit)
  float4* geo_b = nullptr;   // (log_scale.x, .y, .z, 0)
  float4* geo_q = nullptr;   // quaternion (w, x, y, z), as given
  float* sh = nullptr;       // planes [3*K][n]: plane (k*3 + channel)
  size_t bytes = 0;
};

// ---------------------------------------------------------------------------
// Per-Gaussian outputs of Preprocess
// ---------------------------------------------------------------------------
// Render record, 64 bytes, read by the blend kernel through the sorted ids.
// The splatting opacity (Eq. 2) in the log2 domain, on the principal axes of
// the conic:
//   q = ql - a1 u^2 - a2 v^2,  u = rc dx - rs dy,  v = rs dx + rc dy,
//   alpha = min(alpha_max, 2^q),
// with ql = log2(opacity), (a1, a2) the eigenvalues of (log2(e) / 2) conic
// and dx = x - i, dy = y - j for pixel (i, j).
struct alignas(16) RenderRecord {
  uint32_t box_x;         // lo | hi << 16: pixel columns that may have alpha >= alpha_low
  uint32_t box_y;         // lo | hi << 16: pixel rows (lo > hi: none)
  uint32_t depth_key;     // bits of the fp32 view-space depth
  float ql;
  double x, y;            // projected centre, pixel centres at integers
  float rc, rs, a1, a2;
  float r, g, b;
  float dq;               // bound on the FP32 error of q where it matters (+inf: decide in FP64)
};
static_assert(sizeof(RenderRecord) == 64, "render record is four 16-byte loads");

// FP64 values for exact decisions near alpha_low and t_min.
struct alignas(16) ExactRecord {
  double ca, cb, cc;      // conic = Sigma'^-1 (a, b, c)
  double opacity;
};

// ---------------------------------------------------------------------------
// Camera and parameters as kernel arguments
// ---------------------------------------------------------------------------
struct CamArgs {
  double r[9];
  double t[3];
  double cam_pos[3];
  double fx, fy, cx, cy;
  double near_z;
  double lim_x, lim_y;      // EWA clamp of x/z and y/z
  int32_t width, height;
  int32_t tiles_x, tiles_y;
};

struct CullArgs {
  int32_t mode;
  int32_t quad_cull;        // render-side 8 x 8 quadrant cull in the culling modes
  double alpha_low;
  double q_low;             // log2(alpha_low)
  double lowpass;
};

struct BlendArgs {
  float alpha_max;
  float t_min;
  float q_low;              // log2(alpha_low) rounded to float
  float band_floor;         // added to each Gaussian's exponent error bound (0: no FP64 bands)
  // FP64 transmittance replay when |T - t_min| < t_err_scale D + t_err_floor,
  // D the running bound on |T - T_fp64|; both 0: no replays
  float t_err_scale, t_err_floor;
  double alpha_low_d, alpha_max_d, t_min_d;
  float bg[3];
  int32_t lb_cap;
  int32_t exact;
};

// ---------------------------------------------------------------------------
// Host objects behind the opaque handles
// ---------------------------------------------------------------------------
struct SortBuffers {
  uint32_t* keys[2] = {nullptr, nullptr};
  uint32_t* vals[2] = {nullptr, nullptr};
  int64_t capacity = 0;
};

}  // namespace adr

struct adr_scene {
  adr::DeviceScene d;
  uint64_t uid = 0;  // unique per created scene in this process (a freed scene's address may be reused)
};

struct adr_workspace {
  // per Gaussian
  int64_t gauss_capacity = 0;
  adr::RenderRecord* rec = nullptr;
  adr::ExactRecord* exact = nullptr;
  uint2* tile_rect = nullptr;      // (tx_lo | tx_hi << 16, ty_lo | ty_hi << 16)
  uint32_t* touched = nullptr;
  uint32_t* offsets = nullptr;     // inclusive sum of touched in depth order
  uint32_t* touched_sorted = nullptr;  // tiles_touched in depth order
  adr::SortBuffers depth;          // (depth key, id) of every Gaussian, sorted by depth
  uint32_t* scan_partials = nullptr;
  int64_t scan_partials_capacity = 0;
  // per DuplicateWithKeys workgroup (kDupPairs pairs): the depth-order index
  // of the Gaussian that holds its first pair, written by the InclusiveSum
  uint32_t* dup_first = nullptr;
  int64_t dup_first_capacity = 0;
  ulonglong4* block_parts = nullptr;  // per Preprocess workgroup: pairs, visible, depth-key min, max
  int64_t block_parts_capacity = 0;
  // per pair
  adr::SortBuffers pairs;          // (tile id, Gaussian id), sorted by tile
  uint32_t* sort_scratch = nullptr;
  int64_t sort_scratch_capacity = 0;
  // per tile
  uint32_t* ranges = nullptr;      // 2 * tiles
  int64_t ranges_capacity = 0;
  uint32_t* tile_order = nullptr;  // render order of the tiles, longest lists first
  int64_t tile_order_capacity = 0;
  uint32_t* order_counts = nullptr;  // per-block bucket counts of the tile order
  int64_t order_counts_capacity = 0;
  // per frame: counters and the two sort histograms, zeroed (with the tile
  // ranges and the caller's load sums) by one kernel at the start of the frame
  unsigned long long* dev_counters = nullptr;  // kCounterSlots u64, see below
  uint32_t* hists = nullptr;                   // 2 x kHistWords: depth sort, tile sort
  unsigned long long* wave_sums = nullptr;     // 4 x u64 per render wave (load-sum partials)
  int64_t wave_sums_capacity = 0;
  unsigned long long* host_counters = nullptr; // pinned copy for adr_workspace_counters
  // mapped pinned memory the Preprocess kernel writes the pair count into
  unsigned long long* notify_host = nullptr;
  unsigned long long* notify_dev = nullptr;
  unsigned long long frame_seq = 0;
  static constexpr int kEvents = 11;
  hipEvent_t ev[kEvents] = {};
  bool timing_valid = false;
  hipStream_t last_stream = nullptr;
  int64_t last_pairs = 0;
  int32_t last_depth_bits = 0;  // key bits the last frame's depth sort covered
  // the last frame rendered on this workspace (what adr_render_backward differentiates)
  const adr_scene* last_scene = nullptr;
  uint64_t last_scene_uid = 0;
  adr_camera last_cam{};
  adr_render_params last_params{};
  const uint32_t* last_vals = nullptr;  // its sorted Gaussian ids
  float* grad2d = nullptr;              // kGrad2d floats per Gaussian
  int64_t grad2d_capacity = 0;
};

namespace adr {

// dev_counters slots
constexpr int kCntPairs = 0;       // sum of tiles_touched (u64)
constexpr int kCntVisible = 1;     // Gaussians with tiles_touched > 0
constexpr int kCntBand = 2;        // FP64 re-decisions near alpha_low
constexpr int kCntReplay = 3;      // FP64 transmittance replays near t_min
constexpr int kCntDepthMin = 4;    // smallest depth key of a visible Gaussian
constexpr int kCntDepthMax = 5;    // largest depth key of a visible Gaussian
constexpr int kCntBadIndex = 6;    // sort values or positions out of range (0 unless a kernel is wrong)
constexpr int kNotifySlots = 8;    // mapped words: pairs, visible, frame number, depth min, depth max
constexpr int kCounterSlots = 8;
constexpr int kHistWords = 4 * 256;  // digit histograms of up to four 8-bit passes

// Thread-local error message for adr_last_error.
void set_error(const std::string& msg);
// Host-side checks of adr_render's arguments (everything but the workspace).
adr_status validate_render_args(const adr_scene* scene, const adr_camera* cam, const adr_render_params* p,
                                const adr_frame* out);
adr_status hip_fail(hipError_t e, const char* what);

#define ADR_HIP(call)                                          \
  do {                                                         \
    hipError_t _e = (call);                                    \
    if (_e != hipSuccess) return ::adr::hip_fail(_e, #call);   \
  } while (0)

// Launchers (each enqueues on `stream`, returns hipSuccess or the error).
hipError_t launch_pack_scene(const adr_scene_desc& desc, const float* means, const float* log_scales,
                             const float* quats, const float* logits, const float* sh, DeviceScene& d,
                             hipStream_t stream);
hipError_t launch_frame_init(adr_workspace* ws, int64_t n_tiles, uint64_t* load_sums, hipStream_t stream);
int64_t preprocess_blocks(int64_t n);
// Frames whose tile ranges have at most this many words have them cleared
// (with the counters and the load sums) by the kernel that follows
// Preprocess instead of a launch of their own.
constexpr int64_t kNotifyClearMax = (int64_t)1 << 17;
// n_ranges, load_sums: what the frame-init launch clears, cleared here when
// 0 < n_ranges <= kNotifyClearMax (n_ranges = 0: nothing is cleared)
hipError_t launch_preprocess(const DeviceScene& s, const CamArgs& cam, const CullArgs& cull, adr_workspace* ws,
                             int64_t n_ranges, uint64_t* load_sums, hipStream_t stream);
hipError_t launch_inclusive_sum(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* partials,
                                uint32_t* dup_first, hipStream_t stream);
int64_t inclusive_sum_partials(int64_t n);
int64_t duplicate_blocks(int64_t n_pairs);
hipError_t launch_duplicate(const uint32_t* offsets, const uint32_t* dup_first, const uint32_t* order,
                            const uint2* tile_rect, int64_t n_vis, int64_t n_gauss, int64_t n_pairs, int32_t tiles_x,
                            uint32_t* tile_keys, uint32_t* vals, hipStream_t stream);
hipError_t launch_radix_sort(uint32_t* keys[2], uint32_t* vals[2], int64_t n, int n_bits, uint32_t bias,
                             uint32_t lim, uint32_t* scratch, uint32_t* totals, int* result_buffer,
                             hipStream_t stream, unsigned long long* bad_count,
                             const uint32_t* gather_src = nullptr, uint32_t* gather_dst = nullptr,
                             int64_t gather_n = 0);
int64_t sort_scratch_entries(int64_t n);
hipError_t launch_tile_ranges(const uint32_t* tiles, int64_t n_pairs, uint32_t* ranges, int32_t n_tiles,
                              hipStream_t stream);
hipError_t launch_compose_keys(const uint32_t* tiles, const uint32_t* vals, const RenderRecord* rec,
                               int64_t n_pairs, int64_t n_gauss, uint64_t* keys, hipStream_t stream);
int64_t tile_order_scratch(int n_tiles);
hipError_t launch_tile_order(const uint32_t* ranges, int64_t n_pairs, int n_tiles, uint32_t* order, uint32_t* counts,
                             hipStream_t stream);
hipError_t launch_render(const RenderRecord* rec, const ExactRecord* exact, const uint32_t* vals,
                         const uint32_t* ranges, const uint32_t* order, int64_t n_pairs, int64_t n_gauss,
                         const CamArgs& cam, const BlendArgs& blend, adr_frame* out, adr_workspace* ws,
                         hipStream_t stream);
hipError_t launch_load_sums(adr_workspace* ws, int n_tiles, uint64_t* load_sums, hipStream_t stream);
// Backward (gradients). Screen-space gradients per Gaussian, kGrad2d floats:
// d/dx, d/dy, d/d conic (A, B, C), d/d opacity, d/d colour (r, g, b), unused.
constexpr int kGrad2d = 10;
hipError_t launch_render_backward(const RenderRecord* rec, const ExactRecord* exact, const uint32_t* vals,
                                  const uint32_t* ranges, int64_t n_pairs, int64_t n_gauss, const CamArgs& cam,
                                  const BlendArgs& blend, const float* final_t, const uint32_t* l_iter,
                                  const float* dl_dimage, const float* dl_dload, float* grad2d,
                                  hipStream_t stream);
hipError_t launch_preprocess_backward(const DeviceScene& s, const CamArgs& cam, double lowpass, const float* grad2d,
                                      const adr_scene_grads& out, hipStream_t stream);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t stream);
hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, int64_t n, hipStream_t stream);

}  // namespace adr
