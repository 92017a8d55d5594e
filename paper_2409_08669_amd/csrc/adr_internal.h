// Internal declarations of the gfx950 rasterizer library: device layouts,
// launch helpers and the host-side objects behind the opaque C handles.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/adr.h"

namespace adr {

constexpr int kTile = 16;     // 16 x 16 pixel tiles (Sec. 3.2)
constexpr int kDupPairs = 2048;  // pairs emitted per DuplicateWithKeys workgroup
constexpr int kQuad = 8;      // each wave of a tile's workgroup owns an 8 x 8 quadrant
constexpr int kWave = 64;     // CDNA wavefront

// ---------------------------------------------------------------------------
// Scene in device memory
// ---------------------------------------------------------------------------
// An owned scene is a structure of arrays, coalesced per Gaussian index: three
// float4 planes and 3K SH planes. A borrowed scene is the caller's row-major
// arrays, read in place.
struct DeviceScene {
  int64_t n = 0;
  int32_t sh_degree = 0;
  int32_t n_coeff = 1;       // (degree+1)^2
  bool borrowed = false;
  // owned layout
  float4* geo_a = nullptr;   // (mean.x, mean.y, mean.z, opacity logit)
  float4* geo_b = nullptr;   // (log_scale.x, .y, .z, 0)
  float4* geo_q = nullptr;   // quaternion (w, x, y, z), as given
  float* sh = nullptr;       // planes [3*K][n]: plane (k*3 + channel)
  // borrowed layout (adr_scene_desc's arrays)
  const float* means = nullptr;
  const float* log_scales = nullptr;
  const float* quats = nullptr;
  const float* logits = nullptr;
  const float* sh_rows = nullptr;  // N x K x 3
  size_t bytes = 0;
};

// Device reads of one Gaussian's inputs, for either scene layout. Entry i of
// the SH coefficients is coefficient i / 3, channel i % 3.
struct PlanarScene {
  const float4* __restrict__ geo_a;
  const float4* __restrict__ geo_b;
  const float4* __restrict__ geo_q;
  const float* __restrict__ sh;
  int64_t n;
  __device__ float4 a(int64_t g) const { return geo_a[g]; }
  __device__ float4 b(int64_t g) const { return geo_b[g]; }
  __device__ float4 q(int64_t g) const { return geo_q[g]; }
  __device__ float coef(int i, int64_t g) const { return sh[(int64_t)i * n + g]; }
};

struct RowMajorScene {
  const float* __restrict__ means;
  const float* __restrict__ log_scales;
  const float* __restrict__ quats;
  const float* __restrict__ logits;
  const float* __restrict__ sh;
  int32_t per;  // 3K floats per Gaussian
  __device__ float4 a(int64_t g) const {
    return make_float4(means[3 * g], means[3 * g + 1], means[3 * g + 2], logits[g]);
  }
  __device__ float4 b(int64_t g) const {
    return make_float4(log_scales[3 * g], log_scales[3 * g + 1], log_scales[3 * g + 2], 0.f);
  }
  __device__ float4 q(int64_t g) const { return *reinterpret_cast<const float4*>(quats + 4 * g); }
  __device__ float coef(int i, int64_t g) const { return sh[g * per + i]; }
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
};

// One device allocation carved into a workspace's arrays.
struct Arena {
  uint8_t* base = nullptr;
  size_t bytes = 0;
};

// How a workspace gets memory when a frame needs more than it holds.
enum class Growth {
  kAllocator,  // the caller's adr_allocator: alloc the new arena, stream-ordered free of the old
  kDefault,    // hipMalloc; the old arena is kept until reserve/destroy (no hipFree in a render)
  kNone,       // fixed memory (the no-allocation entry point): too small is an error
};

}  // namespace adr

struct adr_scene {
  adr::DeviceScene d;
  uint64_t uid = 0;  // unique per created scene in this process (a freed scene's address may be reused)
  adr_allocator alloc{};  // provider of the owned copy (alloc == NULL: hipMalloc)
};

#ifndef ADR_FRAME_SLOTS
#define ADR_FRAME_SLOTS 3
#endif
static_assert(ADR_FRAME_SLOTS >= 2, "a pipelined workspace needs at least two frame slots");

struct adr_workspace {
  adr::Growth growth = adr::Growth::kDefault;
  bool headroom = true;  // grow arenas 25% past the frame's need
  adr_allocator alloc{};
  adr::Arena gauss_arena, pair_arena, tile_arena, fixed_arena, grad_arena;
  std::vector<adr::Arena> retired;  // kDefault: arenas replaced during renders, freed at reserve/destroy
  // capacities the arenas are carved for
  int64_t gauss_capacity = 0, pair_capacity = 0, tile_capacity = 0, grad_capacity = 0;
  // per Gaussian (gauss arena)
  adr::RenderRecord* rec = nullptr;
  adr::ExactRecord* exact = nullptr;
  uint2* tile_rect = nullptr;      // (tx_lo | tx_hi << 16, ty_lo | ty_hi << 16)
  uint32_t* touched = nullptr;
  uint32_t* offsets = nullptr;     // inclusive sum of touched in depth order
  uint32_t* touched_sorted = nullptr;  // tiles_touched in depth order
  adr::SortBuffers depth;          // (depth key, id) of every Gaussian, sorted by depth
  uint32_t* scan_partials = nullptr;
  ulonglong4* block_parts = nullptr;  // per Preprocess workgroup: pairs, visible, depth-key min, max
  uint32_t* depth_scratch = nullptr;  // radix digit counts of the depth sort
  // per pair (pair arena)
  adr::SortBuffers pairs;          // (tile id, Gaussian id), sorted by tile
  // per DuplicateWithKeys workgroup (kDupPairs pairs): the depth-order index
  // of the Gaussian that holds its first pair, written by the InclusiveSum
  uint32_t* dup_first = nullptr;
  uint32_t* pair_scratch = nullptr;   // radix digit counts of the tile sort
  // per tile (tile arena)
  uint32_t* ranges = nullptr;      // 2 * tiles
  uint32_t* tile_order = nullptr;  // render order of the tiles, longest lists first
  uint32_t* order_counts = nullptr;  // per-block bucket counts of the tile order
  unsigned long long* wave_sums = nullptr;     // 4 x u64 per render wave (load-sum partials)
  // fixed arena: counters and the two sort digit totals, and the frame's load
  // accumulators; cleared at the start of every frame
  unsigned long long* dev_counters = nullptr;  // kCounterSlots u64, see below
  uint32_t* hists = nullptr;                   // 2 x kHistWords: depth sort, tile sort
  unsigned long long* load_acc = nullptr;      // kLoadAccWords: four sums, a block ticket
  unsigned long long* notify_slot = nullptr;   // kNotifySlots device words (when notify_host is NULL)
  // gradients (grad arena)
  float* grad2d = nullptr;              // kGrad2d floats per Gaussian
  unsigned long long* host_counters = nullptr; // pinned copy for adr_workspace_counters
  // mapped pinned memory the kernel after Preprocess writes the pair count
  // into; NULL: it writes notify_slot, which the host copies back
  unsigned long long* notify_host = nullptr;
  unsigned long long* notify_dev = nullptr;
  unsigned long long frame_seq = 0;
  // ev[0..10]: the stage boundaries of a timed frame; ev[11]: the blend's start
  // on the caller's stream (after any wait for the previous frame)
  static constexpr int kEvents = 12;
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
  // A pipelined workspace (adr_workspace_create) has kFrameSlots frame slots
  // that consecutive frames take in turn: this handle (slot 0), which owns
  // the others, and slots 1.. . A frame of an owned scene runs its stages up
  // to the tile order on its slot's side stream, which waits only for the
  // previous frame of the same slot, so they overlap the early stages and
  // the blend of the frames before it. Every slot has its own arenas, side
  // stream, events and pinned words.
  static constexpr int kFrameSlots = ADR_FRAME_SLOTS;
  adr_workspace* slots[kFrameSlots] = {};  // (slot 0) every slot, slots[0] == this; null when not pipelined
  hipStream_t side = nullptr;
  hipEvent_t prep_done = nullptr;     // the slot's stages up to the tile order (side stream)
  hipEvent_t slot_free = nullptr;     // the slot's last frame or backward (caller's stream)
  int next_slot = 0;                  // (slot 0) the slot of the next frame
  adr_workspace* last_slot = nullptr;  // (slot 0) the slot of the last frame
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
constexpr int kLoadAccWords = 8;     // sum l_blend, sum l_blend^2, sum l_iter, sum l_iter^2, ticket, unused

// Arena layouts. Each carves an arena at base for the given capacity and,
// when ws is given, points the workspace's arrays into it; base == nullptr
// only sizes it. Returns the arena's bytes (every array 256-byte aligned).
size_t carve_gauss_arena(uint8_t* base, int64_t n, adr_workspace* ws);
size_t carve_pair_arena(uint8_t* base, int64_t n_pairs, adr_workspace* ws);
size_t carve_tile_arena(uint8_t* base, int64_t n_tiles, adr_workspace* ws);
size_t carve_fixed_arena(uint8_t* base, adr_workspace* ws);

// The stages of one frame, split where the serving path batches the blend
// of several frames: prepare runs Preprocess through the tile order (one
// host wait for the pair count), finish runs the blend, the load sums and
// the optional copies. adr_render is prepare + finish.
struct FramePlan {
  CamArgs cam;
  CullArgs cull;
  BlendArgs blend;
  int64_t n_tiles = 0;
  int64_t n_pairs = 0;
  const uint32_t* tiles = nullptr;  // sorted tile ids of the pairs
  const uint32_t* vals = nullptr;   // sorted Gaussian ids of the pairs
  bool want_load = false;           // load sums or statistics requested
};
adr_status render_prepare(const adr_scene* scene, const adr_camera* cam, const adr_render_params* p,
                          adr_frame* out, adr_workspace* ws, hipStream_t stream, FramePlan& plan);
adr_status render_finish(const adr_scene* scene, const adr_camera* cam, const adr_render_params* p,
                         adr_frame* out, adr_workspace* ws, hipStream_t stream, const FramePlan& plan,
                         bool blend_launched);
// Returns the per-Gaussian, per-pair and per-tile arenas to the allocator
// (nothing may use them any more); the next frame acquires them again.
void workspace_release_frame_arenas(adr_workspace* ws);
// Grows ws's arenas for a frame (nothing is enqueued); ADR_E_WORKSPACE for
// a fixed-memory workspace that is too small.
adr_status ensure_capacity(adr_workspace* ws, int64_t n_gauss, int64_t n_pairs, int64_t n_tiles, hipStream_t stream);

// Creates a workspace; pipelined: with the frame slots and side streams of
// adr_workspace_create (the server's slots are not pipelined).
adr_status workspace_create(const adr_allocator* allocator, bool pipelined, adr_workspace** out);

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
hipError_t launch_frame_init(adr_workspace* ws, int64_t n_tiles, hipStream_t stream);
int64_t preprocess_blocks(int64_t n);
// Frames whose tile ranges have at most this many words have them cleared
// (with the counters and the load sums) by the kernel that follows
// Preprocess instead of a launch of their own.
constexpr int64_t kNotifyClearMax = (int64_t)1 << 17;
// n_ranges: what the frame-init launch clears (the tile ranges, with the
// counters and load accumulators) is cleared here when
// 0 < n_ranges <= kNotifyClearMax (n_ranges = 0: nothing is cleared)
hipError_t launch_preprocess(const DeviceScene& s, const CamArgs& cam, const CullArgs& cull, adr_workspace* ws,
                             int64_t n_ranges, hipStream_t stream);
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
hipError_t launch_tile_order(const uint32_t* ranges, int64_t n_pairs, int tiles_x, int tiles_y, uint32_t* order,
                             uint32_t* counts, hipStream_t stream);
hipError_t launch_render(const RenderRecord* rec, const ExactRecord* exact, const uint32_t* vals,
                         const uint32_t* ranges, const uint32_t* order, int64_t n_pairs, int64_t n_gauss,
                         const CamArgs& cam, const BlendArgs& blend, const adr_frame* out, bool want_load,
                         adr_workspace* ws, hipStream_t stream);
// One frame's blend in a batched launch (the serving path): its buffers,
// camera and blend arguments, and its workgroups [block_base,
// block_base + n_tiles) of the launch.
struct BlendJob {
  const RenderRecord* rec;
  const ExactRecord* exact;
  const uint32_t* vals;
  const uint32_t* ranges;
  const uint32_t* order;
  float* image;
  float* final_t;
  uint32_t* l_iter;
  uint32_t* l_blend;
  ulonglong4* wave_sums;
  unsigned long long* counters;
  uint32_t n_pairs, n_gauss;
  int32_t n_tiles, block_base;
  CamArgs cam;
  BlendArgs blend;
};
BlendJob make_blend_job(const adr_workspace* ws, const RenderRecord* rec, const ExactRecord* exact,
                        const uint32_t* vals, const CamArgs& cam, const BlendArgs& blend, int64_t n_pairs,
                        int64_t n_gauss, const adr_frame* out, bool want_load);
// jobs_dev: n_jobs jobs in device memory, ascending block_base, covering
// [0, total_blocks); any_cap: some job has a load-balancing cap
hipError_t launch_render_batch(const BlendJob* jobs_dev, int n_jobs, int64_t total_blocks, bool any_cap,
                               hipStream_t stream);
// Reduces the render waves' load partials into ws->load_acc; the last
// workgroup writes the caller's load_sums and load_stats (either may be NULL).
hipError_t launch_load_sums(adr_workspace* ws, int n_tiles, int64_t n_pixels, uint64_t* load_sums,
                            double* load_stats, hipStream_t stream);
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
