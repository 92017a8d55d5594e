/*
 * adr.h - C ABI of the MI355X (gfx950) AdR-Gaussian tile rasterizer.
 *
 * Forward path of "AdR-Gaussian: Accelerating Gaussian Splatting with
 * Adaptive Radius" (arXiv 2409.08669): the six-stage tile rasterizer of
 * Sec. 3.2 with the early culling of Gaussian-tile pairs by adaptive radius
 * (Sec. 4.2, Eqs. 5-8) or by the axis-aligned bounding box (Sec. 4.3,
 * Eqs. 9-11), the per-pixel load counters of Eq. 12, the load statistic of
 * Eq. 13, and a load-balancing render mode that caps the number of Gaussians
 * a pixel blends.
 *
 * Conventions shared by every entry point:
 *  - All device pointers refer to memory of the current HIP device.
 *  - Work is enqueued on the caller's stream (a hipStream_t passed as void*;
 *    NULL = the null stream). adr_render waits once per frame, after
 *    Preprocess, for the pair count (the GPU writes it to mapped pinned host
 *    memory); everything else is asynchronous.
 *  - Device memory for scenes and workspaces comes from an adr_allocator the
 *    caller may supply (NULL: hipMalloc). Nothing in adr_render or
 *    adr_render_backward frees device memory with hipFree (which would
 *    synchronise the whole device).
 *  - Functions return ADR_OK or a negative adr_status; adr_last_error()
 *    returns a thread-local message for the last failure. No C++ exception
 *    crosses this boundary.
 *  - Argument errors (NULL pointers, bad sizes, unsupported modes) are
 *    detected on the host before anything is enqueued.
 */
#ifndef ADR_H
#define ADR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ADR_OK = 0,
  ADR_E_INVALID = -1,     /* bad argument; nothing was enqueued */
  ADR_E_OOM = -2,         /* a device or pinned allocation failed */
  ADR_E_HIP = -3,         /* a HIP runtime call or kernel launch failed */
  ADR_E_UNSUPPORTED = -4, /* valid request this library does not implement */
  ADR_E_WORKSPACE = -5    /* caller's pair buffers too small; see adr_frame.n_pairs */
} adr_status;

/* Pair culling of the Preprocess stage. */
/* The adaptive and AABB modes also reuse their (uncapped) extent inside the
 * Render stage: a wave skips a Gaussian for an 8 x 8 pixel quadrant that the
 * extent misses. The 3-sigma baseline evaluates every entry of a tile's list
 * for every pixel of the tile. All three give the same image. */
typedef enum {
  ADR_CULL_3SIGMA = 0,   /* baseline: square of radius r_o = 3 sqrt(lambda'_max) (Sec. 4.2) */
  ADR_CULL_ADAPTIVE = 1, /* r = min(sqrt(2 lambda'_max ln(sigma/alpha_low)), r_o) (Eqs. 7-8) */
  ADR_CULL_AABB = 2      /* r_x, r_y = min(sqrt(2 Sigma'_X|Y ln(sigma/alpha_low)), r_o) (Eqs. 10-11) */
} adr_cull;

/* Opaque scene: the Gaussians of Sec. 3.1 (Eq. 1) in library-owned device
 * memory, immutable after creation; may be shared by concurrent renders. */
typedef struct adr_scene adr_scene;

/* Opaque scratch (per-Gaussian records, pair and sort buffers, tile
 * ranges): four device arenas (per Gaussian, per pair, per tile, and a few
 * fixed counters), each one allocation, per frame slot (see
 * adr_workspace_create). Grows on demand. Calls on one workspace must come
 * from one host thread at a time; consecutive renders may be enqueued
 * without waiting for the earlier ones. */
typedef struct adr_workspace adr_workspace;

/* Caller-supplied device memory (for example a caching allocator).
 *   alloc(bytes, stream, ctx) returns device memory of the current device,
 *     at least `bytes` long and 256-byte aligned, usable by work enqueued on
 *     `stream` (a hipStream_t as void*); NULL on failure (the library then
 *     returns ADR_E_OOM).
 *   free(ptr, bytes, stream, ctx) releases a block from alloc. The block may
 *     still be read or written by work already enqueued on `stream`: the
 *     allocator must reuse it only for work ordered after that (a
 *     stream-ordered release, as a caching allocator does).
 * Both are called on the thread that called into the library. */
typedef struct {
  void* (*alloc)(size_t bytes, void* stream, void* ctx);
  void (*free)(void* ptr, size_t bytes, void* stream, void* ctx);
  void* ctx;
} adr_allocator;

/* Scene description (Sec. 3.1): centre, covariance as scale and rotation,
 * opacity and SH colour. Arrays are row-major float32, one row per Gaussian:
 *   means          N x 3           world-space centres
 *   log_scales     N x 3           per-axis log standard deviation
 *   quats          N x 4           rotation quaternion (w, x, y, z), any norm > 0
 *   opacity_logits N               opacity = 1 / (1 + exp(-logit))
 *   sh             N x K x 3       real SH coefficients, K = (sh_degree+1)^2,
 *                                  index l*l + l + m (Condon-Shortley phase)
 * pointers_on_device = 1: device pointers; 0: host.
 * borrow = 0: the arrays are copied (and transposed to planes) during
 *   adr_create_scene; the caller keeps ownership of its arrays.
 * borrow = 1 (device pointers only): no copy. The scene reads the caller's
 *   arrays in place, in the row-major layout above, for every render; the
 *   caller keeps them allocated and unchanged until adr_destroy_scene. */
typedef struct {
  int64_t n;
  int32_t sh_degree; /* 0..3 */
  int32_t pointers_on_device;
  int32_t borrow;
  int32_t reserved;  /* 0 */
  const float* means;
  const float* log_scales;
  const float* quats;
  const float* opacity_logits;
  const float* sh;
} adr_scene_desc;

/* Pinhole camera, OpenCV axes (x right, y down, z forward).
 * p_cam = R p_world + t with world_to_cam = [R | t] row-major 3 x 4.
 * Pixel (i, j) covers [i, i+1) x [j, j+1) in image coordinates u = fx x/z + cx.
 * Gaussians with camera-space z <= near_z are not drawn. */
typedef struct {
  double world_to_cam[12];
  double fx, fy, cx, cy;
  int32_t width, height; /* 1 .. 65535 each */
  double near_z;
} adr_camera;

/* Flags of adr_render_params.flags */
#define ADR_FLAG_TIMING 1u      /* record per-stage HIP events; see adr_workspace_stage_times */
#define ADR_FLAG_NO_EXACT_BAND 2u /* skip the FP64 re-decision of near-threshold alphas and
                                     transmittances (faster, no longer bit-matched to FP64) */
#define ADR_FLAG_NO_QUAD_CULL 4u  /* adaptive/AABB modes: cull Gaussian-tile pairs only, and evaluate
                                     every list entry for every pixel of the tile (ablation; same output) */

typedef struct {
  int32_t cull;      /* adr_cull */
  int32_t lb_cap;    /* load-balancing mode: a pixel stops after blending this many Gaussians; 0 = off */
  double alpha_low;  /* minimum splatting opacity, 1/255 (Sec. 5.1.2); cull and skip threshold */
  double alpha_max;  /* upper clamp of alpha, 0.99 */
  double t_min;      /* a pixel stops once its transmittance falls below this, 1e-4 */
  double lowpass;    /* added to the diagonal of Sigma', 0.3 */
  double ewa_clamp;  /* EWA Jacobian evaluated at x/z clamped to +- ewa_clamp * (W/2)/fx, 1.3 */
  float background[3];
  uint32_t flags;    /* ADR_FLAG_* */
} adr_render_params;

/* Outputs of one frame. Every pointer is caller-owned device memory; all but
 * image may be NULL to skip that output.
 *   image         3 x H x W float32, C + T * background (Eq. 3)
 *   final_t       H x W     float32, transmittance when the pixel stopped
 *   l_iter        H x W     uint32, entries of the tile list examined (the thread's work)
 *   l_blend       H x W     uint32, Gaussians blended (Eq. 12)
 *   load_sums     4         uint64: sum l_blend, sum l_blend^2, sum l_iter, sum l_iter^2
 *                           over H x W
 *   load_stats    4         double: mean and population standard deviation of l_blend over
 *                           the H x W pixels (the load statistic of Eq. 13, zero-load pixels
 *                           included), then the same of l_iter; from the exact integer sums
 *   tiles_touched N         uint32 per Gaussian (Preprocess)
 *   keys, values  pair_capacity   sorted (tile << 32 | depth bits) keys and Gaussian ids
 *   ranges        2 x T     uint32 [first, last+1) per tile, (0, 0) when empty,
 *                           T = ceil(W/16) * ceil(H/16), tile id = ty * ceil(W/16) + tx
 * n_pairs is written on return (host) with the frame's Gaussian-tile pair count.
 * If keys/values are given and n_pairs > pair_capacity, adr_render returns
 * ADR_E_WORKSPACE after writing the image (the pair lists are not copied). */
typedef struct {
  float* image;
  float* final_t;
  uint32_t* l_iter;
  uint32_t* l_blend;
  uint64_t* load_sums;
  double* load_stats;
  uint32_t* tiles_touched;
  uint64_t* keys;
  uint32_t* values;
  uint32_t* ranges;
  int64_t pair_capacity;
  int64_t n_pairs;
} adr_frame;

/* Per-Gaussian gradients, same shapes as adr_scene_desc arrays (device). */
typedef struct {
  float* d_means;
  float* d_log_scales;
  float* d_quats;
  float* d_opacity_logits;
  float* d_sh;
} adr_scene_grads;

/* Creates a scene from desc (see adr_scene_desc), the Gaussians of Sec. 3.1.
 * allocator (may be NULL: hipMalloc/hipFree) provides the device copy and
 * the staging of host arrays; it must stay valid until adr_destroy_scene.
 * Returns ADR_E_INVALID for n < 0, sh_degree outside 0..3, NULL arrays with
 * n > 0, or borrow = 1 with host pointers; ADR_E_OOM when the device copy
 * cannot be allocated. Synchronous (a borrowed scene enqueues nothing). */
adr_status adr_create_scene(const adr_scene_desc* desc, const adr_allocator* allocator, adr_scene** out);
void adr_destroy_scene(adr_scene* scene);
int64_t adr_scene_size(const adr_scene* scene);
/* Device bytes the scene holds (0 for a borrowed scene). */
int64_t adr_scene_bytes(const adr_scene* scene);

/* Creates an empty workspace on the current device. It holds three frame
 * slots that consecutive adr_render calls take in turn, each with a side
 * stream (default priority): for a scene that is not borrowed, a frame's
 * stages up to the tile order run on its slot's side stream, which waits
 * only for the previous frame of the same slot (three frames earlier: its
 * blend, copies and any backward), not for the caller's stream, so they
 * overlap the early stages and the blend of the frames before it; the blend
 * and everything after it run on the caller's stream after the side
 * stream's part. Outputs are only written on the caller's stream, and an
 * owned scene is immutable, so every frame's results are as if all of it
 * ran on the caller's stream. A borrowed scene runs every stage on the
 * caller's stream (the caller may change its arrays between frames).
 * allocator (may be NULL)
 * provides its arenas and must stay valid until adr_workspace_destroy. With
 * a caller allocator an arena that is too small for a frame is replaced
 * inside adr_render (alloc the new one, stream-ordered free of the old one).
 * With NULL the library allocates with hipMalloc and never calls hipFree
 * inside a render: a replaced arena is kept until the next
 * adr_workspace_reserve or adr_workspace_destroy, which free it (and
 * synchronise the device). ADR_E_OOM if the pinned counters cannot be
 * allocated. */
adr_status adr_workspace_create(const adr_allocator* allocator, adr_workspace** out);
/* Waits for the device, then releases every arena. */
void adr_workspace_destroy(adr_workspace* ws);
/* Grows the arenas of every frame slot (never shrinks them) to hold a
 * frame of n_gauss Gaussians, n_pairs Gaussian-tile pairs and n_tiles tiles,
 * and frees the arenas kept from earlier growth. Synchronises the device. A
 * render that stays within the reserved sizes allocates nothing. */
adr_status adr_workspace_reserve(adr_workspace* ws, int64_t n_gauss, int64_t n_pairs, int64_t n_tiles);
/* Device bytes one frame slot needs for such a frame (arena sizes, without
 * growth headroom); -1 for negative arguments. Host arithmetic only. A
 * workspace reserved for the frame holds three times this (three slots). */
int64_t adr_workspace_bytes(int64_t n_gauss, int64_t n_pairs, int64_t n_tiles);
/* Device bytes the arenas of all slots hold now, kept arenas included. */
int64_t adr_workspace_capacity_bytes(const adr_workspace* ws);

/* Renders one frame: Preprocess (projection, SH colour, cull per params.cull),
 * InclusiveSum, DuplicateWithKeys, SortPairs, IdentifyTileRanges and Render
 * (Sec. 3.2), ordered on the given stream: for a scene that is not borrowed
 * the stages before Render run on the frame slot's side stream, which the
 * given stream then waits for (see adr_workspace_create). Outputs are
 * written into out, on the given stream only. */
adr_status adr_render(const adr_scene* scene, const adr_camera* cam, const adr_render_params* params,
                      adr_frame* out, adr_workspace* ws, void* stream);

/* Gradient of a scalar loss L with respect to the scene inputs, given
 * dl_dimage = dL/dimage (3 x H x W float32, device): the derivative of the
 * forward definition (Eqs. 2-3 over the blended list entries, Preprocess of
 * Sec. 3.1) on the piece fixed by the forward's decisions; clamped alpha,
 * colour channels and EWA slopes pass no derivative.
 * Differentiates the frame of the last adr_render on ws, which must have had
 * the same scene (the same scene object: one destroyed and re-created does
 * not match, even at the same address), camera and params, and must have
 * enqueued its Render stage: a call that failed before it leaves nothing to
 * differentiate (ADR_E_INVALID otherwise); fwd is that
 * call's frame, whose final_t and l_iter are required (each pixel walks its
 * list back to front from them: nothing else is stored per entry).
 * grads: caller-owned device arrays in the layout of adr_scene_desc (any may be
 * NULL to skip it); every element is written (zero for Gaussians behind the
 * near plane). float32 atomics add the per-pixel contributions, so results
 * vary in the last bits from call to call. Asynchronous on stream; ws is
 * used as scratch (40 bytes per Gaussian). */
adr_status adr_render_backward(const adr_scene* scene, const adr_camera* cam, const adr_render_params* params,
                               const adr_frame* fwd, const float* dl_dimage, adr_scene_grads* grads,
                               adr_workspace* ws, void* stream);

/* adr_render_backward with a second term: dl_dload (H x W float32, device, may
 * be NULL) is dL/dl_blend per pixel for a loss on the per-pixel load (Eq. 12;
 * e.g. its standard deviation, Eq. 13, in the load-balancing loss, Eq. 14).
 * The load is an integer count; its derivative is read as 1 with respect to
 * the alpha of every entry the pixel blended (a straight-through reading; the
 * paper does not say how the load's gradient is formed). Same requirements,
 * errors and outputs as adr_render_backward. */
adr_status adr_render_backward_load(const adr_scene* scene, const adr_camera* cam, const adr_render_params* params,
                                    const adr_frame* fwd, const float* dl_dimage, const float* dl_dload,
                                    adr_scene_grads* grads, adr_workspace* ws, void* stream);

/* adr_render for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, hosts that forbid allocation). Same
 * arguments, outputs and errors as adr_render, without a workspace: the
 * frame's workspace is carved from one static device array of
 * adr_noalloc_scratch_bytes() bytes (256 MiB) that each GPU holds from the
 * first call on it until the process ends. The call allocates nothing: no
 * hipMalloc or hipFree, no pinned host memory, no events (so no stage
 * timing); the pair count comes back by a device-to-host copy and a wait on
 * the stream. The kernels and their launch configuration are adr_render's,
 * so the outputs are bitwise the same.
 * Limits: the per-Gaussian (about 133 bytes each) and per-tile (about 149
 * bytes each) arrays must fit in the array with room for pairs, else
 * ADR_E_WORKSPACE before anything is enqueued; the pairs (about 16.1 bytes
 * each with the sort scratch) take what is left, and a frame with more returns ADR_E_WORKSPACE after
 * Preprocess with out->n_pairs set (1M Gaussians at 1920 x 1080, ~2.2M
 * pairs, fit). Every call on a GPU shares that GPU's array: calls are
 * serialised on the host, but the kernels of a call still running on one
 * stream race with a later call's on another stream of the same GPU;
 * synchronise between such calls. Not differentiable (adr_render_backward
 * needs a workspace). */
adr_status adr_render_noalloc(const adr_scene* scene, const adr_camera* cam, const adr_render_params* params,
                              adr_frame* out, void* stream);
/* Size in bytes of the static device array adr_render_noalloc carves. */
int64_t adr_noalloc_scratch_bytes(void);

/* Stage durations (ms) of the last adr_render on ws that had ADR_FLAG_TIMING:
 * [0] preprocess, [1] host wait for the pair count, [2] depth sort of the
 * Gaussians, [3] inclusive sum, [4] duplicate with keys, [5] tile sort of the
 * pairs, [6] tile ranges, [7] tile render order, [8] render (the blend kernel
 * alone, from its own start: on a pipelined workspace the stages before it
 * run on the frame slot's side stream and may end before the previous frame's
 * blend does), [9] load-sum reduction.
 * Waits for the frame to finish. Returns the number of stages written. */
int32_t adr_workspace_stage_times(adr_workspace* ws, float* ms, int32_t n);

/* Per-frame counters of the last adr_render on ws (host values; the frame
 * must have finished): [0] pairs, [1] visible Gaussians (tiles_touched > 0),
 * [2] exact-band alpha re-decisions, [3] exact-band transmittance replays,
 * [4] key bits the depth sort of the Gaussians covered (the visible depth
 * keys' range; 8 per radix pass), [5] sort values or output positions found
 * out of range and dropped (always 0 unless a kernel is wrong; a dropped value
 * is never used as an index). Returns the number of entries written. */
int32_t adr_workspace_counters(adr_workspace* ws, int64_t* out, int32_t n);

/* Serving: resident scenes, continuous batching of render requests.
 *
 * A server keeps no scenes of its own: requests name scenes the caller
 * created (resident in device memory) and caller-owned output buffers.
 * Requests are admitted in arrival order as render slots and device memory
 * free up. Admission reserves the request's workspace footprint,
 * adr_workspace_bytes(N, pairs, tiles), against memory_budget, with pairs
 * estimated from the last frame of the same scene, resolution and cull mode
 * (4 N before the first); at least one request is always admitted. An
 * admitted request runs Preprocess through the tile order (Sec. 3.2, stages
 * 1-5) on its slot's stream, so the stages of several requests overlap on the
 * device. Whenever frames are ready, one launch blends all of them: every
 * (request, tile) item of the batch is a workgroup of that launch, while the
 * next requests' earlier stages keep running. Each frame's outputs are
 * bitwise those adr_render gives for the same request alone. Workspace
 * arenas come from a device pool the server owns (sized blocks kept for
 * reuse, released at adr_server_destroy); a request returns its arenas to
 * the pool when its frame is done. */
typedef struct adr_server adr_server;

typedef struct {
  int32_t n_slots;       /* requests in flight at once, 1..64 */
  int32_t max_batch;     /* frames per blend launch, 1..64 */
  int64_t memory_budget; /* device bytes admitted requests may reserve, > 0 */
} adr_server_config;

typedef struct {
  int32_t status;    /* adr_status of the frame (ADR_OK, or its error; see adr_last_error after the wait) */
  int32_t batch_size; /* frames blended in the same launch as this one */
  int64_t n_pairs;   /* the frame's Gaussian-tile pair count */
  int64_t batch_id;  /* index of that launch (0, 1, ...) */
  int64_t footprint; /* bytes reserved at admission */
  double arrival_s;  /* adr_clock_s(): as given at submission */
  double submit_s;   /* when submitted */
  double start_s;    /* when admitted to a slot */
  double done_s;     /* when its blend launch was seen finished */
} adr_request_info;

typedef struct {
  int64_t requests_done;
  int64_t batches;
  int32_t max_batch_seen;
  int32_t reserved1;
  int64_t reserved_bytes_peak; /* largest sum of admitted footprints */
  int64_t pool_bytes;          /* device bytes the pool holds */
} adr_server_stats;

/* Creates a server on the current device: config->n_slots slot threads, each
 * with a HIP stream (default priority) and a workspace, and one thread that
 * forms and launches the batched blends on a stream of its own. ADR_E_INVALID
 * for a NULL or out-of-range config; ADR_E_HIP or ADR_E_OOM if a stream,
 * event, workspace or staging buffer cannot be created. */
adr_status adr_server_create(const adr_server_config* config, adr_server** out);
/* Finishes every queued and running request, then releases the slots and
 * the pool. */
void adr_server_destroy(adr_server* server);
/* Queues one frame; writes its ticket. arrival_s (adr_clock_s() seconds, or
 * 0 for the time of the call) is when the request is taken to have arrived,
 * the origin of its latency. Argument errors are reported here, before
 * anything is queued. The scene, the frame's output buffers and the params'
 * and camera's values are read when the request runs: the scene and buffers
 * must stay valid until adr_server_wait returns for the ticket. */
adr_status adr_server_submit(adr_server* server, const adr_scene* scene, const adr_camera* cam,
                             const adr_render_params* params, const adr_frame* frame, double arrival_s,
                             uint64_t* ticket);
/* Blocks until the ticket's frame has finished on the device, fills info and
 * retires the ticket. ADR_E_INVALID for an unknown ticket. */
adr_status adr_server_wait(adr_server* server, uint64_t ticket, adr_request_info* info);
/* Counters since creation. */
adr_status adr_server_stats_get(adr_server* server, adr_server_stats* out);
/* Seconds of the steady clock the server time-stamps requests with. */
double adr_clock_s(void);

const char* adr_last_error(void);
const char* adr_version(void);

#ifdef __cplusplus
}
#endif
#endif /* ADR_H */
