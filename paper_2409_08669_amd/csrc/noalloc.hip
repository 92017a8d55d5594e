// adr_render_noalloc: adr_render for callers that cannot allocate device
// memory (code under stream capture, tight serving loops, hosts that forbid
// allocation). Its workspace is carved from one static device array of fixed
// size that each GPU holds from the first call on it until the process ends;
// the call allocates nothing (no hipMalloc, hipFree, pinned host memory or
// events). The kernels are the ones adr_render runs, in the same launch
// configuration, so a frame is bitwise what adr_render gives.
//
// The array's name is a host-side stand-in in host code: its device address
// is looked up once per device with hipGetSymbolAddress (with that device
// current) and only that address is handed to kernels.
#include <mutex>
#include <string>

#include "adr_internal.h"

namespace adr {
namespace {

constexpr size_t kNoAllocScratchBytes = (size_t)256 << 20;  // 256 MiB per device
constexpr int kNoAllocMaxDevices = 64;

}  // namespace
}  // namespace adr

// Every call on a device shares that device's copy; contents persist from
// call to call (what a frame needs zeroed, the kernels clear at its start).
static __device__ __align__(256) uint8_t scratch[adr::kNoAllocScratchBytes];

namespace adr {
namespace {

struct NoAllocDevice {
  std::once_flag once;
  hipError_t lookup = hipSuccess;
  uint8_t* ptr = nullptr;  // this device's address of `scratch`
  std::mutex mu;           // host-side state of the calls on this device
  adr_workspace ws;        // arenas carved from ptr; no pinned memory, no events
};

NoAllocDevice g_noalloc[kNoAllocMaxDevices];

// Largest pair capacity whose arena fits in `bytes`.
int64_t pairs_that_fit(size_t bytes) {
  if (carve_pair_arena(nullptr, 0, nullptr) > bytes) return -1;
  int64_t lo = 0, hi = (int64_t)1 << 32;  // carve_pair_arena(lo) fits
  while (hi - lo > 1) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (carve_pair_arena(nullptr, mid, nullptr) <= bytes)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

}  // namespace
}  // namespace adr

using namespace adr;

extern "C" int64_t adr_noalloc_scratch_bytes(void) { return (int64_t)kNoAllocScratchBytes; }

extern "C" adr_status adr_render_noalloc(const adr_scene* scene, const adr_camera* cam,
                                         const adr_render_params* params, adr_frame* out, void* stream_ptr) {
  adr_status st = validate_render_args(scene, cam, params, out);
  if (st != ADR_OK) return st;
  int dev = -1;
  ADR_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoAllocMaxDevices) {
    set_error("adr_render_noalloc: device index beyond the supported " + std::to_string(kNoAllocMaxDevices));
    return ADR_E_UNSUPPORTED;
  }
  NoAllocDevice& d = g_noalloc[dev];
  std::call_once(d.once, [&d] {
    void* p = nullptr;
    d.lookup = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (d.lookup == hipSuccess && p == nullptr) d.lookup = hipErrorInvalidSymbol;
    if (d.lookup != hipSuccess) (void)hipGetLastError();
    d.ptr = static_cast<uint8_t*>(p);
  });
  if (d.lookup != hipSuccess) return hip_fail(d.lookup, "adr_render_noalloc: hipGetSymbolAddress(scratch)");

  std::lock_guard<std::mutex> lock(d.mu);
  adr_workspace& ws = d.ws;
  const int64_t n = scene->d.n;
  const int64_t n_tiles = (int64_t)((cam->width + kTile - 1) / kTile) * ((cam->height + kTile - 1) / kTile);
  // Layout: fixed words, then the per-tile and per-Gaussian arenas at this
  // frame's sizes; the pair arena takes all that is left.
  const size_t fixed_b = carve_fixed_arena(nullptr, nullptr);
  const size_t tile_b = carve_tile_arena(nullptr, n_tiles, nullptr);
  const size_t gauss_b = carve_gauss_arena(nullptr, n, nullptr);
  const size_t used = fixed_b + tile_b + gauss_b;
  const int64_t pair_cap = used <= kNoAllocScratchBytes ? pairs_that_fit(kNoAllocScratchBytes - used) : -1;
  if (pair_cap < 0) {
    set_error("adr_render_noalloc: " + std::to_string(n) + " Gaussians and " + std::to_string(n_tiles) +
              " tiles need " + std::to_string(used) + " bytes before any pair; the fixed scratch holds " +
              std::to_string(kNoAllocScratchBytes));
    return ADR_E_WORKSPACE;
  }
  uint8_t* base = d.ptr;
  ws.growth = Growth::kNone;
  ws.headroom = false;
  ws.fixed_arena = Arena{base, fixed_b};
  carve_fixed_arena(base, &ws);
  ws.tile_arena = Arena{base + fixed_b, tile_b};
  ws.tile_capacity = n_tiles;
  carve_tile_arena(base + fixed_b, n_tiles, &ws);
  ws.gauss_arena = Arena{base + fixed_b + tile_b, gauss_b};
  ws.gauss_capacity = n;
  carve_gauss_arena(base + fixed_b + tile_b, n, &ws);
  ws.pair_arena = Arena{base + used, kNoAllocScratchBytes - used};
  ws.pair_capacity = pair_cap;
  carve_pair_arena(base + used, pair_cap, &ws);
  // The pair count comes back by a copy of the device words and a wait on
  // the stream (no mapped host memory); no stage timing (no events).
  ws.notify_host = nullptr;
  ws.notify_dev = ws.notify_slot;

  hipStream_t stream = (hipStream_t)stream_ptr;
  FramePlan plan;
  if ((st = render_prepare(scene, cam, params, out, &ws, stream, plan)) != ADR_OK) {
    if (st == ADR_E_WORKSPACE)
      set_error("adr_render_noalloc: the frame's " + std::to_string(out->n_pairs) +
                " Gaussian-tile pairs exceed the " + std::to_string(pair_cap) +
                " that fit in the fixed scratch beside its Gaussians and tiles");
    return st;
  }
  return render_finish(scene, cam, params, out, &ws, stream, plan, false);
}
