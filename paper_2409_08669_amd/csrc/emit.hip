// DuplicateWithKeys and IdentifyTileRanges (Sec. 3.2, stages 3 and 5).
//
// Pair emission is pair-parallel and balanced: workgroup b writes pairs
// [2048 b, 2048 b + 2048). The InclusiveSum has recorded, per such chunk, the
// Gaussian (in depth order) holding its first pair; the workgroup stages the
// offsets of the Gaussians from that one to the next chunk's in LDS, and each
// pair finds its Gaussian by binary search there. One Gaussian with a huge rectangle
// therefore spreads over many workgroups, and consecutive lanes write
// consecutive pairs. Within a Gaussian the tiles are emitted row-major over
// its tile rectangle. Each pair carries the tile id as its sort key; the depth
// order is already in the emission order.
#include "adr_internal.h"

namespace adr {

namespace {

constexpr int kDupThreads = 256;

__global__ void __launch_bounds__(kDupThreads) duplicate_kernel(const uint32_t* __restrict__ offsets,
                                                                const uint32_t* __restrict__ dup_first,
                                                                const uint32_t* __restrict__ order,
                                                                const uint2* __restrict__ tile_rect, uint32_t n_vis,
                                                                uint32_t n_gauss, uint32_t n_pairs, int32_t tiles_x,
                                                                uint32_t* __restrict__ tile_keys,
                                                                uint32_t* __restrict__ vals) {
  // inclusive offsets of the workgroup's Gaussians: those holding its pairs
  // (at most kDupPairs, each holds one or more) and possibly the next one
  __shared__ uint32_t s_end[kDupPairs + 1];
  const int tid = threadIdx.x;
  const uint32_t p0 = blockIdx.x * (uint32_t)kDupPairs;
  const uint32_t p1 = min(p0 + (uint32_t)kDupPairs, n_pairs) - 1;  // last pair of the workgroup
  // the Gaussians holding pair p0 and the next workgroup's first pair (or the
  // last visible one): the one holding p1 lies between them
  const uint32_t r_lo = min(dup_first[blockIdx.x], n_vis - 1);
  const uint32_t r_hi = blockIdx.x + 1 < gridDim.x ? min(dup_first[blockIdx.x + 1], n_vis - 1) : n_vis - 1;
  const uint32_t cnt = min(r_hi >= r_lo ? r_hi - r_lo + 1 : 1u, (uint32_t)kDupPairs + 1);
  for (uint32_t i = tid; i < cnt; i += kDupThreads) s_end[i] = offsets[r_lo + i];
  const uint32_t start_lo = r_lo > 0 ? offsets[r_lo - 1] : 0u;  // first pair of Gaussian r_lo
  __syncthreads();
  for (uint32_t p = p0 + tid; p <= p1; p += kDupThreads) {
    uint32_t lo = 0, hi = cnt - 1;  // smallest i with s_end[i] > p
    while (lo < hi) {
      const uint32_t mid = (lo + hi) >> 1;
      if (s_end[mid] > p)
        hi = mid;
      else
        lo = mid + 1;
    }
    const uint32_t first = lo > 0 ? s_end[lo - 1] : start_lo;
    const uint32_t k = p - first;
    const uint32_t g = min(order[r_lo + lo], n_gauss - 1);  // (a sorted id is always below n_gauss)
    const uint2 r = tile_rect[g];
    const uint32_t tx_lo = r.x & 0xffffu, tx_hi = r.x >> 16;
    const uint32_t ty_lo = r.y & 0xffffu;
    const uint32_t w = tx_hi - tx_lo + 1;
    tile_keys[p] = (ty_lo + k / w) * (uint32_t)tiles_x + tx_lo + k % w;
    vals[p] = g;
  }
}

__global__ void __launch_bounds__(256) tile_ranges_kernel(const uint32_t* __restrict__ tiles, int64_t n_pairs,
                                                          uint32_t* __restrict__ ranges, uint32_t n_tiles) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_pairs) return;
  const uint32_t t = tiles[p];
  if (t >= n_tiles) return;  // cannot happen for keys built by duplicate_kernel
  if (p == 0 || tiles[p - 1] != t) ranges[2 * (int64_t)t] = (uint32_t)p;
  if (p == n_pairs - 1 || tiles[p + 1] != t) ranges[2 * (int64_t)t + 1] = (uint32_t)(p + 1);
}

// The 64-bit keys of the sorted pairs, (tile << 32) | depth bits.
__global__ void __launch_bounds__(256) compose_keys_kernel(const uint32_t* __restrict__ tiles,
                                                           const uint32_t* __restrict__ vals,
                                                           const RenderRecord* __restrict__ rec, int64_t n_pairs,
                                                           uint32_t n_gauss, uint64_t* __restrict__ keys) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_pairs) return;
  keys[p] = ((uint64_t)tiles[p] << 32) | rec[min(vals[p], n_gauss - 1)].depth_key;
}

// Clears everything a frame accumulates into: counters, sort histograms,
// the load accumulators and the tile ranges (empty tiles keep (0, 0)).
// Used when the kernel after Preprocess cannot do it: an empty scene (no
// Preprocess) or more tile-range words than that one workgroup clears.
__global__ void __launch_bounds__(256) frame_init_kernel(unsigned long long* __restrict__ counters,
                                                         uint32_t* __restrict__ hists,
                                                         unsigned long long* __restrict__ load_acc,
                                                         uint32_t* __restrict__ ranges, int64_t n_ranges) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kCounterSlots) counters[i] = 0ull;
  if (i < 2 * kHistWords) hists[i] = 0u;
  if (i < kLoadAccWords) load_acc[i] = 0ull;
  if (i < n_ranges) ranges[i] = 0u;
}

__global__ void fill_u32_kernel(uint32_t* __restrict__ p, uint32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void fill_u64_kernel(unsigned long long* __restrict__ p, unsigned long long v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

int64_t duplicate_blocks(int64_t n_pairs) { return (n_pairs + kDupPairs - 1) / kDupPairs; }

// dup_first: per workgroup, written by launch_inclusive_sum over the same offsets
hipError_t launch_duplicate(const uint32_t* offsets, const uint32_t* dup_first, const uint32_t* order,
                            const uint2* tile_rect, int64_t n_vis, int64_t n_gauss, int64_t n_pairs, int32_t tiles_x,
                            uint32_t* tile_keys, uint32_t* vals, hipStream_t stream) {
  if (n_pairs <= 0 || n_vis <= 0) return hipSuccess;
  if (n_pairs >= (int64_t)1 << 32 || n_vis > n_gauss || n_gauss >= (int64_t)1 << 32) return hipErrorInvalidValue;
  duplicate_kernel<<<dim3((unsigned)duplicate_blocks(n_pairs)), kDupThreads, 0, stream>>>(
      offsets, dup_first, order, tile_rect, (uint32_t)n_vis, (uint32_t)n_gauss, (uint32_t)n_pairs, tiles_x, tile_keys,
      vals);
  return hipGetLastError();
}

// ranges must be zero on entry (cleared at the start of the frame, by the
// kernel after Preprocess or by the frame-init kernel)
hipError_t launch_tile_ranges(const uint32_t* tiles, int64_t n_pairs, uint32_t* ranges, int32_t n_tiles,
                              hipStream_t stream) {
  if (n_pairs <= 0) return hipSuccess;
  tile_ranges_kernel<<<dim3((unsigned)((n_pairs + 255) / 256)), 256, 0, stream>>>(tiles, n_pairs, ranges,
                                                                                  (uint32_t)n_tiles);
  return hipGetLastError();
}

hipError_t launch_compose_keys(const uint32_t* tiles, const uint32_t* vals, const RenderRecord* rec,
                               int64_t n_pairs, int64_t n_gauss, uint64_t* keys, hipStream_t stream) {
  if (n_pairs <= 0 || n_gauss <= 0) return hipSuccess;
  compose_keys_kernel<<<dim3((unsigned)((n_pairs + 255) / 256)), 256, 0, stream>>>(tiles, vals, rec, n_pairs,
                                                                                   (uint32_t)n_gauss, keys);
  return hipGetLastError();
}

hipError_t launch_frame_init(adr_workspace* ws, int64_t n_tiles, hipStream_t stream) {
  if (n_tiles > ws->tile_capacity) return hipErrorInvalidValue;
  int64_t n = 2 * n_tiles;
  if (n < 2 * kHistWords) n = 2 * kHistWords;
  frame_init_kernel<<<dim3((unsigned)((n + 255) / 256)), 256, 0, stream>>>(ws->dev_counters, ws->hists, ws->load_acc,
                                                                           ws->ranges, 2 * n_tiles);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  fill_u32_kernel<<<dim3((unsigned)((n + 255) / 256)), 256, 0, stream>>>(p, v, n);
  return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, int64_t n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  fill_u64_kernel<<<dim3((unsigned)((n + 255) / 256)), 256, 0, stream>>>(p, v, n);
  return hipGetLastError();
}

}  // namespace adr
