// SortPairs (Sec. 3.2, stage 4) as two stable LSD radix sorts.
//
// Sorting the Gaussian-tile pairs by the 64-bit key (tile << 32 | depth bits)
// is done in two steps that give the same order: the visible Gaussians are
// sorted once by their 32-bit depth key (ties keep id order), their pairs are
// then emitted in that order, and a stable sort on the tile id alone (13 bits
// at 1080p) groups them by tile without disturbing the depth order. Each pair
// is moved in two passes instead of the five or six its 38-47 key bits need.
//
// A pass only looks at the bits that vary: keys are mapped to
// min(key - bias, lim) before the digit is taken, which keeps their order
// (every key above lim is an invisible Gaussian's all-ones key, and those
// tie). With the bias at the smallest visible depth key the 32-bit depth keys
// of a scene usually need three 8-bit passes instead of four.
//
// Each pass is reduce-then-scan: per-workgroup digit counts, one workgroup
// per digit scans them into scatter offsets, and a downsweep ranks the
// workgroup's 2048, 4096 or 8192 keys in LDS and scatters them. Ranking is stable and uses wave64
// ballots: the lanes of a row that share a digit are found with eight
// ballots, one per digit bit, and counted with popcounts, so no atomics decide
// an order. (A single-launch decoupled look-back was tried first; its chain of
// device-coherent loads across the eight XCDs cost ~0.5 ms per pass.)
#include "adr_internal.h"

namespace adr {

namespace {

// Eight waves per workgroup. Keys per lane: 4 (2048 per workgroup) up to
// 1.5M keys, so that a million depth keys still give every CU a few
// workgroups; 8 (4096) up to 3M; 16 (8192) above. Larger workgroups make
// each digit's run in the output longer, so the scattered stores fill more
// of each cache line.
constexpr int kThreads = 512;
constexpr int kWaves = kThreads / 64;
constexpr int kSmallSortItems = 4, kMidSortItems = 8, kLargeSortItems = 16;
constexpr int64_t kSmallSortMax = 1536 * 1024, kMidSortMax = 3 * 1024 * 1024;

__host__ __device__ constexpr int sort_items(int64_t n) {
  return n <= kSmallSortMax ? kSmallSortItems : n <= kMidSortMax ? kMidSortItems : kLargeSortItems;
}
constexpr int kRadix = 256;
constexpr int kMaxPasses = 4;

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, int lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t u = __shfl_up(v, off, 64);
    if (lane >= off) v += u;
  }
  return v;
}

__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* smem4) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint32_t s = wave_incl_scan(v, lane);
  if (lane == 63) smem4[wid] = s;
  __syncthreads();
  uint32_t before = 0;
  for (int w = 0; w < wid; ++w) before += smem4[w];
  __syncthreads();
  return s + before - v;
}

struct KeyMap {
  uint32_t bias;
  uint32_t lim;
};

__device__ __forceinline__ uint32_t digit_of(uint32_t k, KeyMap km, int shift) {
  const uint32_t m = min(k - km.bias, km.lim);
  return (m >> shift) & 0xffu;
}

// Per-workgroup digit counts of one pass: counts[d * nb + b].
template <int kItems>
__global__ void __launch_bounds__(kThreads) upsweep_kernel(const uint32_t* __restrict__ kin, int64_t n, int shift,
                                                           KeyMap km, uint32_t* __restrict__ counts, int64_t nb) {
  __shared__ uint32_t wh[kWaves][kRadix];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  for (int i = tid; i < kWaves * kRadix; i += kThreads) (&wh[0][0])[i] = 0u;
  __syncthreads();
  constexpr int kTileKeys = kThreads * kItems;
  const int64_t wave_base = (int64_t)blockIdx.x * kTileKeys + (int64_t)wid * (kItems * 64);
#pragma unroll 4
  for (int r = 0; r < kItems; ++r) {
    const int64_t idx = wave_base + r * 64 + lane;
    if (idx < n) atomicAdd(&wh[wid][digit_of(kin[idx], km, shift)], 1u);
  }
  __syncthreads();
  if (tid < kRadix) {
    uint32_t c = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) c += wh[w][tid];
    counts[(int64_t)tid * nb + blockIdx.x] = c;
  }
}

// One workgroup per digit d: counts[d * nb + b] becomes the number of keys
// with digit d in workgroups before b, and totals[d] the digit's total. (The
// downsweep adds the totals of the smaller digits itself, so no workgroup
// waits for another and no global atomics are needed.)
__global__ void __launch_bounds__(kThreads) digit_offsets_kernel(uint32_t* __restrict__ counts, int64_t nb,
                                                                 uint32_t* __restrict__ totals) {
  __shared__ uint32_t scan_tmp[kWaves];
  __shared__ uint32_t s_last;
  const int d = blockIdx.x;
  uint32_t carry = 0;
  uint32_t* row = counts + (int64_t)d * nb;
  for (int64_t b0 = 0; b0 < nb; b0 += kThreads) {
    const int64_t b = b0 + threadIdx.x;
    const uint32_t v = b < nb ? row[b] : 0u;
    const uint32_t ex = block_excl_scan(v, scan_tmp);
    if (threadIdx.x == kThreads - 1) s_last = ex + v;
    __syncthreads();
    if (b < nb) row[b] = carry + ex;
    carry += s_last;
    __syncthreads();
  }
  if (threadIdx.x == 0) totals[d] = carry;
}

// Stable rank of the workgroup's keys and scatter to the offsets of the
// pass.
template <int kItems>
__global__ void __launch_bounds__(kThreads) downsweep_kernel(const uint32_t* __restrict__ kin,
                                                             const uint32_t* __restrict__ vin,
                                                             uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                             int64_t n, int shift, KeyMap km,
                                                             const uint32_t* __restrict__ offsets, int64_t nb,
                                                             const uint32_t* __restrict__ totals,
                                                             const uint32_t* __restrict__ gather_src,
                                                             uint32_t* __restrict__ gather_dst, uint32_t gather_n,
                                                             unsigned long long* __restrict__ bad_count) {
  constexpr int kTileKeys = kThreads * kItems;
  __shared__ uint32_t skeys[kTileKeys];
  __shared__ uint32_t svals[kTileKeys];
  __shared__ uint32_t wcnt[kWaves][kRadix];
  __shared__ uint32_t blk_start[kRadix];
  __shared__ uint32_t glob_base[kRadix];
  __shared__ uint32_t scan_tmp[kWaves];

  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const uint32_t bid = blockIdx.x;
  for (int i = tid; i < kWaves * kRadix; i += kThreads) (&wcnt[0][0])[i] = 0u;
  // start of digit tid's run in the output: keys with a smaller digit, plus
  // keys with this digit in earlier workgroups
  {
    const uint32_t gb = block_excl_scan(tid < kRadix ? totals[tid] : 0u, scan_tmp);
    if (tid < kRadix) glob_base[tid] = gb + offsets[(int64_t)tid * nb + bid];
  }
  __syncthreads();
  const int64_t wave_base = (int64_t)bid * kTileKeys + (int64_t)wid * (kItems * 64);
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

  uint32_t k[kItems];
  uint32_t v[kItems];
  uint32_t rank[kItems];
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const int64_t idx = wave_base + r * 64 + lane;
    const bool valid = idx < n;
    k[r] = valid ? kin[idx] : 0xffffffffu;
    v[r] = valid ? vin[idx] : 0u;
  }
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const int64_t idx = wave_base + r * 64 + lane;
    const bool valid = idx < n;
    const uint32_t d = digit_of(k[r], km, shift);
    // lanes of this row holding the same digit, from one ballot per digit bit
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      m &= bit ? bb : ~bb;
    }
    const uint32_t below = (uint32_t)__popcll(m & lt_mask);
    const uint32_t cnt = (uint32_t)__popcll(m);
    uint32_t old = 0;
    if (valid) old = wcnt[wid][d];
    rank[r] = old + below;
    if (valid && below == 0) wcnt[wid][d] = old + cnt;
  }
  __syncthreads();

  // Per digit: offsets of the waves and the workgroup's digit starts.
  const int d = tid;
  uint32_t dsum = 0;
  if (d < kRadix) {
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      const uint32_t c = wcnt[w][d];
      wcnt[w][d] = dsum;
      dsum += c;
    }
  }
  {
    const uint32_t bs = block_excl_scan(dsum, scan_tmp);
    if (d < kRadix) blk_start[d] = bs;
  }
  // The scan's own barriers come before this write, and the placement below
  // reads the starts of digits that other waves own: a barrier of its own.
  __syncthreads();

  // Stable local order in LDS, then a coalesced scatter per digit run.
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const int64_t idx = wave_base + r * 64 + lane;
    if (idx < n) {
      const uint32_t dd = digit_of(k[r], km, shift);
      const uint32_t pos = blk_start[dd] + wcnt[wid][dd] + rank[r];
      skeys[pos] = k[r];
      svals[pos] = v[r];
    }
  }
  __syncthreads();
  const int64_t left = n - (int64_t)bid * kTileKeys;
  const int count = left < kTileKeys ? (int)left : kTileKeys;
  for (int i = tid; i < count; i += kThreads) {
    const uint32_t key = skeys[i];
    const uint32_t dd = digit_of(key, km, shift);
    const uint32_t o = glob_base[dd] + (uint32_t)i - blk_start[dd];
    if (o < (uint64_t)n) {  // always true for a correct ranking
      const uint32_t val = svals[i];
      kout[o] = key;
      vout[o] = val;
      if (gather_dst) {  // the caller's per-value array, in sorted order
        if (val < gather_n) {
          gather_dst[o] = gather_src[val];
        } else {  // a value that cannot index the array: counted, never read
          gather_dst[o] = 0u;
          atomicAdd(bad_count, 1ull);
        }
      }
    } else {
      atomicAdd(bad_count, 1ull);
    }
  }
}

// One 8-bit pass: digit counts per workgroup, their scan, the downsweep.
template <int kItems>
void sort_pass(uint32_t* keys[2], uint32_t* vals[2], int cur, int64_t n, int p, KeyMap km, uint32_t* counts,
               int64_t nb, uint32_t* totals, const uint32_t* gs, uint32_t* gd, int64_t gather_n,
               unsigned long long* bad_count, hipStream_t stream) {
  upsweep_kernel<kItems><<<dim3((unsigned)nb), kThreads, 0, stream>>>(keys[cur], n, 8 * p, km, counts, nb);
  digit_offsets_kernel<<<dim3(kRadix), kThreads, 0, stream>>>(counts, nb, totals);
  downsweep_kernel<kItems><<<dim3((unsigned)nb), kThreads, 0, stream>>>(keys[cur], vals[cur], keys[cur ^ 1],
                                                                       vals[cur ^ 1], n, 8 * p, km, counts, nb, totals,
                                                                       gs, gd, (uint32_t)gather_n, bad_count);
}

}  // namespace

int64_t sort_scratch_entries(int64_t n) {
  const int64_t tile = (int64_t)kThreads * sort_items(n);
  const int64_t nb = (n + tile - 1) / tile;
  return (int64_t)kRadix * (nb > 0 ? nb : 1);  // digit counts / offsets [256][nb]
}

// Stable sort of (key, value) by min(key - bias, lim), whose n_bits low bits
// are all that vary. totals: 256 words of scratch. If gather_dst is given,
// the last pass also writes gather_dst[i] = gather_src[value i] for values
// below gather_n (gather_src's length). bad_count: a device counter that
// every value at or past gather_n and every out-of-range output position
// increments (0 for a correct ranking).
hipError_t launch_radix_sort(uint32_t* keys[2], uint32_t* vals[2], int64_t n, int n_bits, uint32_t bias,
                             uint32_t lim, uint32_t* scratch, uint32_t* totals, int* result_buffer,
                             hipStream_t stream, unsigned long long* bad_count, const uint32_t* gather_src,
                             uint32_t* gather_dst, int64_t gather_n) {
  *result_buffer = 0;
  if (n <= 1 || n_bits <= 0) return hipSuccess;
  if (gather_dst && (!gather_src || gather_n <= 0 || gather_n > 0xffffffffll)) return hipErrorInvalidValue;
  const int n_pass = (n_bits + 7) / 8;
  if (n_pass > kMaxPasses) return hipErrorInvalidValue;
  const int items = sort_items(n);
  const int64_t tile = (int64_t)kThreads * items;
  const int64_t nb = (n + tile - 1) / tile;
  uint32_t* counts = scratch;
  const KeyMap km{bias, lim};
  hipError_t e;
  int cur = 0;
  for (int p = 0; p < n_pass; ++p) {
    const bool last = p == n_pass - 1;
    const uint32_t* gs = last ? gather_src : nullptr;
    uint32_t* gd = last ? gather_dst : nullptr;
    if (items == kSmallSortItems)
      sort_pass<kSmallSortItems>(keys, vals, cur, n, p, km, counts, nb, totals, gs, gd, gather_n, bad_count, stream);
    else if (items == kMidSortItems)
      sort_pass<kMidSortItems>(keys, vals, cur, n, p, km, counts, nb, totals, gs, gd, gather_n, bad_count, stream);
    else
      sort_pass<kLargeSortItems>(keys, vals, cur, n, p, km, counts, nb, totals, gs, gd, gather_n, bad_count, stream);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    cur ^= 1;
  }
  *result_buffer = cur;
  return hipSuccess;
}

}  // namespace adr
