// SortPairs (Sec. 3.2, stage 4): stable LSD radix sort of (u64 key, u32 id)
// pairs over the key bits that can be non-zero (32 depth bits plus the tile
// id bits), 8 bits per pass.
//
// One histogram launch reads the keys once and counts the digits of every
// pass. Each pass is then a single launch in the "onesweep" style (Adinets &
// Merrill 2022): a workgroup ranks 4096 keys in LDS, publishes its per-digit
// counts, obtains the counts of all earlier workgroups by decoupled
// look-back, and scatters. Ranking is stable and uses wave64 ballots: the
// lanes of a row that share a digit are found with eight ballots, one per
// digit bit, and counted with popcounts, so no LDS atomics decide an order.
#include "adr_internal.h"

namespace adr {

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 16;
constexpr int kTileKeys = kThreads * kItems;  // 4096 keys per workgroup
constexpr int kRadix = 256;
constexpr int kMaxPasses = 8;
constexpr uint32_t kFlagAggregate = 1u << 30;
constexpr uint32_t kFlagInclusive = 2u << 30;
constexpr uint32_t kValueMask = (1u << 30) - 1;
constexpr uint32_t kSpinLimit = 1u << 22;

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

__global__ void __launch_bounds__(kThreads) digit_histogram_kernel(const uint64_t* __restrict__ keys, int64_t n,
                                                                   int n_pass, uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[kMaxPasses][kRadix];
  for (int i = threadIdx.x; i < kMaxPasses * kRadix; i += kThreads) (&h[0][0])[i] = 0u;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) {
    const uint64_t k = keys[i];
    for (int p = 0; p < n_pass; ++p) atomicAdd(&h[p][(k >> (8 * p)) & 0xff], 1u);
  }
  __syncthreads();
  for (int p = 0; p < n_pass; ++p) {
    const uint32_t c = h[p][threadIdx.x];
    if (c) atomicAdd(&hist[p * kRadix + threadIdx.x], c);
  }
}

__global__ void __launch_bounds__(kThreads) onesweep_kernel(const uint64_t* __restrict__ kin,
                                                            const uint32_t* __restrict__ vin,
                                                            uint64_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                            int64_t n, int shift, const uint32_t* __restrict__ hist,
                                                            uint32_t* __restrict__ status,
                                                            uint32_t* __restrict__ tile_counter,
                                                            unsigned long long* __restrict__ err) {
  __shared__ uint64_t skeys[kTileKeys];
  __shared__ uint32_t svals[kTileKeys];
  __shared__ uint32_t wcnt[4][kRadix];
  __shared__ uint32_t blk_start[kRadix];
  __shared__ uint32_t glob_base[kRadix];
  __shared__ uint32_t scan_tmp[4];
  __shared__ uint32_t s_bid;

  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  if (tid == 0) s_bid = atomicAdd(tile_counter, 1u);
  for (int i = tid; i < 4 * kRadix; i += kThreads) (&wcnt[0][0])[i] = 0u;
  __syncthreads();
  const uint32_t bid = s_bid;
  const int64_t wave_base = (int64_t)bid * kTileKeys + (int64_t)wid * (kItems * 64);
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

  uint64_t k[kItems];
  uint32_t v[kItems];
  uint32_t rank[kItems];
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const int64_t idx = wave_base + r * 64 + lane;
    const bool valid = idx < n;
    k[r] = valid ? kin[idx] : ~0ull;
    v[r] = valid ? vin[idx] : 0u;
    const uint32_t d = (uint32_t)(k[r] >> shift) & 0xffu;
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

  // Per digit: offsets of the four waves and the workgroup total.
  const int d = tid;
  const uint32_t c0 = wcnt[0][d], c1 = wcnt[1][d], c2 = wcnt[2][d], c3 = wcnt[3][d];
  const uint32_t tot = c0 + c1 + c2 + c3;
  wcnt[0][d] = 0u;
  wcnt[1][d] = c0;
  wcnt[2][d] = c0 + c1;
  wcnt[3][d] = c0 + c1 + c2;
  uint32_t* my_status = status + (int64_t)bid * kRadix + d;
  __hip_atomic_store(my_status, (bid == 0 ? kFlagInclusive : kFlagAggregate) | tot, __ATOMIC_RELEASE,
                     __HIP_MEMORY_SCOPE_AGENT);
  blk_start[d] = block_excl_scan(tot, scan_tmp);
  const uint32_t digit_base = block_excl_scan(hist[d], scan_tmp);

  // Decoupled look-back over earlier workgroups, one digit per thread.
  uint32_t excl = 0;
  if (bid > 0) {
    int64_t j = (int64_t)bid - 1;
    uint32_t spins = 0;
    while (true) {
      const uint32_t s = __hip_atomic_load(status + j * kRadix + d, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
      const uint32_t flag = s & ~kValueMask;
      if (flag == 0u) {
        if (++spins > kSpinLimit) {  // never expected; guarantees termination
          atomicAdd(err, 1ull);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
        continue;
      }
      excl += s & kValueMask;
      if (flag == kFlagInclusive || j == 0) break;
      --j;
    }
    __hip_atomic_store(my_status, kFlagInclusive | (excl + tot), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
  glob_base[d] = digit_base + excl;
  __syncthreads();

  // Stable local order in LDS, then a coalesced scatter per digit run.
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const int64_t idx = wave_base + r * 64 + lane;
    if (idx < n) {
      const uint32_t dd = (uint32_t)(k[r] >> shift) & 0xffu;
      const uint32_t pos = blk_start[dd] + wcnt[wid][dd] + rank[r];
      skeys[pos] = k[r];
      svals[pos] = v[r];
    }
  }
  __syncthreads();
  const int64_t left = n - (int64_t)bid * kTileKeys;
  const int count = left < kTileKeys ? (int)left : kTileKeys;
  for (int i = tid; i < count; i += kThreads) {
    const uint64_t key = skeys[i];
    const uint32_t dd = (uint32_t)(key >> shift) & 0xffu;
    const uint32_t o = glob_base[dd] + (uint32_t)i - blk_start[dd];
    if (o < (uint64_t)n) {  // always true for a correct ranking; keeps a fault impossible
      kout[o] = key;
      vout[o] = svals[i];
    }
  }
}

}  // namespace

int64_t sort_hist_entries(int64_t n_pairs) {
  const int64_t nb = (n_pairs + kTileKeys - 1) / kTileKeys;
  // per pass: status[nb][256], then counters[kMaxPasses], hist[kMaxPasses][256]
  return (int64_t)kMaxPasses * nb * kRadix + kMaxPasses + kMaxPasses * kRadix;
}

hipError_t launch_sort_pairs(SortBuffers& sb, int64_t n_pairs, int n_bits, int* result_buffer,
                             hipStream_t stream) {
  *result_buffer = 0;
  if (n_pairs <= 1) return hipSuccess;
  const int n_pass = (n_bits + 7) / 8;
  if (n_pass > kMaxPasses) return hipErrorInvalidValue;
  const int64_t nb = (n_pairs + kTileKeys - 1) / kTileKeys;
  uint32_t* status = sb.block_hist;
  uint32_t* counters = status + (int64_t)kMaxPasses * nb * kRadix;
  uint32_t* hist = counters + kMaxPasses;
  hipError_t e = launch_fill_u32(sb.block_hist, 0u, (int64_t)n_pass * nb * kRadix, stream);
  if (e == hipSuccess) e = launch_fill_u32(counters, 0u, kMaxPasses + kMaxPasses * kRadix, stream);
  if (e != hipSuccess) return e;
  int64_t hist_blocks = (n_pairs + kThreads * 16 - 1) / (kThreads * 16);
  if (hist_blocks > 2048) hist_blocks = 2048;
  digit_histogram_kernel<<<dim3((unsigned)hist_blocks), kThreads, 0, stream>>>(sb.keys[0], n_pairs, n_pass, hist);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  int cur = 0;
  for (int p = 0; p < n_pass; ++p) {
    onesweep_kernel<<<dim3((unsigned)nb), kThreads, 0, stream>>>(
        sb.keys[cur], sb.vals[cur], sb.keys[cur ^ 1], sb.vals[cur ^ 1], n_pairs, 8 * p, hist + p * kRadix,
        status + (int64_t)p * nb * kRadix, counters + p, sb.err);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    cur ^= 1;
  }
  *result_buffer = cur;
  return hipSuccess;
}

}  // namespace adr
