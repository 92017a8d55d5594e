// InclusiveSum (Sec. 3.2, stage 2): offsets of each Gaussian's pairs, taken
// over the Gaussians in depth order (out[r] = sum of in[r'] for r' <= r; the
// depth sort's last pass writes tiles_touched in that order).
// Reduce-then-scan in two launches: per-block totals, then each block adds up
// the totals of the blocks before it (a few hundred words, read from L2) and
// rescans its 2048 entries from that prefix. The rescan also records, for
// every chunk of kDupPairs pairs, the Gaussian whose pairs [out[r-1], out[r])
// hold the chunk's first pair, so that each DuplicateWithKeys workgroup finds
// its Gaussians with one load instead of a search.
#include "adr_internal.h"

namespace adr {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanBlock = kScanThreads * kScanItems;  // 2048 entries per block

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, int lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t u = __shfl_up(v, off, 64);
    if (lane >= off) v += u;
  }
  return v;
}

// Inclusive scan of one value per thread over a 256-thread block; returns
// the thread's inclusive prefix and writes the block total to *total.
__device__ __forceinline__ uint32_t block_incl_scan(uint32_t v, uint32_t* smem4, uint32_t* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t s = wave_incl_scan(v, lane);
  if (lane == 63) smem4[wid] = s;
  __syncthreads();
  uint32_t before = 0;
  for (int w = 0; w < wid; ++w) before += smem4[w];
  *total = smem4[0] + smem4[1] + smem4[2] + smem4[3];
  __syncthreads();
  return s + before;
}

__global__ void __launch_bounds__(kScanThreads) block_totals_kernel(const uint32_t* __restrict__ in, int64_t n,
                                                                    uint32_t* __restrict__ partials) {
  __shared__ uint32_t smem[4];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + threadIdx.x * kScanItems;
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n) s += in[base + i];
  uint32_t total;
  (void)block_incl_scan(s, smem, &total);
  if (threadIdx.x == 0) partials[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kScanThreads) scan_blocks_kernel(const uint32_t* __restrict__ in, int64_t n,
                                                                   const uint32_t* __restrict__ partials,
                                                                   uint32_t* __restrict__ out,
                                                                   uint32_t* __restrict__ dup_first) {
  __shared__ uint32_t smem[4];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = base + i < n ? in[base + i] : 0u;
    s += v[i];
  }
  // prefix of the earlier blocks' totals
  uint32_t before = 0;
  for (int64_t b = threadIdx.x; b < (int64_t)blockIdx.x; b += kScanThreads) before += partials[b];
  uint32_t total, prefix;
  (void)block_incl_scan(before, smem, &prefix);
  const uint32_t incl = block_incl_scan(s, smem, &total);
  uint32_t run = prefix + incl - s;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const uint32_t before = run;
    run += v[i];
    if (base + i < n) {
      out[base + i] = run;
      // chunks c whose first pair c * kDupPairs lies in [before, run)
      for (uint64_t c = ((uint64_t)before + kDupPairs - 1) / kDupPairs; c * kDupPairs < run; ++c)
        dup_first[c] = (uint32_t)(base + i);
    }
  }
}

}  // namespace

int64_t inclusive_sum_partials(int64_t n) { return (n + kScanBlock - 1) / kScanBlock; }

// dup_first: duplicate_blocks(total of in) words
hipError_t launch_inclusive_sum(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* partials,
                                uint32_t* dup_first, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const int64_t nb = inclusive_sum_partials(n);
  block_totals_kernel<<<dim3((unsigned)nb), kScanThreads, 0, stream>>>(in, n, partials);
  scan_blocks_kernel<<<dim3((unsigned)nb), kScanThreads, 0, stream>>>(in, n, partials, out, dup_first);
  return hipGetLastError();
}

}  // namespace adr
