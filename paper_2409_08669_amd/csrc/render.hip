// Render (Sec. 3.2, stage 6): pixel-parallel, Gaussian-serial front-to-back
// blending (Eqs. 2-3), per-pixel load counters (Eq. 12) and the
// load-balancing cap.
//
// Layout: one 256-lane workgroup per 16 x 16 tile; each wave64 owns an 8 x 8
// quadrant, split into four 4 x 4 sub-blocks of 16 lanes, and walks the
// tile's depth-sorted list on its own. Per batch of 64 list entries every
// lane loads one id and that Gaussian's cull box (8 bytes) and tests it
// against the four sub-blocks; the record of every entry that meets one is
// staged in LDS, and each sub-block gets the list of its own entries
// (compacted with ballots, in list order). The wave then steps through the
// four lists together: on each step the 16 lanes of a sub-block evaluate that
// sub-block's next Gaussian. An entry whose box misses a sub-block has
// alpha < alpha_low at all its pixels, so skipping it changes nothing; a
// Gaussian is evaluated only by the lanes whose pixels it can reach.
//
// Precision: the record centre is made quadrant-relative in FP64 before the
// FP32 evaluation. The skip decision alpha < alpha_low is re-taken in FP64
// when the FP32 exponent falls in a narrow band around log2(alpha_low); when
// a transmittance lands in a narrow band around t_min the whole wave
// recomputes that pixel's transmittance in FP64 over the list so far, and the
// stop decision uses that value. The blended sequence and the load counters
// therefore follow an FP64 evaluation of the same definition.
#include "adr_internal.h"

namespace adr {

namespace {

struct alignas(16) Staged {
  float4 a;  // x - qx0, y - qy0, rc, rs
  float4 b;  // a1, a2, ql, exponent band (the FP32 error bound + floor)
};

constexpr int kSub = 4;  // 4 x 4 pixel sub-blocks, 16 lanes each

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    lo = __shfl_xor(lo, off, 64);
    hi = __shfl_xor(hi, off, 64);
    v += ((unsigned long long)hi << 32) | lo;
  }
  return v;
}

__device__ __forceinline__ double wave_prod_f64(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    uint32_t lo = (uint32_t)u, hi = (uint32_t)(u >> 32);
    lo = __shfl_xor(lo, off, 64);
    hi = __shfl_xor(hi, off, 64);
    v *= __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
  }
  return v;
}

__device__ __forceinline__ bool box_has(uint32_t bx, uint32_t by, int i, int j) {
  return (int)(bx & 0xffffu) <= i && (int)(bx >> 16) >= i && (int)(by & 0xffffu) <= j && (int)(by >> 16) >= j;
}

// FP64 splatting opacity at pixel (pi, pj) (Eq. 2), clamped at alpha_max.
__device__ __forceinline__ double alpha_fp64(const ExactRecord& e, double x, double y, int pi, int pj,
                                             double alpha_max) {
  const double dx = x - (double)pi, dy = y - (double)pj;
  const double power = -0.5 * (e.ca * dx * dx + 2.0 * e.cb * dx * dy + e.cc * dy * dy);
  return fmin(alpha_max, e.opacity * exp(power));
}

// The out-of-line FP64 helpers below receive generic pointers; reading
// through global-address-space pointers lets their loads be waited for one by
// one (a generic load also counts as an LDS access, so every wait for one
// would wait for all).
template <class T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* global_ptr(const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}

// FP64 alpha of Gaussian g at pixel (pi, pj); kept out of line so the rare
// FP64 path does not raise the register count of the blend loop.
__device__ __noinline__ double alpha_fp64_at(const RenderRecord* __restrict__ rec_,
                                             const ExactRecord* __restrict__ exact_, uint32_t g, int pi, int pj,
                                             double alpha_max) {
  const auto* rec = global_ptr(rec_);
  const auto* exact = global_ptr(exact_);
  ExactRecord e;
  e.ca = exact[g].ca;
  e.cb = exact[g].cb;
  e.cc = exact[g].cc;
  e.opacity = exact[g].opacity;
  const double x = rec[g].x, y = rec[g].y;
  return alpha_fp64(e, x, y, pi, pj, alpha_max);
}

// log2-domain exponent of a staged Gaussian at the lane's pixel (lx, ly),
// on its principal axes: every term has the sign of its sum.
__device__ __forceinline__ float quad_form(const float4& A, const float4& B, float fx, float fy) {
  const float dx = A.x - fx, dy = A.y - fy;
  const float u = fmaf(A.z, dx, -(A.w * dy));
  const float v = fmaf(A.w, dx, A.z * dy);
  return fmaf(-(B.x * u), u, fmaf(-(B.y * v), v, B.z));
}

// FP64 transmittance of pixel (ri, rj) after list entries [s, k_now]: the
// wave's lanes take every 64th entry and the partial products are combined.
// A lane's id loads run two entries ahead and its box loads one entry ahead
// (clamped to the range, so none waits on a branch); the FP64 record of an
// entry whose box holds the pixel is read with a single wait. A lane's
// product runs over its entries in list order.
__device__ __noinline__ double replay_fp64(const RenderRecord* __restrict__ rec_,
                                           const ExactRecord* __restrict__ exact_,
                                           const uint32_t* __restrict__ vals_, uint32_t n_gauss, uint32_t s,
                                           uint32_t k_now, int ri, int rj, int lane, const BlendArgs& bl) {
  const auto* rec = global_ptr(rec_);
  const auto* exact = global_ptr(exact_);
  const auto* vals = global_ptr(vals_);
  const double alpha_max = bl.alpha_max_d, alpha_low = bl.alpha_low_d;
  double prod = 1.0;
  uint64_t kk = (uint64_t)s + lane;
  const uint64_t kl = k_now;
  uint32_t g = min(vals[min(kk, kl)], n_gauss - 1);
  uint32_t g_n = min(vals[min(kk + 64, kl)], n_gauss - 1);
  uint32_t bx = rec[g].box_x, by = rec[g].box_y;
  for (; kk <= kl; kk += 64) {
    const uint32_t bx_n = rec[g_n].box_x, by_n = rec[g_n].box_y;
    const uint32_t raw_nn = vals[min(kk + 128, kl)];
    if (box_has(bx, by, ri, rj)) {
      ExactRecord e;
      e.ca = exact[g].ca;
      e.cb = exact[g].cb;
      e.cc = exact[g].cc;
      e.opacity = exact[g].opacity;
      const double ad = alpha_fp64(e, rec[g].x, rec[g].y, ri, rj, alpha_max);
      if (ad >= alpha_low) prod *= 1.0 - ad;
    }
    g = g_n;
    bx = bx_n;
    by = by_n;
    g_n = min(raw_nn, n_gauss - 1);
  }
  return wave_prod_f64(prod);
}

// Marks v as needed here: its load stays where it was issued, one loop
// iteration ahead of its use, instead of being moved down next to the use
// (where its latency would stall the step).
__device__ __forceinline__ void ready(const float4& v) {
  asm volatile("" ::"v"(v.x), "v"(v.y), "v"(v.z), "v"(v.w));
}

// Makes v available only from here on: nothing computed from it (a store
// included) is moved above this point, so its load is waited for here.
__device__ __forceinline__ void from_here(float4& v) {
  asm volatile("" : "+v"(v.x), "+v"(v.y), "+v"(v.z), "+v"(v.w));
}

__device__ __forceinline__ void ready(float v) { asm volatile("" ::"v"(v)); }

// Index of the lowest set bit of m, which is cleared; 64 (the null slot)
// once m is empty.
__device__ __forceinline__ int next_slot(uint64_t& m) {
  const int slot = m ? (int)__builtin_ctzll(m) : 64;
  m &= m - 1;
  return slot;
}

// Cull box of Gaussian g (first 8 bytes of its record).
__device__ __forceinline__ uint2 load_box(const RenderRecord* __restrict__ rec, uint32_t g) {
  return *reinterpret_cast<const uint2*>(&rec[g].box_x);
}

// The box of a list position past the list's end: lo 65535, hi 0 on both
// axes. It meets no sub-block: a column test needs hi >= qx0, so qx0 = 0,
// and there lo <= qx0 + 7 fails (a box with lo 1, hi 0 would pass both at
// the image's first quadrant).
__device__ __forceinline__ uint2 no_box() { return make_uint2(0xffffu, 0xffffu); }

// Ballots of one batch: bit l of m[t] is set when the box of lane l's entry
// meets sub-block t of the quadrant at (qx0, qy0).
struct SubMasks {
  uint64_t m[4];
  __device__ bool any_lane(int lane) const { return (((m[0] | m[1] | m[2] | m[3]) >> lane) & 1ull) != 0; }
};

__device__ __forceinline__ SubMasks sub_masks(uint2 box, int qx0, int qy0) {
  const int bxl = (int)(box.x & 0xffffu), bxh = (int)(box.x >> 16);
  const int byl = (int)(box.y & 0xffffu), byh = (int)(box.y >> 16);
  const bool c0 = bxl <= qx0 + 3 && bxh >= qx0, c1 = bxl <= qx0 + 7 && bxh >= qx0 + 4;
  const bool r0 = byl <= qy0 + 3 && byh >= qy0, r1 = byl <= qy0 + 7 && byh >= qy0 + 4;
  SubMasks s;
  s.m[0] = __ballot(c0 && r0);
  s.m[1] = __ballot(c1 && r0);
  s.m[2] = __ballot(c0 && r1);
  s.m[3] = __ballot(c1 && r1);
  return s;
}

// The part of a render record the batch staging needs (centre, exponent
// coefficients, error bound), loaded one batch ahead of its use.
struct Fetched {
  double x, y;
  float4 q;  // rc, rs, a1, a2
  float ql;
  float dq;  // exponent error bound
};

__device__ __forceinline__ Fetched fetch(const RenderRecord* __restrict__ rec, uint32_t g) {
  const RenderRecord& r = rec[g];
  Fetched f;
  f.x = r.x;
  f.y = r.y;
  f.q = *reinterpret_cast<const float4*>(&r.rc);
  f.ql = r.ql;
  f.dq = r.dq;
  return f;
}

// Longest lists first: workgroups start in launch order, so the tiles whose
// waves run longest (the heavy-load pixels of Sec. 4.4) start first and the
// short ones fill in around them. Buckets of floor(log2(length)), longest
// bucket first; the order inside a bucket does not affect any output.
constexpr int kOrderBuckets = 33;

__device__ __forceinline__ int order_bucket(const uint32_t* __restrict__ ranges, int t, uint32_t n_pairs) {
  const uint32_t e = min(ranges[2 * t + 1], n_pairs), s = min(ranges[2 * t], e);
  const uint32_t len = e - s;
  return len == 0 ? kOrderBuckets - 1 : (kOrderBuckets - 2) - (31 - __clz(len));
}

// Lanes of the wave whose bucket equals this lane's (6 ballots over its bits).
__device__ __forceinline__ uint64_t same_bucket(int b, bool valid) {
  uint64_t m = __ballot(valid);
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const bool bit = (b >> k) & 1;
    const uint64_t bb = __ballot(bit);
    m &= bit ? bb : ~bb;
  }
  return m;
}

// Counting sort of the tiles by bucket in two launches, one workgroup per
// superblock of 16 x 16 tiles: per-block bucket counts, then each block finds
// its buckets' bases (all blocks' counts are a few thousand words at most)
// and scatters its tiles. Each wave groups its tiles by bucket with ballots,
// so LDS atomics are per bucket per wave rather than per tile.
//
// Inside a bucket the tiles are ranked in scan order (superblocks row by
// row, each row-major inside) and the ranks are dealt to the XCDs in
// contiguous runs: the render's workgroup at position p runs on XCD p mod 8,
// so the k-th eighth of every bucket's ranks takes the bucket's positions
// with p mod 8 = k. Tiles that run on one XCD at the same time are then
// neighbours, which share most of their Gaussians, and the records those
// tiles read are fetched into that XCD's L2 once rather than once per XCD.
constexpr int kOrderBlock = 256;
constexpr int kOrderSuper = 16;  // superblock side in tiles (kOrderSuper^2 = kOrderBlock)
constexpr int kXcds = 8;

// This lane's tile of the superblock blockIdx.x, or valid = false past the grid.
__device__ __forceinline__ int superblock_tile(int tiles_x, int tiles_y, bool& valid) {
  const int n_sbx = (tiles_x + kOrderSuper - 1) / kOrderSuper;
  const int tx = ((int)blockIdx.x % n_sbx) * kOrderSuper + ((int)threadIdx.x % kOrderSuper);
  const int ty = ((int)blockIdx.x / n_sbx) * kOrderSuper + ((int)threadIdx.x / kOrderSuper);
  valid = tx < tiles_x && ty < tiles_y;
  return valid ? ty * tiles_x + tx : 0;
}

// Position of rank r among the n tiles of the bucket whose positions start
// at b0: residue k = 0, 1, ... takes the next run of ranks, placed at the
// bucket's positions p with p mod 8 = k in increasing order (a bijection of
// [0, n) onto [b0, b0 + n)).
__device__ __forceinline__ uint32_t xcd_position(uint32_t b0, uint32_t n, uint32_t r) {
  uint32_t start = 0;
#pragma unroll
  for (uint32_t k = 0; k < (uint32_t)kXcds; ++k) {
    const uint32_t first = b0 + (k + kXcds - b0 % kXcds) % kXcds;
    const uint32_t cnt = first < b0 + n ? (b0 + n - first + kXcds - 1) / kXcds : 0u;
    if (r < start + cnt) return first + kXcds * (r - start);
    start += cnt;
  }
  return b0 + r;  // not reached for r < n
}

__global__ void __launch_bounds__(kOrderBlock) order_count_kernel(const uint32_t* __restrict__ ranges, int tiles_x,
                                                                  int tiles_y, uint32_t n_pairs,
                                                                  uint32_t* __restrict__ counts) {
  __shared__ uint32_t cnt[kOrderBuckets];
  const int lane = threadIdx.x & 63;
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  if (threadIdx.x < kOrderBuckets) cnt[threadIdx.x] = 0u;
  __syncthreads();
  bool valid;
  const int t = superblock_tile(tiles_x, tiles_y, valid);
  const int b = valid ? order_bucket(ranges, t, n_pairs) : 0;
  const uint64_t m = same_bucket(b, valid);
  if (valid && (m & lt) == 0) atomicAdd(&cnt[b], (uint32_t)__popcll(m));
  __syncthreads();
  if (threadIdx.x < kOrderBuckets) counts[threadIdx.x * gridDim.x + blockIdx.x] = cnt[threadIdx.x];
}

__global__ void __launch_bounds__(kOrderBlock) order_scatter_kernel(const uint32_t* __restrict__ ranges, int tiles_x,
                                                                    int tiles_y, uint32_t n_pairs,
                                                                    const uint32_t* __restrict__ counts,
                                                                    uint32_t* __restrict__ order) {
  __shared__ uint32_t base[kOrderBuckets];    // first position of the bucket
  __shared__ uint32_t total[kOrderBuckets];   // tiles in the bucket
  __shared__ uint32_t before[kOrderBuckets];  // the bucket's tiles in earlier blocks
  __shared__ uint32_t wave_cnt[kOrderBlock / 64][kOrderBuckets];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int nb = gridDim.x;
  const uint32_t n_tiles = (uint32_t)tiles_x * (uint32_t)tiles_y;
  if (threadIdx.x < kOrderBuckets) {
    uint32_t tot = 0, bef = 0;
    for (int k = 0; k < nb; ++k) {
      const uint32_t c = counts[threadIdx.x * nb + k];
      tot += c;
      bef += k < (int)blockIdx.x ? c : 0u;
    }
    before[threadIdx.x] = bef;
    total[threadIdx.x] = tot;
  }
  for (int i = threadIdx.x; i < (kOrderBlock / 64) * kOrderBuckets; i += kOrderBlock) (&wave_cnt[0][0])[i] = 0u;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int k = 0; k < kOrderBuckets; ++k) {
      base[k] = run;
      run += total[k];
    }
  }
  bool valid;
  const int t = superblock_tile(tiles_x, tiles_y, valid);
  const int b = valid ? order_bucket(ranges, t, n_pairs) : 0;
  const uint64_t m = same_bucket(b, valid);
  if (valid && (m & lt) == 0) wave_cnt[wid][b] = (uint32_t)__popcll(m);
  __syncthreads();
  if (valid) {
    uint32_t r = before[b] + (uint32_t)__popcll(m & lt);
    for (int w = 0; w < wid; ++w) r += wave_cnt[w][b];
    const uint32_t pos = xcd_position(base[b], total[b], r);
    if (pos < n_tiles) order[pos] = (uint32_t)t;
  }
}

// Per-pixel blend state (Eqs. 2-3) and its load counters.
struct Pixel {
  float T, cr, cg, cb;
  float D;          // bound on |T - T_fp64|
  uint32_t nb;      // blended entries (l_blend)
  uint32_t stop_k;  // list position of the entry that stopped the pixel
  uint32_t n_rare;   // FP64 re-decisions (low 16 bits) and replays (high 16 bits)
};

// One front-to-back blend of the Gaussian staged in slot (A, B, and C: colour
// and alpha's relative error bound) at the lane's pixel; returns the lanes
// whose pixel stops at this entry. The FP32
// exponent decides alpha >= alpha_low unless it lies within the Gaussian's
// error band of log2(alpha_low), where FP64 decides. D bounds the error of
// the FP32 transmittance: T' = T (1 - a) carries the old error scaled by
// (1 - a), plus T a times alpha's relative error (the exponent bound times
// ln 2, plus the exp2 and rounding error), plus the rounding of T' (counted
// as 2^-23 T', which also covers the product terms of errors left out). When
// T lands within 1.5 D (plus t_min's rounding) of t_min, the whole wave
// recomputes the pixel's transmittance in FP64 over the list so far, and that
// value decides the stop. A lane that has stopped evaluates only the null
// record (exponent -1e30, band 0), which changes nothing. Every lane of the
// wave must call it.
template <bool kCap>
__device__ __forceinline__ uint64_t blend_step(Pixel& px, const float4& A, const float4& B, const float4& col,
                                               int slot, uint32_t base, const uint32_t* gids, float fx, float fy,
                                               int pi, int pj, int lane, uint32_t cap, uint32_t s,
                                               const RenderRecord* __restrict__ rec,
                                               const ExactRecord* __restrict__ exact,
                                               const uint32_t* __restrict__ vals, uint32_t n_gauss,
                                               const BlendArgs& bl) {
  // Decisions are kept as wave masks (one bit per lane) so that they combine
  // with scalar instructions.
  const float q = quad_form(A, B, fx, fy);
  const float e2 = __builtin_amdgcn_exp2f(q);
  float a = __builtin_fminf(e2, bl.alpha_max);
  uint64_t blend_m = __ballot(q >= bl.q_low);
  const bool near_low = fabsf(q - bl.q_low) < B.w;
  float af = __builtin_amdgcn_inverse_ballot_w64(blend_m) ? a : 0.f;
  float w = af * px.T;
  float Tn = fmaf(-af, px.T, px.T);  // T (1 - alpha) with one rounding
  float Dn = fmaf(Tn, 0x1p-23f, fmaf(w, col.w, fmaf(-af, px.D, px.D)));
  uint64_t near_t = blend_m & __ballot(fmaf(-bl.t_err_scale, Dn, fabsf(Tn - bl.t_min)) < bl.t_err_floor);
  uint64_t stop_fix = 0;  // lanes whose FP64 stop decision differs from the FP32 test of their replayed T
  if (__builtin_expect((__ballot(near_low) | near_t) != 0, 0)) {
    // Rare (wave-uniform branch): an exponent within its band of
    // log2(alpha_low) is decided in FP64; a transmittance near t_min is
    // recomputed in FP64 by the whole wave over the list so far.
    const uint64_t low_m = __ballot(near_low);
    if (near_low) {
      const double ad = alpha_fp64_at(rec, exact, gids[slot], pi, pj, bl.alpha_max_d);
      const bool blend = ad >= bl.alpha_low_d;
      af = blend ? (float)ad : 0.f;
      w = af * px.T;
      Tn = fmaf(-af, px.T, px.T);
      Dn = fmaf(Tn, 0x1p-23f, fmaf(w, 0x1p-23f, fmaf(-af, px.D, px.D)));  // alpha rounded from FP64
      px.n_rare += 1u;
    }
    if (low_m) {
      const uint64_t low_blend = __ballot(near_low & (af > 0.f));
      blend_m = (blend_m & ~low_m) | low_blend;
      near_t = (near_t & ~low_m) |
               (low_blend & __ballot(fmaf(-bl.t_err_scale, Dn, fabsf(Tn - bl.t_min)) < bl.t_err_floor));
    }
    uint64_t rm = near_t;
    while (rm) {
      const int L = __builtin_ctzll(rm);
      rm &= rm - 1;
      const int ri = __builtin_amdgcn_readlane(pi, L), rj = __builtin_amdgcn_readlane(pj, L);
      const uint32_t k_now = base + (uint32_t)__builtin_amdgcn_readlane(slot, L);
      const double prod = replay_fp64(rec, exact, vals, n_gauss, s, k_now, ri, rj, lane, bl);  // same in all lanes
      stop_fix |= __ballot((prod < bl.t_min_d) != ((float)prod < bl.t_min)) & (1ull << L);
      if (lane == L) {
        Tn = (float)prod;
        Dn = Tn * 0x1p-24f;  // only the rounding to float remains
        px.n_rare += 1u << 16;
      }
    }
  }
  px.cr = fmaf(col.x, w, px.cr);
  px.cg = fmaf(col.y, w, px.cg);
  px.cb = fmaf(col.z, w, px.cb);
  px.T = Tn;
  px.D = Dn;
  px.nb += __builtin_amdgcn_inverse_ballot_w64(blend_m) ? 1u : 0u;
  return blend_m & ((__ballot(Tn < bl.t_min) ^ stop_fix) | (kCap ? __ballot(px.nb == cap) : 0ull));
}

// LDS of one tile's workgroup: per wave, per batch slot (= list position -
// batch start), the staged record, its colour and its Gaussian id (slot 64 is
// a null record), and per step i of the candidate pass a word whose byte t is
// the slot of sub-block t's i-th entry (64 past the end of its list; word 64
// is all 64).
struct TileLds {
  Staged stage[4][65];
  float4 stage_col[4][65];
  uint32_t stage_gid[4][65];
  uint32_t step_table[4][65];
};

// The blend of the tile at position blk of the frame's tile order, by the
// 256 lanes of the calling workgroup.
template <bool kCap>
__device__ __forceinline__ void render_tile(
    TileLds& lds, const RenderRecord* __restrict__ rec, const ExactRecord* __restrict__ exact,
    const uint32_t* __restrict__ vals, const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ order,
    uint32_t n_pairs, uint32_t n_gauss, const CamArgs& cam, const BlendArgs& bl, int n_tiles, int blk,
    float* __restrict__ image, float* __restrict__ final_t, uint32_t* __restrict__ l_iter,
    uint32_t* __restrict__ l_blend, ulonglong4* __restrict__ wave_sums, unsigned long long* __restrict__ counters) {
  auto& stage = lds.stage;
  auto& stage_col = lds.stage_col;
  auto& stage_gid = lds.stage_gid;
  auto& step_table = lds.step_table;
  const int tile = (int)min(order[blk], (uint32_t)(n_tiles - 1));
  const int W = cam.width, H = cam.height;
  const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int qx0 = tx * kTile + (wid & 1) * kQuad;
  const int qy0 = ty * kTile + (wid >> 1) * kQuad;
  if (qx0 >= W || qy0 >= H) {  // quadrant entirely outside the image (wave-uniform)
    if (wave_sums && lane == 0) wave_sums[4 * blk + wid] = make_ulonglong4(0ull, 0ull, 0ull, 0ull);
    return;
  }
  // lane -> pixel: sub-block sb = lane / 16 at (4 (sb & 1), 4 (sb >> 1)) in the quadrant
  const int sb = lane >> 4;
  const int lx = (sb & 1) * kSub + (lane & 3), ly = (sb >> 1) * kSub + ((lane >> 2) & 3);
  const int pi = qx0 + lx, pj = qy0 + ly;
  const bool inside = pi < W && pj < H;
  const float fx = (float)lx, fy = (float)ly;
  Staged* my = stage[wid];
  float4* my_col = stage_col[wid];
  uint32_t* my_gid = stage_gid[wid];
  uint32_t* my_steps = step_table[wid];
  if (lane == 0) {  // exponent -1e30: alpha 0, colour 0; evaluating it changes nothing
    Staged z;
    z.a = make_float4(0.f, 0.f, 0.f, 0.f);
    z.b = make_float4(0.f, 0.f, -1e30f, 0.f);  // q = -1e30 and band 0: never a candidate
    my[64] = z;
    my_col[64] = make_float4(0.f, 0.f, 0.f, 0.f);
    my_gid[64] = 0u;
    my_steps[64] = 0x40404040u;
  }

  // ranges come from this frame's sorted keys; the clamps only make a
  // corrupted table unable to send a load outside the buffers
  const uint32_t e = min(ranges[2 * tile + 1], n_pairs);
  const uint32_t s = min(ranges[2 * tile], e);
  Pixel px;
  px.T = 1.f;
  px.D = 0.f;
  px.cr = px.cg = px.cb = 0.f;
  px.nb = 0;
  px.stop_k = 0xffffffffu;
  px.n_rare = 0;
  bool done = !inside;
  const uint32_t cap = bl.lb_cap > 0 ? (uint32_t)bl.lb_cap : 0xffffffffu;
  // The longest lists bound the kernel's duration: on a shared SIMD, waves
  // issue in order of their list's length relative to the frame's longest
  // (the first tile of the order): at least 3/4, 1/2, 1/4 of it. Wave
  // priority only; no effect on results.
  {
    const int t0 = (int)min(order[0], (uint32_t)(n_tiles - 1));
    const uint32_t e0 = min(ranges[2 * t0 + 1], n_pairs), s0 = min(ranges[2 * t0], e0);
    const uint64_t len0 = e0 - s0, len = e - s;
    if (len * 4 >= len0 * 3)
      __builtin_amdgcn_s_setprio(3);
    else if (len * 2 >= len0)
      __builtin_amdgcn_s_setprio(2);
    else if (len * 4 >= len0)
      __builtin_amdgcn_s_setprio(1);
  }

  // Batches of 64 list entries, software-pipelined: while batch b is
  // evaluated, the records of batch b+1's hits, the cull boxes of batch b+2
  // and the ids of batch b+3 are in flight.
  // Every prefetch load is unconditional, so that nothing waits for it
  // before its use one iteration later: list positions past the end read the
  // last entry (their boxes are replaced by an empty one at use), and lanes
  // whose entry misses the quadrant read record 0 (one shared cache line).
  const uint2 kNoBox = no_box();
  const uint32_t last = e > s ? e - 1 : s;  // the loop below runs only when e > s
  uint32_t g_b = 0, g_n1 = 0, raw_n2 = 0;
  uint2 box_n1 = kNoBox;
  SubMasks hm = sub_masks(kNoBox, qx0, qy0);
  Fetched f_b{};
  if (e > s) {
    g_b = min(vals[min(s + lane, last)], n_gauss - 1);
    g_n1 = min(vals[min(s + 64 + lane, last)], n_gauss - 1);
    raw_n2 = vals[min(s + 128 + lane, last)];
    box_n1 = load_box(rec, g_n1);
    hm = sub_masks(s + lane < e ? load_box(rec, g_b) : kNoBox, qx0, qy0);
    f_b = fetch(rec, hm.any_lane(lane) ? g_b : 0u);
  }
  for (uint32_t base = s; base < e; base += 64) {
    const uint64_t any = hm.m[0] | hm.m[1] | hm.m[2] | hm.m[3];
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    my_steps[lane] = 0x40404040u;  // every entry past a list's end names the null slot
    if ((any >> lane) & 1ull) {
      uint8_t* steps_bytes = reinterpret_cast<uint8_t*>(my_steps);
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if ((hm.m[t] >> lane) & 1ull) steps_bytes[4 * __popcll(hm.m[t] & lt) + t] = (uint8_t)lane;
      Staged st;
      st.a = make_float4((float)(f_b.x - (double)qx0), (float)(f_b.y - (double)qy0), f_b.q.x, f_b.q.y);
      const float band = bl.exact ? f_b.dq + bl.band_floor : 0.f;
      st.b = make_float4(f_b.q.z, f_b.q.w, f_b.ql, band);
      my[lane] = st;
      my_gid[lane] = g_b;
    }
    // colours are needed only by phase 2: their load overlaps phase 1
    float4 col_b = *reinterpret_cast<const float4*>(&rec[((any >> lane) & 1ull) ? g_b : 0u].r);
    // the sub-block's entries of this batch, in list order: the set bits
    const int n_iter = max(max(__popcll(hm.m[0]), __popcll(hm.m[1])), max(__popcll(hm.m[2]), __popcll(hm.m[3])));
    // issue the next batches' loads before evaluating this one
    hm = sub_masks(base + 64 + lane < e ? box_n1 : kNoBox, qx0, qy0);
    g_b = g_n1;
    f_b = fetch(rec, hm.any_lane(lane) ? g_b : 0u);
    g_n1 = min(raw_n2, n_gauss - 1);
    box_n1 = load_box(rec, g_n1);
    raw_n2 = vals[min(base + 192 + lane, last)];
    if (any == 0) continue;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    // Phase 1, candidates: the 16 lanes of a sub-block step through its
    // entries (lowest set bit first) and mark, per pixel, the batch slots
    // whose exponent reaches log2(alpha_low) less twice the Gaussian's
    // band. No step depends on the previous one; two register sets alternate
    // so that each record is read from LDS one step before its use. Every
    // unmarked entry has alpha < alpha_low at this pixel in FP32 and lies
    // outside the band: its blend would leave T and the colour bitwise
    // unchanged. (Steps past a list's end read the null slot.)
    uint64_t cand = 0;
    {
      // Step i reads one word of the batch's step table (the same address
      // for every lane, read two steps ahead) and takes its sub-block's byte:
      // the slot of the sub-block's i-th entry, or 64 past its list's end.
      const uint32_t shift = 8u * (uint32_t)sb;
      auto slot_at = [&](uint32_t word) -> int { return (int)__builtin_amdgcn_ubfe(word, shift, 8u); };
      uint32_t w2 = my_steps[2];
      int s0 = slot_at(my_steps[0]), s1 = slot_at(my_steps[1]);
      float4 A0 = my[s0].a, B0 = my[s0].b, A1, B1;
      ready(A0);
      ready(B0);
#pragma unroll 1
      for (int i = 0; i < n_iter; i += 2) {
        A1 = my[s1].a;
        B1 = my[s1].b;
        const uint32_t w3 = my_steps[min(i + 3, 64)];
        __builtin_amdgcn_sched_barrier(0);  // issue the reads here, one step before their use
        float q = quad_form(A0, B0, fx, fy);
        cand |= (q >= fmaf(-2.f, B0.w, bl.q_low)) ? (1ull << (s0 & 63)) : 0ull;  // never true for slot 64
        s0 = slot_at(w2);
        __builtin_amdgcn_sched_barrier(0);  // the step above completes before the wait below
        ready(A1);
        ready(B1);
        A0 = my[s0].a;
        B0 = my[s0].b;
        w2 = my_steps[min(i + 4, 64)];
        __builtin_amdgcn_sched_barrier(0);
        q = quad_form(A1, B1, fx, fy);
        cand |= (q >= fmaf(-2.f, B1.w, bl.q_low)) ? (1ull << (s1 & 63)) : 0ull;
        s1 = slot_at(w3);
        __builtin_amdgcn_sched_barrier(0);
        ready(A0);
        ready(B0);
      }
    }
    from_here(col_b);  // (not merged into the staging above, which would wait for the load there)
    if ((any >> lane) & 1ull) {
      // w: alpha's relative error bound, the band times ln 2 (rounded up) plus
      // the exp2 error; 1 stands for an unbounded one (those Gaussians are
      // decided in FP64 wherever they are finite, so it never enters D)
      col_b.w = __builtin_fminf(fmaf(bl.exact ? col_b.w + bl.band_floor : 0.f, 0.7f, 0x1p-20f), 1.f);
      my_col[lane] = col_b;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // Phase 2, blending: each lane walks its candidates in slot order, which
    // is list (depth) order, with the exact decision logic; two register
    // sets alternate as above. The wave steps while any lane has candidates
    // left. A lane that stops drops its remaining ones and turns the record
    // already read for its next step into the null record (exponent -1e30 and
    // band 0: a Gaussian decided in FP64 only has an infinite band, which
    // would otherwise send the no-op step down the FP64 path).
    {
      uint64_t cm = done ? 0ull : cand;
      int s0 = next_slot(cm), s1 = next_slot(cm);
      float4 A0 = my[s0].a, B0 = my[s0].b, A1, B1;
      ready(A0);
      ready(B0);
#pragma unroll 1
      while (__ballot(s0 != 64) != 0) {
        const float4 C0 = my_col[s0];  // read before the next step's record, used within this step
        A1 = my[s1].a;
        B1 = my[s1].b;
        __builtin_amdgcn_sched_barrier(0);
        uint64_t stop = blend_step<kCap>(px, A0, B0, C0, s0, base, my_gid, fx, fy, pi, pj, lane, cap, s, rec, exact, vals,
                               n_gauss, bl);
        const int k0 = s0;
        s0 = next_slot(cm);
        __builtin_amdgcn_sched_barrier(0);
        ready(A1);
        ready(B1);
        if (__builtin_expect(stop != 0, 0)) {
          if (__builtin_amdgcn_inverse_ballot_w64(stop)) {
            px.stop_k = base + (uint32_t)k0;
            done = true;
            cm = 0;
            s0 = 64;
            s1 = 64;
            B1 = make_float4(0.f, 0.f, -1e30f, 0.f);  // the null record: band 0 too, so no FP64 path is taken
          }
        }
        if (__ballot(s1 != 64) == 0) break;
        const float4 C1 = my_col[s1];
        A0 = my[s0].a;
        B0 = my[s0].b;
        __builtin_amdgcn_sched_barrier(0);
        stop = blend_step<kCap>(px, A1, B1, C1, s1, base, my_gid, fx, fy, pi, pj, lane, cap, s, rec, exact, vals,
                          n_gauss, bl);
        const int k1 = s1;
        s1 = next_slot(cm);
        __builtin_amdgcn_sched_barrier(0);
        ready(A0);
        ready(B0);
        if (__builtin_expect(stop != 0, 0)) {
          if (__builtin_amdgcn_inverse_ballot_w64(stop)) {
            px.stop_k = base + (uint32_t)k1;
            done = true;
            cm = 0;
            s0 = 64;
            s1 = 64;
            B0 = make_float4(0.f, 0.f, -1e30f, 0.f);
          }
        }
      }
    }
    if (__ballot(!done) == 0) goto finished;
    __builtin_amdgcn_wave_barrier();  // all reads of this batch's slots before the next writes
  }
finished:
  uint32_t ni = 0;
  if (inside) {
    ni = px.stop_k != 0xffffffffu ? px.stop_k - s + 1 : e - s;
    const int64_t pix = (int64_t)pj * W + pi;
    const int64_t plane = (int64_t)W * H;
    image[pix] = px.cr + px.T * bl.bg[0];
    image[plane + pix] = px.cg + px.T * bl.bg[1];
    image[2 * plane + pix] = px.cb + px.T * bl.bg[2];
    if (final_t) final_t[pix] = px.T;
    if (l_iter) l_iter[pix] = ni;
    if (l_blend) l_blend[pix] = px.nb;
  }
  if (wave_sums) {
    // per-wave partial sums for Eq. 13, reduced by load_sums_kernel
    const unsigned long long b1 = wave_sum_u64(px.nb), b2 = wave_sum_u64((unsigned long long)px.nb * px.nb);
    const unsigned long long i1 = wave_sum_u64(ni), i2 = wave_sum_u64((unsigned long long)ni * ni);
    if (lane == 0) wave_sums[4 * blk + wid] = make_ulonglong4(b1, b2, i1, i2);
  }
  if (counters) {
    const unsigned long long nbd = wave_sum_u64(px.n_rare & 0xffffu), nrp = wave_sum_u64(px.n_rare >> 16);
    if (lane == 0) {
      if (nbd) atomicAdd(&counters[kCntBand], nbd);
      if (nrp) atomicAdd(&counters[kCntReplay], nrp);
    }
  }
}

template <bool kCap>
__global__ void __launch_bounds__(256, 4) render_kernel(
    const RenderRecord* __restrict__ rec, const ExactRecord* __restrict__ exact, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ order, uint32_t n_pairs, uint32_t n_gauss,
    CamArgs cam, BlendArgs bl, int n_tiles, float* __restrict__ image, float* __restrict__ final_t,
    uint32_t* __restrict__ l_iter, uint32_t* __restrict__ l_blend, ulonglong4* __restrict__ wave_sums,
    unsigned long long* __restrict__ counters) {
  __shared__ TileLds lds;
  render_tile<kCap>(lds, rec, exact, vals, ranges, order, n_pairs, n_gauss, cam, bl, n_tiles, (int)blockIdx.x, image,
                    final_t, l_iter, l_blend, wave_sums, counters);
}

// The blends of several frames in one launch: workgroup b renders item
// b - block_base of the job whose [block_base, block_base + n_tiles) holds b
// (jobs in ascending block_base). Every frame's tiles are computed exactly as
// render_kernel computes them alone.
template <bool kCap>
__global__ void __launch_bounds__(256, 4) render_batch_kernel(const BlendJob* __restrict__ jobs, int n_jobs) {
  __shared__ TileLds lds;
  const int b = (int)blockIdx.x;
  int j = 0;
  for (int k = 1; k < n_jobs; ++k)
    if (b >= jobs[k].block_base) j = k;
  const BlendJob& job = jobs[j];
  const int blk = b - job.block_base;
  if (blk < 0 || blk >= job.n_tiles) return;  // (cannot happen for a consistent table)
  render_tile<kCap>(lds, job.rec, job.exact, job.vals, job.ranges, job.order, job.n_pairs, job.n_gauss, job.cam,
                    job.blend, job.n_tiles, blk, job.image, job.final_t, job.l_iter, job.l_blend, job.wave_sums,
                    job.counters);
}

// Mean and population standard deviation of a per-pixel load over n pixels
// (Eq. 13) from its exact integer sums s1 = sum l, s2 = sum l^2: the variance
// numerator n s2 - s1^2 is formed exactly in 128-bit integers (it is >= 0),
// then divided by n^2 in FP64.
__device__ void load_moments(unsigned long long s1, unsigned long long s2, unsigned long long n, double* out) {
  const unsigned long long a_lo = n * s2, a_hi = __umul64hi(n, s2);
  const unsigned long long b_lo = s1 * s1, b_hi = __umul64hi(s1, s1);
  const unsigned long long d_lo = a_lo - b_lo;
  const unsigned long long d_hi = a_hi - b_hi - (a_lo < b_lo ? 1ull : 0ull);
  const double num = (double)d_hi * 18446744073709551616.0 + (double)d_lo;
  const double nn = (double)n;
  out[0] = (double)s1 / nn;
  out[1] = sqrt(num / (nn * nn));
}

// Adds the per-wave partials into the four load accumulators (zeroed at the
// start of the frame; integer sums, so the result does not depend on the
// order). The last workgroup to finish copies the sums to the caller and
// turns them into the load statistics of Eq. 13.
__global__ void __launch_bounds__(256) load_sums_kernel(const ulonglong4* __restrict__ wave_sums, int n,
                                                        unsigned long long* __restrict__ acc,
                                                        unsigned long long n_pixels,
                                                        unsigned long long* __restrict__ sums_out,
                                                        double* __restrict__ stats_out) {
  __shared__ unsigned long long part[4][4];
  __shared__ bool last;
  unsigned long long a = 0, b = 0, c = 0, d = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const ulonglong4 v = wave_sums[i];
    a += v.x;
    b += v.y;
    c += v.z;
    d += v.w;
  }
  a = wave_sum_u64(a);
  b = wave_sum_u64(b);
  c = wave_sum_u64(c);
  d = wave_sum_u64(d);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    part[wid][0] = a;
    part[wid][1] = b;
    part[wid][2] = c;
    part[wid][3] = d;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    const unsigned long long t = part[0][threadIdx.x] + part[1][threadIdx.x] + part[2][threadIdx.x] +
                                 part[3][threadIdx.x];
    if (t) atomicAdd(&acc[threadIdx.x], t);
  }
  // every sum of this workgroup is in acc before its ticket is taken
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) last = atomicAdd(&acc[4], 1ull) == (unsigned long long)gridDim.x - 1;
  __syncthreads();
  if (last && threadIdx.x == 0) {
    __threadfence();
    unsigned long long v[4];
    for (int k = 0; k < 4; ++k) v[k] = __hip_atomic_load(&acc[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (sums_out)
      for (int k = 0; k < 4; ++k) sums_out[k] = v[k];
    if (stats_out) {
      load_moments(v[0], v[1], n_pixels, stats_out);
      load_moments(v[2], v[3], n_pixels, stats_out + 2);
    }
  }
}

// ---------------------------------------------------------------------------
// Backward of the blend (Eqs. 2-3)
// ---------------------------------------------------------------------------
// For C = sum_k c_k alpha_k T_k + T_N bg over the entries a pixel blended,
// with L depending on C through g = dL/dC:
//   dL/dc_k     = g alpha_k T_k
//   dL/dalpha_k = g . c_k T_k - (g . S_k + T_N g . bg) / (1 - alpha_k),
//                 S_k = sum_{j > k} c_j alpha_j T_j,
// and where alpha_k = sigma_k G_k is below its clamp, G_k = exp(power_k),
// power = -1/2 (A dx^2 + 2 B dx dy + C dy^2), dx = x - i, dy = y - j:
//   dL/dsigma = dL/dalpha G,  dL/dpower = dL/dalpha alpha,
//   dL/dx = -dL/dpower (A dx + B dy),  dL/dy = -dL/dpower (B dx + C dy),
//   dL/dA = -dL/dpower dx^2 / 2,  dL/dB = -dL/dpower dx dy,  dL/dC = -dL/dpower dy^2 / 2.
// Each pixel walks its tile list back to front from the last entry it
// examined (l_iter of the forward), recovering T_k = T_{k+1} / (1 - alpha_k)
// from the final transmittance, so no per-entry state is stored. Which entries
// it blended is decided exactly as in the forward: the same staged values, the
// FP32 exponent outside the Gaussian's error band and FP64 inside it. Per
// batch of 64 list entries a wave stages the entries that meet its quadrant
// and steps through them from the last to the first, all lanes on the same
// entry; a step where some pixel blends sums the nine contributions over
// each 16-lane row with cross-lane (DPP) adds, and the first lane of each row
// adds the row sums to the entry's LDS accumulators. After the batch one
// global add per entry and component goes to the Gaussian's screen-space
// gradients.
// Sum over each 16-lane row of the wave (every lane of a row receives it).
__device__ __forceinline__ float row_sum_dpp(float v) {
  v += __builtin_amdgcn_update_dpp(0.f, v, 0xb1, 0xf, 0xf, false);   // quad_perm 1,0,3,2
  v += __builtin_amdgcn_update_dpp(0.f, v, 0x4e, 0xf, 0xf, false);   // quad_perm 2,3,0,1
  v += __builtin_amdgcn_update_dpp(0.f, v, 0x141, 0xf, 0xf, false);  // row_half_mirror: 8 lanes
  v += __builtin_amdgcn_update_dpp(0.f, v, 0x140, 0xf, 0xf, false);  // row_mirror: the 16-lane row
  return v;
}

__global__ void __launch_bounds__(256) render_backward_kernel(
    const RenderRecord* __restrict__ rec, const ExactRecord* __restrict__ exact, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ ranges, uint32_t n_pairs, uint32_t n_gauss, CamArgs cam, BlendArgs bl,
    const float* __restrict__ final_t, const uint32_t* __restrict__ l_iter, const float* __restrict__ dl_dimage,
    const float* __restrict__ dl_dload, float* __restrict__ grad2d) {
  __shared__ Staged stage[4][64];
  __shared__ float4 stage_col[4][64];  // r, g, b, opacity
  __shared__ float4 stage_con[4][64];  // conic A, B, C, Gaussian id (bits)
  __shared__ float acc[4][9][64];
  const int tile = blockIdx.x;
  const int W = cam.width, H = cam.height;
  const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int qx0 = tx * kTile + (wid & 1) * kQuad;
  const int qy0 = ty * kTile + (wid >> 1) * kQuad;
  if (qx0 >= W || qy0 >= H) return;  // wave-uniform
  const uint32_t e = min(ranges[2 * tile + 1], n_pairs);
  const uint32_t s = min(ranges[2 * tile], e);
  if (e <= s) return;
  float* my_acc = &acc[wid][0][0];
#pragma unroll
  for (int c = 0; c < 9; ++c) my_acc[c * 64 + lane] = 0.f;
  const int sb = lane >> 4;
  const int lx = (sb & 1) * kSub + (lane & 3), ly = (sb >> 1) * kSub + ((lane >> 2) & 3);
  const int pi = qx0 + lx, pj = qy0 + ly;
  const bool inside = pi < W && pj < H;
  const float fx = (float)lx, fy = (float)ly;
  const int64_t plane = (int64_t)W * H;
  const int64_t pix = inside ? (int64_t)pj * W + pi : 0;
  const uint32_t n_ex = inside ? min(l_iter[pix], e - s) : 0u;
  float T = inside ? final_t[pix] : 1.f;
  const float g0 = inside ? dl_dimage[pix] : 0.f;
  const float g1 = inside ? dl_dimage[plane + pix] : 0.f;
  const float g2 = inside ? dl_dimage[2 * plane + pix] : 0.f;
  // dL/d(load of this pixel): each blended entry counts 1, read as d load / d alpha = 1
  const float g_load = (inside && dl_dload) ? dl_dload[pix] : 0.f;
  const float bg_t = T * (g0 * bl.bg[0] + g1 * bl.bg[1] + g2 * bl.bg[2]);
  float S0 = 0.f, S1 = 0.f, S2 = 0.f;
  uint32_t n_max = n_ex;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) n_max = max(n_max, (uint32_t)__shfl_xor((int)n_max, off, 64));
  const uint2 kNoBox = no_box();
  for (int b = ((int)n_max - 1) >> 6; b >= 0; --b) {
    const uint32_t base = s + 64u * (uint32_t)b;
    const uint32_t k_lane = base + (uint32_t)lane;
    const bool valid = k_lane < s + n_max;
    const uint32_t g = valid ? min(vals[k_lane], n_gauss - 1) : 0u;
    const SubMasks hm = sub_masks(valid ? load_box(rec, g) : kNoBox, qx0, qy0);
    const uint64_t any = hm.m[0] | hm.m[1] | hm.m[2] | hm.m[3];
    if ((any >> lane) & 1ull) {  // the forward's staging, bit for bit
      const RenderRecord& r = rec[g];
      Staged st;
      st.a = make_float4((float)(r.x - (double)qx0), (float)(r.y - (double)qy0), r.rc, r.rs);
      st.b = make_float4(r.a1, r.a2, r.ql, bl.exact ? r.dq + bl.band_floor : 0.f);
      stage[wid][lane] = st;
      const ExactRecord& ex = exact[g];
      stage_col[wid][lane] = make_float4(r.r, r.g, r.b, (float)ex.opacity);
      stage_con[wid][lane] = make_float4((float)ex.ca, (float)ex.cb, (float)ex.cc, __uint_as_float(g));
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // the entries of this batch this lane examined and whose box meets its sub-block
    uint64_t my_mask = sb == 0 ? hm.m[0] : sb == 1 ? hm.m[1] : sb == 2 ? hm.m[2] : hm.m[3];
    const uint32_t lim = n_ex > base - s ? n_ex - (base - s) : 0u;
    if (!inside || lim == 0) my_mask = 0ull;
    if (lim < 64) my_mask &= (1ull << lim) - 1ull;
    uint64_t rem = any;
    while (rem) {
      const int k = 63 - (int)__builtin_clzll(rem);  // back to front, the whole wave on entry k
      rem &= ~(1ull << k);
      const bool act = (my_mask >> k) & 1ull;
      const float4 A = stage[wid][k].a, B = stage[wid][k].b;
      const float q = quad_form(A, B, fx, fy);
      bool blend = act && q >= bl.q_low;
      const bool near_low = act && fabsf(q - bl.q_low) < B.w;
      if (__ballot(near_low) != 0ull) {
        if (near_low)
          blend = alpha_fp64_at(rec, exact, __float_as_uint(stage_con[wid][k].w), pi, pj, bl.alpha_max_d) >=
                  bl.alpha_low_d;
      }
      if (__ballot(blend) == 0ull) continue;
      float d[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      if (blend) {
        const float4 col = stage_col[wid][k], con = stage_con[wid][k];
        const float dx = A.x - fx, dy = A.y - fy;
        const float power = -0.5f * (con.x * dx * dx + 2.f * con.y * dx * dy + con.z * dy * dy);
        const float G = __expf(power);
        const float a_raw = col.w * G;
        const float a = fminf(a_raw, bl.alpha_max);
        const float inv = __builtin_amdgcn_rcpf(1.f - a);
        const float Tk = T * inv;
        const float dl_da =
            (g0 * col.x + g1 * col.y + g2 * col.z) * Tk - (g0 * S0 + g1 * S1 + g2 * S2 + bg_t) * inv + g_load;
        const float w = a * Tk;
        d[6] = g0 * w;
        d[7] = g1 * w;
        d[8] = g2 * w;
        S0 = fmaf(col.x, w, S0);
        S1 = fmaf(col.y, w, S1);
        S2 = fmaf(col.z, w, S2);
        T = Tk;
        if (a_raw < bl.alpha_max) {
          const float dp = dl_da * a;
          d[0] = -dp * (con.x * dx + con.y * dy);
          d[1] = -dp * (con.y * dx + con.z * dy);
          d[2] = -0.5f * dp * dx * dx;
          d[3] = -dp * dx * dy;
          d[4] = -0.5f * dp * dy * dy;
          d[5] = dl_da * G;
        }
      }
#pragma unroll
      for (int c = 0; c < 9; ++c) d[c] = row_sum_dpp(d[c]);
      if ((lane & 15) == 0) {
#pragma unroll
        for (int c = 0; c < 9; ++c)
          if (d[c] != 0.f) atomicAdd(&my_acc[c * 64 + k], d[c]);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // lane k adds entry k's sums to its Gaussian and clears them
    if ((any >> lane) & 1ull) {
      const uint32_t gk = __float_as_uint(stage_con[wid][lane].w);
#pragma unroll
      for (int c = 0; c < 9; ++c) {
        const float v = my_acc[c * 64 + lane];
        if (v != 0.f) {
          atomicAdd(&grad2d[(int64_t)gk * kGrad2d + c], v);
          my_acc[c * 64 + lane] = 0.f;
        }
      }
    }
    __builtin_amdgcn_wave_barrier();  // every read of this batch's slots before the next writes
  }
}

}  // namespace

// Superblocks of a tiles_x x tiles_y grid of n tiles: at most
// (tx/16 + 1)(ty/16 + 1) = n/256 + (tx + ty)/16 + 1 <= n/256 + n/16 + 2.
static int64_t order_blocks_bound(int64_t n_tiles) { return n_tiles / 256 + n_tiles / 16 + 2; }

int64_t tile_order_scratch(int n_tiles) { return (int64_t)kOrderBuckets * order_blocks_bound(n_tiles); }

// counts: tile_order_scratch(tiles_x * tiles_y) words
hipError_t launch_tile_order(const uint32_t* ranges, int64_t n_pairs, int tiles_x, int tiles_y, uint32_t* order,
                             uint32_t* counts, hipStream_t stream) {
  if (tiles_x <= 0 || tiles_y <= 0) return hipSuccess;
  const int64_t nb = (int64_t)((tiles_x + kOrderSuper - 1) / kOrderSuper) * ((tiles_y + kOrderSuper - 1) / kOrderSuper);
  if (nb > order_blocks_bound((int64_t)tiles_x * tiles_y)) return hipErrorInvalidValue;
  order_count_kernel<<<(unsigned)nb, kOrderBlock, 0, stream>>>(ranges, tiles_x, tiles_y, (uint32_t)n_pairs, counts);
  order_scatter_kernel<<<(unsigned)nb, kOrderBlock, 0, stream>>>(ranges, tiles_x, tiles_y, (uint32_t)n_pairs, counts,
                                                                  order);
  return hipGetLastError();
}

hipError_t launch_render(const RenderRecord* rec, const ExactRecord* exact, const uint32_t* vals,
                         const uint32_t* ranges, const uint32_t* order, int64_t n_pairs, int64_t n_gauss,
                         const CamArgs& cam, const BlendArgs& blend, const adr_frame* out, bool want_load,
                         adr_workspace* ws, hipStream_t stream) {
  const int n_tiles = cam.tiles_x * cam.tiles_y;
  if (n_tiles > ws->tile_capacity) return hipErrorInvalidValue;
  ulonglong4* ws4 = want_load ? (ulonglong4*)ws->wave_sums : nullptr;
  auto* kernel = blend.lb_cap > 0 ? render_kernel<true> : render_kernel<false>;
  kernel<<<dim3((unsigned)n_tiles), 256, 0, stream>>>(
      rec, exact, vals, ranges, order, (uint32_t)n_pairs, (uint32_t)(n_gauss > 0 ? n_gauss : 1), cam, blend,
      n_tiles, out->image, out->final_t, out->l_iter, out->l_blend, ws4, ws->dev_counters);
  return hipGetLastError();
}

hipError_t launch_render_batch(const BlendJob* jobs_dev, int n_jobs, int64_t total_blocks, bool any_cap,
                               hipStream_t stream) {
  if (n_jobs <= 0 || total_blocks <= 0) return hipSuccess;
  if (total_blocks > 0x7fffffff) return hipErrorInvalidValue;
  auto* kernel = any_cap ? render_batch_kernel<true> : render_batch_kernel<false>;
  kernel<<<dim3((unsigned)total_blocks), 256, 0, stream>>>(jobs_dev, n_jobs);
  return hipGetLastError();
}

BlendJob make_blend_job(const adr_workspace* ws, const RenderRecord* rec, const ExactRecord* exact,
                        const uint32_t* vals, const CamArgs& cam, const BlendArgs& blend, int64_t n_pairs,
                        int64_t n_gauss, const adr_frame* out, bool want_load) {
  BlendJob j{};
  j.rec = rec;
  j.exact = exact;
  j.vals = vals;
  j.ranges = ws->ranges;
  j.order = ws->tile_order;
  j.image = out->image;
  j.final_t = out->final_t;
  j.l_iter = out->l_iter;
  j.l_blend = out->l_blend;
  j.wave_sums = want_load ? (ulonglong4*)ws->wave_sums : nullptr;
  j.counters = ws->dev_counters;
  j.n_pairs = (uint32_t)n_pairs;
  j.n_gauss = (uint32_t)(n_gauss > 0 ? n_gauss : 1);
  j.n_tiles = cam.tiles_x * cam.tiles_y;
  j.block_base = 0;
  j.cam = cam;
  j.blend = blend;
  // a cap of 0 is "off": the capped kernel then compares against a count no pixel reaches
  if (j.blend.lb_cap <= 0) j.blend.lb_cap = 0;
  return j;
}

hipError_t launch_load_sums(adr_workspace* ws, int n_tiles, int64_t n_pixels, uint64_t* load_sums,
                            double* load_stats, hipStream_t stream) {
  if (!load_sums && !load_stats) return hipSuccess;
  if (n_tiles > ws->tile_capacity || n_pixels <= 0) return hipErrorInvalidValue;
  const int n = 4 * n_tiles;
  int blocks = (n + 1023) / 1024;
  if (blocks > 64) blocks = 64;
  if (blocks < 1) blocks = 1;
  load_sums_kernel<<<dim3((unsigned)blocks), 256, 0, stream>>>((const ulonglong4*)ws->wave_sums, n, ws->load_acc,
                                                               (unsigned long long)n_pixels,
                                                               (unsigned long long*)load_sums, load_stats);
  return hipGetLastError();
}

// grad2d: kGrad2d floats per Gaussian, zeroed by the caller
hipError_t launch_render_backward(const RenderRecord* rec, const ExactRecord* exact, const uint32_t* vals,
                                  const uint32_t* ranges, int64_t n_pairs, int64_t n_gauss, const CamArgs& cam,
                                  const BlendArgs& blend, const float* final_t, const uint32_t* l_iter,
                                  const float* dl_dimage, const float* dl_dload, float* grad2d,
                                  hipStream_t stream) {
  const int n_tiles = cam.tiles_x * cam.tiles_y;
  if (n_tiles <= 0 || n_pairs <= 0 || n_gauss <= 0) return hipSuccess;
  render_backward_kernel<<<dim3((unsigned)n_tiles), 256, 0, stream>>>(rec, exact, vals, ranges, (uint32_t)n_pairs,
                                                                      (uint32_t)n_gauss, cam, blend, final_t, l_iter,
                                                                      dl_dimage, dl_dload, grad2d);
  return hipGetLastError();
}

}  // namespace adr

