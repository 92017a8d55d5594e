// Render (Sec. 3.2, stage 6): pixel-parallel, Gaussian-serial front-to-back
// blending (Eqs. 2-3), per-pixel load counters (Eq. 12) and the
// load-balancing cap.
//
// Layout: one 256-lane workgroup per 16 x 16 tile; each wave64 owns an 8 x 8
// quadrant and walks the tile's depth-sorted list on its own, so a quadrant
// whose pixels are all saturated stops without waiting for the others.
// Batches of 64 list entries are loaded one per lane (ids, then 64-byte
// records); a ballot marks the entries whose alpha_low box meets the
// quadrant and only those are evaluated, each broadcast to the wave with
// readlane. Entries outside the box are exactly the ones whose alpha is below
// alpha_low for every pixel of the quadrant, so skipping them changes nothing.
//
// Precision: the record centre is made quadrant-relative in FP64 before the
// FP32 evaluation. The skip decision alpha < alpha_low and the stop decision
// T < t_min are re-taken in FP64 when the FP32 values fall inside a narrow
// band around the threshold, so the blended sequence matches an FP64
// evaluation of the same definition.
#include "adr_internal.h"

namespace adr {

namespace {

__device__ __forceinline__ float bcast_f(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ __forceinline__ uint32_t bcast_u(uint32_t v, int lane) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}
__device__ __forceinline__ double bcast_d(double v, int lane) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const uint32_t lo = bcast_u((uint32_t)u, lane), hi = bcast_u((uint32_t)(u >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

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

// FP64 splatting opacity of Gaussian g at pixel (pi, pj) (Eq. 2), clamped.
__device__ __forceinline__ double alpha_fp64(const ExactRecord& e, double x, double y, int pi, int pj,
                                             double alpha_max) {
  const double dx = x - (double)pi, dy = y - (double)pj;
  const double power = -0.5 * (e.ca * dx * dx + 2.0 * e.cb * dx * dy + e.cc * dy * dy);
  return fmin(alpha_max, e.opacity * exp(power));
}

// Transmittance of pixel (pi, pj) after list entries [s, k_end], in FP64.
__device__ double replay_fp64(const RenderRecord* __restrict__ rec, const ExactRecord* __restrict__ exact,
                              const uint32_t* __restrict__ vals, uint32_t n_gauss, uint32_t s, uint32_t k_end,
                              int pi, int pj, const BlendArgs& bl) {
  double t = 1.0;
  for (uint32_t k = s; k <= k_end; ++k) {
    const uint32_t g = min(vals[k], n_gauss - 1);
    const uint32_t bx = rec[g].box_x, by = rec[g].box_y;
    if ((int)(bx & 0xffffu) > pi || (int)(bx >> 16) < pi || (int)(by & 0xffffu) > pj || (int)(by >> 16) < pj)
      continue;  // outside the alpha_low ellipse: alpha < alpha_low
    const double a = alpha_fp64(exact[g], rec[g].x, rec[g].y, pi, pj, bl.alpha_max_d);
    if (a < bl.alpha_low_d) continue;
    t *= 1.0 - a;
  }
  return t;
}

__global__ void __launch_bounds__(256) render_kernel(
    const RenderRecord* __restrict__ rec, const ExactRecord* __restrict__ exact, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ ranges, uint32_t n_pairs, uint32_t n_gauss, CamArgs cam, BlendArgs bl,
    int n_tiles, int per_xcd,
    float* __restrict__ image, float* __restrict__ final_t, uint32_t* __restrict__ l_iter,
    uint32_t* __restrict__ l_blend, unsigned long long* __restrict__ load_sums,
    unsigned long long* __restrict__ counters) {
  // XCD-aware tile order: workgroups are dealt round-robin to the 8 XCDs, so
  // give each XCD a contiguous band of tiles (neighbouring tiles share
  // Gaussians, which then stay in that XCD's L2).
  const int bid = blockIdx.x;
  const int tile = (bid & 7) * per_xcd + (bid >> 3);
  if (tile >= n_tiles) return;
  const int W = cam.width, H = cam.height;
  const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int qx0 = tx * kTile + (wid & 1) * kQuad;
  const int qy0 = ty * kTile + (wid >> 1) * kQuad;
  if (qx0 >= W || qy0 >= H) return;  // quadrant entirely outside the image (wave-uniform)
  const int qx1 = min(qx0 + kQuad - 1, W - 1), qy1 = min(qy0 + kQuad - 1, H - 1);
  const int lx = lane & 7, ly = lane >> 3;
  const int pi = qx0 + lx, pj = qy0 + ly;
  const bool inside = pi < W && pj < H;
  const float fx = (float)lx, fy = (float)ly;

  // ranges come from this frame's sorted keys; the clamps only make a
  // corrupted table unable to send a load outside the buffers
  const uint32_t e = min(ranges[2 * tile + 1], n_pairs);
  const uint32_t s = min(ranges[2 * tile], e);
  float T = 1.f, cr = 0.f, cg = 0.f, cb = 0.f;
  uint32_t nb = 0;
  int64_t stop_k = -1;
  bool done = !inside;
  uint32_t n_band = 0, n_replay = 0;

  for (uint32_t base = s; base < e; base += 64) {
    const uint32_t k = base + lane;
    const bool valid = k < e;
    uint32_t g = 0;
    RenderRecord r;
    bool hit = false;
    if (valid) {
      g = min(vals[k], n_gauss - 1);
      r = rec[g];
      hit = (int)(r.box_x & 0xffffu) <= qx1 && (int)(r.box_x >> 16) >= qx0 && (int)(r.box_y & 0xffffu) <= qy1 &&
            (int)(r.box_y >> 16) >= qy0;
    } else {
      r = RenderRecord{};
    }
    // centre relative to the quadrant origin, computed in FP64
    const float xr = valid ? (float)(r.x - (double)qx0) : 0.f;
    const float yr = valid ? (float)(r.y - (double)qy0) : 0.f;
    uint64_t mask = __ballot(hit);
    while (mask) {
      const int j = __builtin_ctzll(mask);
      mask &= mask - 1;
      const float gx = bcast_f(xr, j), gy = bcast_f(yr, j);
      const float qa = bcast_f(r.qa, j), qb = bcast_f(r.qb, j), qc = bcast_f(r.qc, j), ql = bcast_f(r.ql, j);
      const float c0 = bcast_f(r.r, j), c1 = bcast_f(r.g, j), c2 = bcast_f(r.b, j);
      if (!done) {
        const float dx = gx - fx, dy = gy - fy;
        const float q = fmaf(qa * dx, dx, fmaf(qb * dx, dy, fmaf(qc * dy, dy, ql)));
        bool blend = q >= bl.q_low;
        float a = 0.f;
        if (bl.exact && fabsf(q - bl.q_low) < bl.q_band) {
          // near alpha_low: decide in FP64
          const uint32_t gj = bcast_u(g, j);
          const double xd = bcast_d(r.x, j), yd = bcast_d(r.y, j);
          const double ad = alpha_fp64(exact[gj], xd, yd, pi, pj, bl.alpha_max_d);
          blend = ad >= bl.alpha_low_d;
          a = (float)ad;
          ++n_band;
        } else if (blend) {
          a = fminf(bl.alpha_max, __builtin_amdgcn_exp2f(q));
        }
        if (blend) {
          const float w = a * T;
          cr = fmaf(c0, w, cr);
          cg = fmaf(c1, w, cg);
          cb = fmaf(c2, w, cb);
          T = T * (1.f - a);
          ++nb;
          bool stop = T < bl.t_min;
          if (bl.exact && T >= bl.t_band_lo && T <= bl.t_band_hi) {
            // near t_min: re-run this pixel's list up to here in FP64
            const double td = replay_fp64(rec, exact, vals, n_gauss, s, base + (uint32_t)j, pi, pj, bl);
            stop = td < bl.t_min_d;
            T = (float)td;
            ++n_replay;
          }
          if (!stop && bl.lb_cap > 0 && nb == (uint32_t)bl.lb_cap) stop = true;
          if (stop) {
            done = true;
            stop_k = (int64_t)base + j;
          }
        }
      }
      if (__ballot(!done) == 0) goto finished;
    }
  }
finished:
  uint32_t ni = 0;
  if (inside) {
    ni = stop_k >= 0 ? (uint32_t)(stop_k - (int64_t)s + 1) : e - s;
    const int64_t pix = (int64_t)pj * W + pi;
    const int64_t plane = (int64_t)W * H;
    image[pix] = cr + T * bl.bg[0];
    image[plane + pix] = cg + T * bl.bg[1];
    image[2 * plane + pix] = cb + T * bl.bg[2];
    if (final_t) final_t[pix] = T;
    if (l_iter) l_iter[pix] = ni;
    if (l_blend) l_blend[pix] = nb;
  }
  if (load_sums) {
    const unsigned long long b1 = wave_sum_u64(nb), b2 = wave_sum_u64((unsigned long long)nb * nb);
    const unsigned long long i1 = wave_sum_u64(ni), i2 = wave_sum_u64((unsigned long long)ni * ni);
    if (lane == 0) {
      if (b1) atomicAdd(&load_sums[0], b1);
      if (b2) atomicAdd(&load_sums[1], b2);
      if (i1) atomicAdd(&load_sums[2], i1);
      if (i2) atomicAdd(&load_sums[3], i2);
    }
  }
  if (counters) {
    const unsigned long long nbd = wave_sum_u64(n_band), nrp = wave_sum_u64(n_replay);
    if (lane == 0) {
      if (nbd) atomicAdd(&counters[2], nbd);
      if (nrp) atomicAdd(&counters[3], nrp);
    }
  }
}

}  // namespace

hipError_t launch_render(const RenderRecord* rec, const ExactRecord* exact, const uint32_t* vals,
                         const uint32_t* ranges, int64_t n_pairs, int64_t n_gauss, const CamArgs& cam,
                         const BlendArgs& blend, adr_frame* out, unsigned long long* counters, hipStream_t stream) {
  const int n_tiles = cam.tiles_x * cam.tiles_y;
  const int per_xcd = (n_tiles + 7) / 8;
  render_kernel<<<dim3((unsigned)(8 * per_xcd)), 256, 0, stream>>>(
      rec, exact, vals, ranges, (uint32_t)n_pairs, (uint32_t)(n_gauss > 0 ? n_gauss : 1), cam, blend, n_tiles,
      per_xcd, out->image, out->final_t, out->l_iter, out->l_blend,
      (unsigned long long*)out->load_sums, counters);
  return hipGetLastError();
}

}  // namespace adr
