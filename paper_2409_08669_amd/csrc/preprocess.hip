// Preprocess (Sec. 3.2, stage 1) with the paper's early culling of
// Gaussian-tile pairs (Sec. 4.2 adaptive radius, Eqs. 5-8; Sec. 4.3 AABB,
// Eqs. 9-11). One lane per Gaussian.
//
// Every scalar that decides an integer (visibility, the pixel and tile
// rectangles, tiles_touched, the depth key) is computed in FP64: the stage
// is HBM-bound and gfx950 runs FP64 FMA at the non-packed FP32 lane rate,
// so this costs little and keeps the integer outputs bit-exact against an
// FP64 reference. The render record is rounded to FP32 at the end.
#include "adr_internal.h"

namespace adr {

// Normalisation constants of the real SH basis, filled on the host from
// N_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!), times sqrt(2) for m != 0.
struct ShConsts {
  float k[16];
};

// Colour from K = (d+1)^2 SH coefficients. All 3K loads are issued before
// any arithmetic (one memory round trip per Gaussian).
template <int K, class Src>
__device__ __forceinline__ void sh_colour_k(const Src& src, int64_t g, const ShConsts& kc, float x, float y,
                                            float z, float& r, float& gr, float& b) {
  float coef[3 * K];
#pragma unroll
  for (int i = 0; i < 3 * K; ++i) coef[i] = src.coef(i, g);
  // Polynomial parts P_l^|m|(cos th) cos(m ph) / sin(|m| ph) on the unit
  // sphere, Condon-Shortley phase included; index l*l + l + m.
  float basis[16];
  basis[0] = 1.f;
  if (K > 1) {
    basis[1] = -y;
    basis[2] = z;
    basis[3] = -x;
  }
  if (K > 4) {
    const float xx = x * x, yy = y * y, zz = z * z;
    basis[4] = 6.f * x * y;
    basis[5] = -3.f * z * y;
    basis[6] = 0.5f * (3.f * zz - 1.f);
    basis[7] = -3.f * z * x;
    basis[8] = 3.f * (xx - yy);
    if (K > 9) {
      const float t = -1.5f * (5.f * zz - 1.f);
      basis[9] = -15.f * (3.f * xx * y - yy * y);
      basis[10] = 30.f * x * y * z;
      basis[11] = t * y;
      basis[12] = 0.5f * (5.f * zz * z - 3.f * z);
      basis[13] = t * x;
      basis[14] = 15.f * z * (xx - yy);
      basis[15] = -15.f * (xx * x - 3.f * x * yy);
    }
  }
  float acc[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const float w = kc.k[k] * basis[k];
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] = fmaf(w, coef[3 * k + c], acc[c]);
  }
  r = fmaxf(acc[0] + 0.5f, 0.f);
  gr = fmaxf(acc[1] + 0.5f, 0.f);
  b = fmaxf(acc[2] + 0.5f, 0.f);
}

template <class Src>
__device__ __forceinline__ void sh_colour(const Src& src, int64_t g, int n_coeff, const ShConsts& kc, float x,
                                          float y, float z, float& r, float& gr, float& b) {
  switch (n_coeff) {
    case 1: sh_colour_k<1>(src, g, kc, x, y, z, r, gr, b); break;
    case 4: sh_colour_k<4>(src, g, kc, x, y, z, r, gr, b); break;
    case 9: sh_colour_k<9>(src, g, kc, x, y, z, r, gr, b); break;
    default: sh_colour_k<16>(src, g, kc, x, y, z, r, gr, b); break;
  }
}

__device__ __forceinline__ uint32_t pack16(int lo, int hi) { return (uint32_t)lo | ((uint32_t)hi << 16); }

// Clipped integer range of pixel centres in [c - r, c + r]; lo > hi when empty.
__device__ __forceinline__ void pixel_span(double c, double r, int size, int& lo, int& hi) {
  double l = ceil(c - r);
  double h = floor(c + r);
  l = fmax(l, 0.0);
  h = fmin(h, (double)(size - 1));
  if (!(l <= h)) {  // also catches NaN
    lo = 1;
    hi = 0;
    return;
  }
  lo = (int)l;
  hi = (int)h;
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

__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const uint32_t lo = __shfl_xor((uint32_t)v, off, 64), hi = __shfl_xor((uint32_t)(v >> 32), off, 64);
    v = min(v, ((unsigned long long)hi << 32) | lo);
  }
  return v;
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const uint32_t lo = __shfl_xor((uint32_t)v, off, 64), hi = __shfl_xor((uint32_t)(v >> 32), off, 64);
    v = max(v, ((unsigned long long)hi << 32) | lo);
  }
  return v;
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = min(v, (uint32_t)__shfl_xor(v, off, 64));
  return v;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = max(v, (uint32_t)__shfl_xor(v, off, 64));
  return v;
}

// Bound on the rounding error of the blend stage's FP32 exponent, evaluated
// on the principal axes of the conic (no cancellation between its terms):
//   u = fma(c, dx, -(s dy)),  v = fma(s, dx, c dy),
//   q = fma(-(a1 u), u, fma(-(a2 v), v, ql)),  dx = fl(fl(x - qx0) - fx)
// with the quadrant offset fx in [0, 7] and c, s, a1, a2, ql rounded from
// FP64. First-order error analysis (unit roundoff u0 = 2^-24) gives, at a
// pixel where P(d) = a1 u^2 + a2 v^2 = p,
//   |q - q_exact| <= u0 [p (8 sqrt(2) (sqrt(a1) + sqrt(a2)) / sqrt(amin) + 6)
//                        + 20 sqrt(p) (sqrt(a1) + sqrt(a2)) + 3 |ql|],
// using |dx| + |dy| <= sqrt(2 p / amin). The bound returned (times 1.5) is
// its value at p = pm, the largest P where q can reach
// log2(alpha_low) - d0. Beyond pm the same bound must keep FP32 from lifting
// q to the candidate threshold log2(alpha_low) - 2 band; if that cannot be
// shown, or the bound exceeds 2^-8, the Gaussian is marked for FP64
// decisions only (+inf).
__device__ double exponent_error_bound(double a1, double a2, double ql, double q_low) {
  const double u0 = 0x1p-24, d0 = 0.02, inf = __builtin_huge_val();
  if (!(a1 > 0.0) || !(a2 > 0.0)) return inf;
  const double ra = sqrt(a1) + sqrt(a2), amin = fmin(a1, a2);
  const double k1 = 1.5 * u0 * (8.0 * 1.4142135623730951 * ra / sqrt(amin) + 6.0);
  const double k2 = 1.5 * u0 * 20.0 * ra;
  const double k0 = 1.5 * u0 * 3.0 * fabs(ql);
  const double m = ql - q_low;  // q = q_low + m - P
  const double pm = fmax(m + d0, 0.0);
  const double dq = k1 * pm + k2 * sqrt(pm) + k0;
  if (!(dq <= 0x1p-8)) return inf;
  // For P = p >= pm: q_fp32 <= q_low + m - p + k1 p + k2 sqrt(p) + k0 must stay
  // below the threshold: f(p) = (1 - k1) p - k2 sqrt(p) - m > 2 band + k0.
  const double A = 1.0 - k1, B = k2;
  if (!(A > 0.5)) return inf;
  const double sp = sqrt(pm), sstar = B / (2.0 * A);
  const double fmin_ = sp >= sstar ? A * pm - B * sp - m : -m - B * B / (4.0 * A);
  const double band = dq + 0x1p-19;
  if (!(fmin_ > 2.0 * band + k0 + 0x1p-19)) return inf;
  return dq;
}

// Principal axes of P = h [[ca, cb], [cb, cc]], h = log2(e) / 2, by one
// Jacobi rotation: P(d) = a1 u^2 + a2 v^2 with u = c dx - s dy, v = s dx + c dy.
__device__ __forceinline__ void principal_axes(double ca, double cb, double cc, double& c, double& s, double& a1,
                                               double& a2) {
  const double h = 0.5 * 1.4426950408889634074;
  const double pa = h * ca, pb = h * cb, pg = h * cc;
  double t = 0.0;
  if (pb != 0.0) {
    const double tau = (pg - pa) / (2.0 * pb);
    t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
  }
  c = 1.0 / sqrt(1.0 + t * t);
  s = t * c;
  a1 = pa - t * pb;
  a2 = pg + t * pb;
}

template <class Src>
__global__ void __launch_bounds__(256) preprocess_kernel(
    Src src, int64_t n, int n_coeff, ShConsts shc, CamArgs cam, CullArgs cull,
    RenderRecord* __restrict__ rec, ExactRecord* __restrict__ exact, uint2* __restrict__ tile_rect,
    uint32_t* __restrict__ depth_key, uint32_t* __restrict__ depth_id, uint32_t* __restrict__ touched_out,
    ulonglong4* __restrict__ block_parts) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t touched = 0;
  uint32_t dkey = 0xffffffffu;  // Gaussians without pairs sort after every visible one
  if (g < n) {
    // all three geometry loads up front: one round trip
    const float4 ga = src.a(g);
    const float4 gb = src.b(g);
    const float4 gq = src.q(g);
    const double mx = ga.x, my = ga.y, mz = ga.z;
    const double px = cam.r[0] * mx + cam.r[1] * my + cam.r[2] * mz + cam.t[0];
    const double py = cam.r[3] * mx + cam.r[4] * my + cam.r[5] * mz + cam.t[1];
    const double pz = cam.r[6] * mx + cam.r[7] * my + cam.r[8] * mz + cam.t[2];
    if (pz > cam.near_z) {
      // Sigma = R S S^T R^T (Sec. 3.1)
      const double s0 = exp((double)gb.x), s1 = exp((double)gb.y), s2 = exp((double)gb.z);
      double qw = gq.x, qx = gq.y, qy = gq.z, qz = gq.w;
      const double qn = 1.0 / sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
      qw *= qn; qx *= qn; qy *= qn; qz *= qn;
      const double R00 = 1 - 2 * (qy * qy + qz * qz), R01 = 2 * (qx * qy - qw * qz), R02 = 2 * (qx * qz + qw * qy);
      const double R10 = 2 * (qx * qy + qw * qz), R11 = 1 - 2 * (qx * qx + qz * qz), R12 = 2 * (qy * qz - qw * qx);
      const double R20 = 2 * (qx * qz - qw * qy), R21 = 2 * (qy * qz + qw * qx), R22 = 1 - 2 * (qx * qx + qy * qy);
      const double M00 = R00 * s0, M01 = R01 * s1, M02 = R02 * s2;
      const double M10 = R10 * s0, M11 = R11 * s1, M12 = R12 * s2;
      const double M20 = R20 * s0, M21 = R21 * s1, M22 = R22 * s2;
      const double S00 = M00 * M00 + M01 * M01 + M02 * M02;
      const double S01 = M00 * M10 + M01 * M11 + M02 * M12;
      const double S02 = M00 * M20 + M01 * M21 + M02 * M22;
      const double S11 = M10 * M10 + M11 * M11 + M12 * M12;
      const double S12 = M10 * M20 + M11 * M21 + M12 * M22;
      const double S22 = M20 * M20 + M21 * M21 + M22 * M22;
      // EWA: local affine approximation of the projection at the centre,
      // evaluated at a clamped x/z, y/z (Sec. 3.1 cites EWA).
      const double xt = pz * fmin(fmax(px / pz, -cam.lim_x), cam.lim_x);
      const double yt = pz * fmin(fmax(py / pz, -cam.lim_y), cam.lim_y);
      const double j00 = cam.fx / pz, j02 = -cam.fx * xt / (pz * pz);
      const double j11 = cam.fy / pz, j12 = -cam.fy * yt / (pz * pz);
      // T = J W (2 x 3), W the world-to-camera rotation
      const double T00 = j00 * cam.r[0] + j02 * cam.r[6];
      const double T01 = j00 * cam.r[1] + j02 * cam.r[7];
      const double T02 = j00 * cam.r[2] + j02 * cam.r[8];
      const double T10 = j11 * cam.r[3] + j12 * cam.r[6];
      const double T11 = j11 * cam.r[4] + j12 * cam.r[7];
      const double T12 = j11 * cam.r[5] + j12 * cam.r[8];
      // U = T Sigma; Sigma' = U T^T + lowpass I
      const double U00 = T00 * S00 + T01 * S01 + T02 * S02;
      const double U01 = T00 * S01 + T01 * S11 + T02 * S12;
      const double U02 = T00 * S02 + T01 * S12 + T02 * S22;
      const double U10 = T10 * S00 + T11 * S01 + T12 * S02;
      const double U11 = T10 * S01 + T11 * S11 + T12 * S12;
      const double U12 = T10 * S02 + T11 * S12 + T12 * S22;
      const double a = U00 * T00 + U01 * T01 + U02 * T02 + cull.lowpass;
      const double b = U00 * T10 + U01 * T11 + U02 * T12;
      const double c = U10 * T10 + U11 * T11 + U12 * T12 + cull.lowpass;
      const double det = a * c - b * b;
      if (det > 0.0) {
        const double ca = c / det, cb = -b / det, cc = a / det;
        // larger eigenvalue, cancellation-free form of mid + sqrt(mid^2 - det)
        const double mid = 0.5 * (a + c);
        const double hd = 0.5 * (a - c);
        const double lam = mid + sqrt(hd * hd + b * b);
        const double r_o = 3.0 * sqrt(lam);
        const double x = cam.fx * px / pz + cam.cx - 0.5;
        const double y = cam.fy * py / pz + cam.cy - 0.5;
        const double op = 1.0 / (1.0 + exp(-(double)ga.w));
        const bool reaches = op >= cull.alpha_low;
        const double lnr = reaches ? log(op / cull.alpha_low) : 0.0;
        // Radii of the cull mode.
        bool keep = true;
        double rx = r_o, ry = r_o;
        if (cull.mode == ADR_CULL_ADAPTIVE) {
          keep = reaches;
          rx = ry = fmin(sqrt(2.0 * lam * lnr), r_o);
        } else if (cull.mode == ADR_CULL_AABB) {
          keep = reaches;
          rx = fmin(sqrt(2.0 * a * lnr), r_o);
          ry = fmin(sqrt(2.0 * c * lnr), r_o);
        }
        int i_lo = 1, i_hi = 0, j_lo = 1, j_hi = 0;
        if (keep) {
          pixel_span(x, rx, cam.width, i_lo, i_hi);
          pixel_span(y, ry, cam.height, j_lo, j_hi);
        }
        if (i_lo <= i_hi && j_lo <= j_hi) {
          const int tx_lo = i_lo / kTile, tx_hi = i_hi / kTile;
          const int ty_lo = j_lo / kTile, ty_hi = j_hi / kTile;
          touched = (uint32_t)(tx_hi - tx_lo + 1) * (uint32_t)(ty_hi - ty_lo + 1);
          tile_rect[g] = make_uint2(pack16(tx_lo, tx_hi), pack16(ty_lo, ty_hi));
          // view-space depth rounded to fp32; its bits order like the depths (z > 0)
          dkey = __float_as_uint((float)pz);
          // Render-side cull box. The blend stage skips a Gaussian for an 8 x 8
          // quadrant that this box misses. In the culling modes it is the
          // mode's extent without the r_o cap (Eq. 7 square, or Eq. 10 box),
          // which contains the whole alpha_low ellipse, so every skipped pixel
          // has alpha < alpha_low. The 3-sigma baseline has no such extent:
          // its box is the whole image and every list entry is evaluated.
          int bx_lo = 0, bx_hi = cam.width - 1, by_lo = 0, by_hi = cam.height - 1;
          if (cull.mode != ADR_CULL_3SIGMA && cull.quad_cull) {
            const double ex = cull.mode == ADR_CULL_AABB ? sqrt(2.0 * a * lnr) : sqrt(2.0 * lam * lnr);
            const double ey = cull.mode == ADR_CULL_AABB ? sqrt(2.0 * c * lnr) : ex;
            pixel_span(x, ex, cam.width, bx_lo, bx_hi);
            pixel_span(y, ey, cam.height, by_lo, by_hi);
          }
          // SH colour from the viewing direction camera -> centre
          double vx = mx - cam.cam_pos[0], vy = my - cam.cam_pos[1], vz = mz - cam.cam_pos[2];
          const double vn = 1.0 / sqrt(vx * vx + vy * vy + vz * vz);
          float cr, cg, cbl;
          sh_colour(src, g, n_coeff, shc, (float)(vx * vn), (float)(vy * vn), (float)(vz * vn), cr, cg, cbl);
          double rc, rs, a1, a2;
          principal_axes(ca, cb, cc, rc, rs, a1, a2);
          const double ql = log2(op);
          RenderRecord rr;
          rr.x = x;
          rr.y = y;
          rr.rc = (float)rc;
          rr.rs = (float)rs;
          rr.a1 = (float)a1;
          rr.a2 = (float)a2;
          rr.ql = (float)ql;
          rr.r = cr;
          rr.g = cg;
          rr.b = cbl;
          rr.box_x = pack16(bx_lo, bx_hi);
          rr.box_y = pack16(by_lo, by_hi);
          rr.depth_key = dkey;
          // FP32 exponent error bound for the blend stage, rounded up
          const double dq = exponent_error_bound(a1, a2, ql, cull.q_low);
          rr.dq = dq > 1e30 ? __builtin_huge_valf() : (float)dq * (1.0f + 0x1p-20f);
          rec[g] = rr;
          ExactRecord er;
          er.ca = ca;
          er.cb = cb;
          er.cc = cc;
          er.opacity = op;
          exact[g] = er;
        }
      }
    }
    touched_out[g] = touched;
    depth_key[g] = dkey;
    depth_id[g] = (uint32_t)g;
  }
  // Per-workgroup pair total (u64, exact), visible count and range of the
  // visible depth keys, reduced by the notify kernel. (Global atomics from
  // every workgroup onto a few words serialise across the XCDs.)
  __shared__ unsigned long long part[4][4];
  const bool vis = touched > 0;
  const unsigned long long wt = wave_sum_u64(touched);
  const unsigned long long wv = wave_sum_u64(vis ? 1ull : 0ull);
  const uint32_t wmin = wave_min_u32(vis ? dkey : 0xffffffffu);
  const uint32_t wmax = wave_max_u32(vis ? dkey : 0u);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    part[0][wid] = wt;
    part[1][wid] = wv;
    part[2][wid] = wmin;
    part[3][wid] = wmax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    ulonglong4 r;
    r.x = part[0][0] + part[0][1] + part[0][2] + part[0][3];
    r.y = part[1][0] + part[1][1] + part[1][2] + part[1][3];
    r.z = min(min(part[2][0], part[2][1]), min(part[2][2], part[2][3]));
    r.w = max(max(part[3][0], part[3][1]), max(part[3][2], part[3][3]));
    block_parts[blockIdx.x] = r;
  }
}

// Runs after Preprocess on the same stream (the kernel boundary makes every
// workgroup's partials visible): reduces them into the frame counters and
// hands the pair count, the visible count and the visible depth-key range to
// the host through mapped pinned memory, then publishes the frame's number.
// It also clears what the rest of the frame accumulates into (the tile
// ranges, the blend's FP64 counters, the load accumulators) when n_ranges > 0.
__global__ void __launch_bounds__(1024) notify_host_kernel(const ulonglong4* __restrict__ block_parts, int nb,
                                                           unsigned long long* __restrict__ counters,
                                                           unsigned long long* __restrict__ notify,
                                                           unsigned long long seq, uint32_t* __restrict__ ranges,
                                                           int64_t n_ranges,
                                                           unsigned long long* __restrict__ load_acc) {
  __shared__ unsigned long long red[4][16];
  for (int64_t i = threadIdx.x; i < n_ranges; i += blockDim.x) ranges[i] = 0u;
  if (n_ranges > 0) {
    if (threadIdx.x == 0) {
      counters[kCntBand] = 0ull;
      counters[kCntReplay] = 0ull;
      counters[kCntBadIndex] = 0ull;
    }
    if (threadIdx.x < kLoadAccWords) load_acc[threadIdx.x] = 0ull;
  }
  unsigned long long t = 0, v = 0, mn = ~0ull, mx = 0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    const ulonglong4 r = block_parts[i];
    t += r.x;
    v += r.y;
    if (r.y) {
      mn = min(mn, r.z);
      mx = max(mx, r.w);
    }
  }
  t = wave_sum_u64(t);
  v = wave_sum_u64(v);
  mn = wave_min_u64(mn);
  mx = wave_max_u64(mx);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wid] = t;
    red[1][wid] = v;
    red[2][wid] = mn;
    red[3][wid] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) / 64;
    for (int w = 1; w < nw; ++w) {
      t += red[0][w];
      v += red[1][w];
      mn = min(mn, red[2][w]);
      mx = max(mx, red[3][w]);
    }
    counters[kCntPairs] = t;
    counters[kCntVisible] = v;
    counters[kCntDepthMin] = mn;
    counters[kCntDepthMax] = mx;
    __hip_atomic_store(&notify[0], t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&notify[1], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&notify[3], mn, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&notify[4], mx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&notify[2], seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

static ShConsts make_sh_consts() {
  ShConsts s{};
  const double pi = 3.14159265358979323846;
  auto fact = [](int v) {
    double f = 1.0;
    for (int i = 2; i <= v; ++i) f *= i;
    return f;
  };
  for (int l = 0; l <= 3; ++l)
    for (int m = -l; m <= l; ++m) {
      const int am = m < 0 ? -m : m;
      double k = sqrt((2.0 * l + 1.0) / (4.0 * pi) * fact(l - am) / fact(l + am));
      if (m != 0) k *= sqrt(2.0);
      s.k[l * l + l + m] = (float)k;
    }
  return s;
}

// ---------------------------------------------------------------------------
// Backward of Preprocess: from the screen-space gradients of a Gaussian (its
// centre x, y, conic A, B, C, opacity and colour) to its inputs, by the chain
// rule through the forward's steps in reverse, in FP32 (the forward's FP64
// decisions are not retaken here, so FP32 is accurate enough):
//   colour  c = max(0, sum_k K_k Y_k(v) sh_k + 1/2), v = unit(mean - camera):
//           d sh_k = dc K_k Y_k, dv = sum_k dc . sh_k K_k grad Y_k, projected
//           onto the tangent plane and divided by |mean - camera|;
//   opacity sigma = 1/(1 + exp(-logit)): d logit = d sigma sigma (1 - sigma);
//   conic   N = M^-1 (M = Sigma'): dM = -N dN N;
//   Sigma'  = T Sigma T^T + lowpass I, T = J W: dSigma = T^T dM T, dT = 2 dM T Sigma;
//   J       from the camera-space centre p (with the forward's clamp of x/z and
//           y/z: a clamped slope has no derivative in p_x, p_y);
//   x, y    = f p_{x,y}/p_z + c - 1/2;  p = W mean + t;
//   Sigma   = M M^T, M = R(q / |q|) diag(exp(log_scale)).
// Gaussians behind the near plane or with a degenerate Sigma' get zeros.
template <int K, class Src>
__global__ void __launch_bounds__(256) preprocess_backward_kernel(
    Src src, int64_t n, ShConsts shc, CamArgs cam, double lowpass,
    const float* __restrict__ grad2d, float* __restrict__ d_means, float* __restrict__ d_log_scales,
    float* __restrict__ d_quats, float* __restrict__ d_logits, float* __restrict__ d_sh) {
  // The colour part is FP32. The covariance part (Sigma, Sigma', its inverse
  // and the chain back to scales, rotation and centre) is FP64: for an
  // elongated Gaussian the gradient along its long axis is a small
  // difference of large terms of dL/dSigma', which FP32 resolves only to a
  // few percent (axis ratio ~100).
  using real = float;
  using dreal = double;
  const real cfx = (real)cam.fx, cfy = (real)cam.fy, clim_x = (real)cam.lim_x, clim_y = (real)cam.lim_y;
  const real ct[3] = {(real)cam.t[0], (real)cam.t[1], (real)cam.t[2]};
  const real cpos[3] = {(real)cam.cam_pos[0], (real)cam.cam_pos[1], (real)cam.cam_pos[2]};
  const real lp = (real)lowpass;
  // the workgroup's SH gradients, written out together (one row of 3K floats
  // per Gaussian would otherwise make every store touch 64 cache lines)
  __shared__ float sh_out[256 * 3 * K];
  const int64_t g0 = (int64_t)blockIdx.x * blockDim.x;
  const int64_t g = g0 + threadIdx.x;
  const int64_t n_here = min((int64_t)blockDim.x, n - g0);
  float* my_sh = sh_out + threadIdx.x * 3 * K;
#pragma unroll
  for (int i = 0; i < 3 * K; ++i) my_sh[i] = 0.f;
  if (g < n) {
  const float4 ga = src.a(g), gb = src.b(g), gq = src.q(g);
  const real mx = ga.x, my = ga.y, mz = ga.z;
  real W[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) W[i] = (real)cam.r[i];
  const real px = W[0] * mx + W[1] * my + W[2] * mz + ct[0];
  const real py = W[3] * mx + W[4] * my + W[5] * mz + ct[1];
  const real pz = W[6] * mx + W[7] * my + W[8] * mz + ct[2];
  dreal dm[3] = {0, 0, 0}, dls[3] = {0, 0, 0}, dq[4] = {0, 0, 0, 0};
  real dlogit = 0;
  bool live = pz > (real)cam.near_z;
  // forward, as in Preprocess
  const dreal sc[3] = {exp((real)gb.x), exp((real)gb.y), exp((real)gb.z)};
  const dreal qn2 = (dreal)gq.x * gq.x + (dreal)gq.y * gq.y + (dreal)gq.z * gq.z + (dreal)gq.w * gq.w;
  const dreal qn = 1.0 / sqrt(qn2);
  const dreal qw = gq.x * qn, qx = gq.y * qn, qy = gq.z * qn, qz = gq.w * qn;
  const dreal R[3][3] = {{1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy)},
                    {2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx)},
                    {2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)}};
  dreal M[3][3], Sg[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) M[i][j] = R[i][j] * sc[j];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Sg[i][j] = M[i][0] * M[j][0] + M[i][1] * M[j][1] + M[i][2] * M[j][2];
  const real zf = live ? pz : 1.0f;
  const real rx = px / zf, ry = py / zf;
  const dreal z = zf;
  const bool cx_free = rx > -clim_x && rx < clim_x, cy_free = ry > -clim_y && ry < clim_y;
  const dreal xt = z * (dreal)fmin(fmax(rx, -clim_x), clim_x);
  const dreal yt = z * (dreal)fmin(fmax(ry, -clim_y), clim_y);
  const dreal dfx = cam.fx, dfy = cam.fy;
  const dreal j00 = dfx / z, j02 = -dfx * xt / (z * z);
  const dreal j11 = dfy / z, j12 = -dfy * yt / (z * z);
  dreal Wd[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) Wd[i] = cam.r[i];
  dreal T[2][3];
  for (int k = 0; k < 3; ++k) {
    T[0][k] = j00 * Wd[k] + j02 * Wd[6 + k];
    T[1][k] = j11 * Wd[3 + k] + j12 * Wd[6 + k];
  }
  dreal TS[2][3];  // T Sigma
  for (int i = 0; i < 2; ++i)
    for (int k = 0; k < 3; ++k) TS[i][k] = T[i][0] * Sg[0][k] + T[i][1] * Sg[1][k] + T[i][2] * Sg[2][k];
  const dreal a = TS[0][0] * T[0][0] + TS[0][1] * T[0][1] + TS[0][2] * T[0][2] + lowpass;
  const dreal b = TS[0][0] * T[1][0] + TS[0][1] * T[1][1] + TS[0][2] * T[1][2];
  const dreal c = TS[1][0] * T[1][0] + TS[1][1] * T[1][1] + TS[1][2] * T[1][2] + lowpass;
  const dreal det = a * c - b * b;
  live = live && det > 0.0;
  if (live) {
    const float* gr = grad2d + g * kGrad2d;
    const real gx = gr[0], gy = gr[1], gA = gr[2], gB = gr[3], gC = gr[4], gO = gr[5];
    real gcol[3] = {gr[6], gr[7], gr[8]};
    // opacity
    const real op = 1.0f / (1.0f + exp(-(real)ga.w));
    dlogit = gO * op * (1.0f - op);
    // colour (SH basis polynomials of the forward, and their gradients)
    real vx = mx - cpos[0], vy = my - cpos[1], vz = mz - cpos[2];
    const real vlen = sqrt(vx * vx + vy * vy + vz * vz);
    vx /= vlen;
    vy /= vlen;
    vz /= vlen;
    // basis polynomials of the forward (Condon-Shortley phase); only the first K
    const real x = vx, y = vy, zz = vz;
    real Y[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) Y[k] = 0.0f;
    Y[0] = 1.0f;
    const real t = -1.5f * (5 * zz * zz - 1), dt = -15 * zz;
    if (K > 1) {
      Y[1] = -y;
      Y[2] = zz;
      Y[3] = -x;
    }
    if (K > 4) {
      Y[4] = 6 * x * y;
      Y[5] = -3 * zz * y;
      Y[6] = 0.5f * (3 * zz * zz - 1);
      Y[7] = -3 * zz * x;
      Y[8] = 3 * (x * x - y * y);
    }
    if (K > 9) {
      Y[9] = -15 * (3 * x * x * y - y * y * y);
      Y[10] = 30 * x * y * zz;
      Y[11] = t * y;
      Y[12] = 0.5f * (5 * zz * zz * zz - 3 * zz);
      Y[13] = t * x;
      Y[14] = 15 * zz * (x * x - y * y);
      Y[15] = -15 * (x * x * x - 3 * x * y * y);
    }
    float coef[3 * K];  // all SH loads issued together
#pragma unroll
    for (int i = 0; i < 3 * K; ++i) coef[i] = src.coef(i, g);
    real raw[3] = {0.5f, 0.5f, 0.5f};
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) raw[ch] += (real)shc.k[k] * Y[k] * coef[3 * k + ch];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch)
      if (raw[ch] < 0.0f) gcol[ch] = 0.0f;  // clamped channel
    // wk = K_k (dc . sh_k): the weight of basis k's gradient in dL/dv
    real wk[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) wk[k] = 0.0f;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      real acc = 0.0f;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        acc += gcol[ch] * coef[3 * k + ch];
        my_sh[3 * k + ch] = (float)(gcol[ch] * shc.k[k] * Y[k]);
      }
      wk[k] = acc * shc.k[k];
    }
    // dL/dv = sum_k wk grad Y_k (gradients of the polynomials in x, y, z)
    real dv[3] = {0, 0, 0};
    if (K > 1) {
      dv[1] -= wk[1];
      dv[2] += wk[2];
      dv[0] -= wk[3];
    }
    if (K > 4) {
      dv[0] += 6 * y * wk[4];
      dv[1] += 6 * x * wk[4];
      dv[1] -= 3 * zz * wk[5];
      dv[2] -= 3 * y * wk[5];
      dv[2] += 3 * zz * wk[6];
      dv[0] -= 3 * zz * wk[7];
      dv[2] -= 3 * x * wk[7];
      dv[0] += 6 * x * wk[8];
      dv[1] -= 6 * y * wk[8];
    }
    if (K > 9) {
      dv[0] -= 90 * x * y * wk[9];
      dv[1] += (-45 * x * x + 45 * y * y) * wk[9];
      dv[0] += 30 * y * zz * wk[10];
      dv[1] += 30 * x * zz * wk[10];
      dv[2] += 30 * x * y * wk[10];
      dv[1] += t * wk[11];
      dv[2] += dt * y * wk[11];
      dv[2] += 0.5f * (15 * zz * zz - 3) * wk[12];
      dv[0] += t * wk[13];
      dv[2] += dt * x * wk[13];
      dv[0] += 30 * x * zz * wk[14];
      dv[1] -= 30 * y * zz * wk[14];
      dv[2] += 15 * (x * x - y * y) * wk[14];
      dv[0] += (-45 * x * x + 45 * y * y) * wk[15];
      dv[1] += 90 * x * y * wk[15];
    }
    const real vdot = dv[0] * vx + dv[1] * vy + dv[2] * vz;
    dm[0] += (dv[0] - vdot * vx) / vlen;
    dm[1] += (dv[1] - vdot * vy) / vlen;
    dm[2] += (dv[2] - vdot * vz) / vlen;
    // conic N = M^-1: dM = -N dN N, with dN = [[gA, gB/2], [gB/2, gC]]
    const dreal NA = c / det, NB = -b / det, NC = a / det;
    const dreal P00 = NA * gA + NB * 0.5 * gB, P01 = NA * 0.5 * gB + NB * gC;
    const dreal P10 = NB * gA + NC * 0.5 * gB, P11 = NB * 0.5 * gB + NC * gC;
    const dreal da = -(P00 * NA + P01 * NB);
    const dreal db = -2.0 * (P00 * NB + P01 * NC);
    const dreal dc = -(P10 * NB + P11 * NC);
    // Sigma' = T Sigma T^T: G = [[da, db/2], [db/2, dc]]
    const dreal G[2][2] = {{da, 0.5 * db}, {0.5 * db, dc}};
    dreal dS[3][3], dT[2][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        dreal acc = 0.0;
        for (int u = 0; u < 2; ++u)
          for (int v = 0; v < 2; ++v) acc += T[u][i] * G[u][v] * T[v][j];
        dS[i][j] = acc;
      }
    for (int u = 0; u < 2; ++u)
      for (int k = 0; k < 3; ++k) dT[u][k] = 2.0 * (G[u][0] * TS[0][k] + G[u][1] * TS[1][k]);
    // T = J W
    const dreal dj00 = dT[0][0] * Wd[0] + dT[0][1] * Wd[1] + dT[0][2] * Wd[2];
    const dreal dj02 = dT[0][0] * Wd[6] + dT[0][1] * Wd[7] + dT[0][2] * Wd[8];
    const dreal dj11 = dT[1][0] * Wd[3] + dT[1][1] * Wd[4] + dT[1][2] * Wd[5];
    const dreal dj12 = dT[1][0] * Wd[6] + dT[1][1] * Wd[7] + dT[1][2] * Wd[8];
    const dreal dpx_ = px, dpy_ = py;
    dreal dpx = 0.0, dpy = 0.0, dpz = 0.0;
    dpz += -dj00 * dfx / (z * z) - dj11 * dfy / (z * z);
    if (cx_free) {  // j02 = -fx px / z^2
      dpx += -dj02 * dfx / (z * z);
      dpz += dj02 * 2.0 * dfx * dpx_ / (z * z * z);
    } else {  // j02 = -fx L / z, L = +-lim_x
      dpz += dj02 * dfx * (xt / z) / (z * z);
    }
    if (cy_free) {
      dpy += -dj12 * dfy / (z * z);
      dpz += dj12 * 2.0 * dfy * dpy_ / (z * z * z);
    } else {
      dpz += dj12 * dfy * (yt / z) / (z * z);
    }
    // projected centre
    dpx += gx * dfx / z;
    dpy += gy * dfy / z;
    dpz += -gx * dfx * dpx_ / (z * z) - gy * dfy * dpy_ / (z * z);
    // p = W mean + t
    dm[0] += Wd[0] * dpx + Wd[3] * dpy + Wd[6] * dpz;
    dm[1] += Wd[1] * dpx + Wd[4] * dpy + Wd[7] * dpz;
    dm[2] += Wd[2] * dpx + Wd[5] * dpy + Wd[8] * dpz;
    // Sigma = M M^T: dM = 2 dS M; M = R diag(s)
    dreal dR[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        const dreal dMij = 2.0 * (dS[i][0] * M[0][j] + dS[i][1] * M[1][j] + dS[i][2] * M[2][j]);
        dR[i][j] = dMij * sc[j];
        dls[j] += dMij * R[i][j] * sc[j];
      }
    // R(q_hat), q_hat = q / |q|
    const dreal dw = 2 * (-qz * dR[0][1] + qy * dR[0][2] + qz * dR[1][0] - qx * dR[1][2] - qy * dR[2][0] + qx * dR[2][1]);
    const dreal dx_ = 2 * (qy * dR[0][1] + qz * dR[0][2] + qy * dR[1][0] - 2 * qx * dR[1][1] - qw * dR[1][2] +
                            qz * dR[2][0] + qw * dR[2][1] - 2 * qx * dR[2][2]);
    const dreal dy_ = 2 * (-2 * qy * dR[0][0] + qx * dR[0][1] + qw * dR[0][2] + qx * dR[1][0] + qz * dR[1][2] -
                            qw * dR[2][0] + qz * dR[2][1] - 2 * qy * dR[2][2]);
    const dreal dz_ = 2 * (-2 * qz * dR[0][0] - qw * dR[0][1] + qx * dR[0][2] + qw * dR[1][0] - 2 * qz * dR[1][1] +
                            qy * dR[1][2] + qx * dR[2][0] + qy * dR[2][1]);
    const dreal dotq = dw * qw + dx_ * qx + dy_ * qy + dz_ * qz;
    dq[0] = (dw - dotq * qw) * qn;
    dq[1] = (dx_ - dotq * qx) * qn;
    dq[2] = (dy_ - dotq * qy) * qn;
    dq[3] = (dz_ - dotq * qz) * qn;
  }
  if (d_means)
    for (int i = 0; i < 3; ++i) d_means[3 * g + i] = (float)dm[i];
  if (d_log_scales)
    for (int i = 0; i < 3; ++i) d_log_scales[3 * g + i] = (float)dls[i];
  if (d_quats)
    for (int i = 0; i < 4; ++i) d_quats[4 * g + i] = (float)dq[i];
  if (d_logits) d_logits[g] = (float)dlogit;
  }  // g < n
  __syncthreads();
  if (d_sh)
    for (int64_t i = threadIdx.x; i < n_here * 3 * K; i += blockDim.x) d_sh[g0 * 3 * K + i] = sh_out[i];
}

int64_t preprocess_blocks(int64_t n) { return (n + 255) / 256; }

PlanarScene planar(const DeviceScene& s) { return PlanarScene{s.geo_a, s.geo_b, s.geo_q, s.sh, s.n}; }
RowMajorScene row_major(const DeviceScene& s) {
  return RowMajorScene{s.means, s.log_scales, s.quats, s.logits, s.sh_rows, 3 * s.n_coeff};
}

hipError_t launch_preprocess(const DeviceScene& s, const CamArgs& cam, const CullArgs& cull, adr_workspace* ws,
                             int64_t n_ranges, hipStream_t stream) {
  if (s.n == 0) return hipSuccess;
  static const ShConsts shc = make_sh_consts();
  const int64_t nb = preprocess_blocks(s.n);
  if (s.n > ws->gauss_capacity || 2 * (int64_t)cam.tiles_x * cam.tiles_y > 2 * ws->tile_capacity ||
      n_ranges > kNotifyClearMax)
    return hipErrorInvalidValue;
  if (s.borrowed)
    preprocess_kernel<<<dim3((unsigned)nb), 256, 0, stream>>>(row_major(s), s.n, s.n_coeff, shc, cam, cull, ws->rec,
                                                              ws->exact, ws->tile_rect, ws->depth.keys[0],
                                                              ws->depth.vals[0], ws->touched, ws->block_parts);
  else
    preprocess_kernel<<<dim3((unsigned)nb), 256, 0, stream>>>(planar(s), s.n, s.n_coeff, shc, cam, cull, ws->rec,
                                                              ws->exact, ws->tile_rect, ws->depth.keys[0],
                                                              ws->depth.vals[0], ws->touched, ws->block_parts);
  notify_host_kernel<<<1, 1024, 0, stream>>>(ws->block_parts, (int)nb, ws->dev_counters, ws->notify_dev,
                                             ws->frame_seq, ws->ranges, n_ranges, ws->load_acc);
  return hipGetLastError();
}

template <class Src>
hipError_t launch_preprocess_backward_src(const Src& src, int64_t n, int n_coeff, const CamArgs& cam, double lowpass,
                                          const float* grad2d, const adr_scene_grads& out, hipStream_t stream) {
  static const ShConsts shc = make_sh_consts();
  auto* kernel = n_coeff == 1   ? preprocess_backward_kernel<1, Src>
                 : n_coeff == 4 ? preprocess_backward_kernel<4, Src>
                 : n_coeff == 9 ? preprocess_backward_kernel<9, Src>
                                : preprocess_backward_kernel<16, Src>;
  kernel<<<dim3((unsigned)preprocess_blocks(n)), 256, 0, stream>>>(src, n, shc, cam, lowpass, grad2d, out.d_means,
                                                                    out.d_log_scales, out.d_quats,
                                                                    out.d_opacity_logits, out.d_sh);
  return hipGetLastError();
}

hipError_t launch_preprocess_backward(const DeviceScene& s, const CamArgs& cam, double lowpass, const float* grad2d,
                                      const adr_scene_grads& out, hipStream_t stream) {
  if (s.n == 0) return hipSuccess;
  if (s.borrowed) return launch_preprocess_backward_src(row_major(s), s.n, s.n_coeff, cam, lowpass, grad2d, out, stream);
  return launch_preprocess_backward_src(planar(s), s.n, s.n_coeff, cam, lowpass, grad2d, out, stream);
}

}  // namespace adr
