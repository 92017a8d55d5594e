// Scene upload: row-major float32 Gaussians -> library-owned planes in HBM.
// Geometry is packed into three float4 planes so Preprocess reads each
// Gaussian with three coalesced 16-byte loads; SH coefficients become 3K
// float planes so a wave reads 64 consecutive floats per coefficient.
#include "adr_internal.h"

#include <atomic>
#include <new>

namespace adr {

__global__ void __launch_bounds__(256) pack_scene_kernel(const float* __restrict__ means,
                                                          const float* __restrict__ log_scales,
                                                          const float* __restrict__ quats,
                                                          const float* __restrict__ logits,
                                                          const float* __restrict__ sh, int64_t n, int n_coeff,
                                                          float4* __restrict__ geo_a, float4* __restrict__ geo_b,
                                                          float4* __restrict__ geo_q, float* __restrict__ planes) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  geo_a[g] = make_float4(means[3 * g], means[3 * g + 1], means[3 * g + 2], logits[g]);
  geo_b[g] = make_float4(log_scales[3 * g], log_scales[3 * g + 1], log_scales[3 * g + 2], 0.f);
  geo_q[g] = make_float4(quats[4 * g], quats[4 * g + 1], quats[4 * g + 2], quats[4 * g + 3]);
  const int per = 3 * n_coeff;
  for (int c = 0; c < per; ++c) planes[(int64_t)c * n + g] = sh[g * per + c];
}

hipError_t launch_pack_scene(const adr_scene_desc& desc, const float* means, const float* log_scales,
                             const float* quats, const float* logits, const float* sh, DeviceScene& d,
                             hipStream_t stream) {
  if (d.n == 0) return hipSuccess;
  dim3 grid((unsigned)((d.n + 255) / 256));
  pack_scene_kernel<<<grid, 256, 0, stream>>>(means, log_scales, quats, logits, sh, d.n, d.n_coeff, d.geo_a,
                                              d.geo_b, d.geo_q, d.sh);
  return hipGetLastError();
}

}  // namespace adr

using namespace adr;

namespace {

void* scene_alloc(const adr_allocator& a, size_t bytes) {
  if (a.alloc) return a.alloc(bytes, nullptr, a.ctx);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void scene_free(const adr_allocator& a, void* p, size_t bytes) {
  if (!p) return;
  if (a.alloc)
    a.free(p, bytes, nullptr, a.ctx);
  else
    (void)hipFree(p);
}

void free_scene(adr_scene* s) {
  DeviceScene& d = s->d;
  if (!d.borrowed) {
    const size_t n_alloc = (size_t)(d.n > 0 ? d.n : 1);
    scene_free(s->alloc, d.geo_a, n_alloc * sizeof(float4));
    scene_free(s->alloc, d.geo_b, n_alloc * sizeof(float4));
    scene_free(s->alloc, d.geo_q, n_alloc * sizeof(float4));
    scene_free(s->alloc, d.sh, n_alloc * 3 * d.n_coeff * sizeof(float));
  }
  d = DeviceScene{};
}

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

}  // namespace

extern "C" adr_status adr_create_scene(const adr_scene_desc* desc, const adr_allocator* allocator,
                                       adr_scene** out) {
  if (!desc || !out) {
    set_error("adr_create_scene: NULL argument");
    return ADR_E_INVALID;
  }
  *out = nullptr;
  if (desc->n < 0 || desc->n > (int64_t)0x7fffffff) {
    set_error("adr_create_scene: n must be in [0, 2^31)");
    return ADR_E_INVALID;
  }
  if (desc->sh_degree < 0 || desc->sh_degree > 3) {
    set_error("adr_create_scene: sh_degree must be 0..3");
    return ADR_E_INVALID;
  }
  if (desc->n > 0 && (!desc->means || !desc->log_scales || !desc->quats || !desc->opacity_logits || !desc->sh)) {
    set_error("adr_create_scene: NULL array with n > 0");
    return ADR_E_INVALID;
  }
  if (allocator && (!allocator->alloc || !allocator->free)) {
    set_error("adr_create_scene: an allocator needs both alloc and free");
    return ADR_E_INVALID;
  }
  if (desc->borrow && !desc->pointers_on_device) {
    set_error("adr_create_scene: borrow = 1 needs device pointers");
    return ADR_E_INVALID;
  }
  if (desc->borrow && desc->n > 0 &&
      (!aligned(desc->quats, 16) || !aligned(desc->means, 4) || !aligned(desc->log_scales, 4) ||
       !aligned(desc->opacity_logits, 4) || !aligned(desc->sh, 4))) {
    set_error("adr_create_scene: a borrowed scene needs 16-byte aligned quats and 4-byte aligned arrays");
    return ADR_E_INVALID;
  }
  static std::atomic<uint64_t> next_uid{1};
  adr_scene* s = new (std::nothrow) adr_scene();
  if (!s) {
    set_error("adr_create_scene: host allocation failed");
    return ADR_E_OOM;
  }
  s->uid = next_uid.fetch_add(1);
  if (allocator) s->alloc = *allocator;
  DeviceScene& d = s->d;
  d.n = desc->n;
  d.sh_degree = desc->sh_degree;
  d.n_coeff = (desc->sh_degree + 1) * (desc->sh_degree + 1);
  const int64_t n = desc->n;
  if (desc->borrow) {
    // zero-copy: every render reads the caller's row-major arrays
    d.borrowed = true;
    d.means = desc->means;
    d.log_scales = desc->log_scales;
    d.quats = desc->quats;
    d.logits = desc->opacity_logits;
    d.sh_rows = desc->sh;
    d.bytes = 0;
    *out = s;
    return ADR_OK;
  }
  const size_t n_alloc = (size_t)(n > 0 ? n : 1);
  const size_t sh_floats = n_alloc * 3 * d.n_coeff;
  d.geo_a = static_cast<float4*>(scene_alloc(s->alloc, n_alloc * sizeof(float4)));
  d.geo_b = static_cast<float4*>(scene_alloc(s->alloc, n_alloc * sizeof(float4)));
  d.geo_q = static_cast<float4*>(scene_alloc(s->alloc, n_alloc * sizeof(float4)));
  d.sh = static_cast<float*>(scene_alloc(s->alloc, sh_floats * sizeof(float)));
  if (!d.geo_a || !d.geo_b || !d.geo_q || !d.sh) {
    free_scene(s);
    delete s;
    set_error("adr_create_scene: device allocation failed");
    return ADR_E_OOM;
  }
  d.bytes = n_alloc * 3 * sizeof(float4) + sh_floats * sizeof(float);
  if (n == 0) {
    *out = s;
    return ADR_OK;
  }
  // Stage host arrays (or use the caller's device arrays directly).
  const float* src[5] = {desc->means, desc->log_scales, desc->quats, desc->opacity_logits, desc->sh};
  const size_t counts[5] = {(size_t)n * 3, (size_t)n * 3, (size_t)n * 4, (size_t)n, (size_t)n * 3 * d.n_coeff};
  float* staged[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  adr_status st = ADR_OK;
  if (!desc->pointers_on_device) {
    for (int i = 0; i < 5 && st == ADR_OK; ++i) {
      staged[i] = static_cast<float*>(scene_alloc(s->alloc, counts[i] * sizeof(float)));
      if (!staged[i]) {
        set_error("adr_create_scene: staging allocation failed");
        st = ADR_E_OOM;
      } else if (hipMemcpy(staged[i], src[i], counts[i] * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
        st = hip_fail(hipGetLastError(), "hipMemcpy(scene upload)");
      }
    }
  }
  if (st == ADR_OK) {
    const float* p[5];
    for (int i = 0; i < 5; ++i) p[i] = desc->pointers_on_device ? src[i] : staged[i];
    hipError_t e = launch_pack_scene(*desc, p[0], p[1], p[2], p[3], p[4], d, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) st = hip_fail(e, "pack_scene_kernel");
  }
  for (int i = 0; i < 5; ++i) scene_free(s->alloc, staged[i], counts[i] * sizeof(float));
  if (st != ADR_OK) {
    free_scene(s);
    delete s;
    return st;
  }
  *out = s;
  return ADR_OK;
}

extern "C" void adr_destroy_scene(adr_scene* scene) {
  if (!scene) return;
  free_scene(scene);
  delete scene;
}

extern "C" int64_t adr_scene_size(const adr_scene* scene) { return scene ? scene->d.n : -1; }

extern "C" int64_t adr_scene_bytes(const adr_scene* scene) { return scene ? (int64_t)scene->d.bytes : -1; }
