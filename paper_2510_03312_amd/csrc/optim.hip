// One optimisation step over a scene's [F][n] parameters (Sec. 4.5 loss
// regularisers and spatial noise, Adam with per-group rates as in Sec. 5.1):
// a single streaming pass that reads params, dparams, m, v (and the noise of
// the three spatial-mean rows) and writes params, m, v in place.
//
// Per row r the host passes the Adam step size lr_r / (1 - beta1^t) and the
// row's regulariser kind; every element then computes
//   g  = dparams + (opacity row: lambda_o sign(o); log-scale rows:
//        lambda_Sigma exp(log s); other rows: 0)
//   m  = beta1 m + (1 - beta1) g,  v = beta2 v + (1 - beta2) g^2
//   p -= step_r m / (sqrt(v) / sqrt(1 - beta2^t) + eps)
// and the spatial-mean rows add lambda_eps * noise afterwards.
#include <cmath>

#include "ubs_internal.hpp"

namespace ubs {

constexpr int kAdamMaxRows = kMaxRows;

enum : uint8_t { kRegNone = 0, kRegOpacity = 1, kRegScale = 2, kRegNoise = 3 };

struct AdamRows {
  float step_size[kAdamMaxRows];   // lr_r / (1 - beta1^t)
  uint8_t kind[kAdamMaxRows];      // kReg* of the row
};

struct AdamScalars {
  float beta1, beta2, eps, inv_sqrt_bc2, lambda_o, lambda_s, lambda_eps;
  int32_t has_noise;
};

constexpr int kAdamItems = 4;   // elements per thread, 256 apart

__device__ __forceinline__ float adam_one(float p, float g, float& m, float& v, float step,
                                          uint8_t kind, const AdamScalars& a) {
  if (kind == kRegOpacity) g += a.lambda_o * (p > 0.0f ? 1.0f : (p < 0.0f ? -1.0f : 0.0f));
  if (kind == kRegScale) g += a.lambda_s * expf(p);
  m = a.beta1 * m + (1.0f - a.beta1) * g;
  v = a.beta2 * v + (1.0f - a.beta2) * g * g;
  return p - step * m / (sqrtf(v) * a.inv_sqrt_bc2 + a.eps);
}


__global__ void __launch_bounds__(256) adam_kernel(AdamRows rows, AdamScalars a, int64_t n,
                                                   float* __restrict__ params,
                                                   const float* __restrict__ dparams,
                                                   float* __restrict__ m, float* __restrict__ v,
                                                   const float* __restrict__ noise) {
  const int r = blockIdx.y;
  const int64_t row = int64_t(r) * n;
  const float step = rows.step_size[r];
  const uint8_t kind = rows.kind[r];
  const int64_t i0 = int64_t(blockIdx.x) * (256 * kAdamItems) + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kAdamItems; ++k) {
    const int64_t i = i0 + int64_t(k) * 256;
    if (i >= n) break;
    float mm = load_stream(m + row + i), vv = load_stream(v + row + i);
    float q = adam_one(load_stream(params + row + i), load_stream(dparams + row + i), mm, vv, step,
                       kind, a);
    // the spatial-mean rows are rows 0-2, noise row r is noise[r * n ...]
    if (kind == kRegNoise && a.has_noise) q += a.lambda_eps * noise[row + i];
    store_stream(params + row + i, q);
    store_stream(m + row + i, mm);
    store_stream(v + row + i, vv);
  }
}

// Same step with 16-byte accesses: four consecutive elements per thread
// (rows must start 16-byte aligned: n % 4 == 0 and aligned buffers).
__global__ void __launch_bounds__(256) adam_kernel_vec4(AdamRows rows, AdamScalars a, int64_t n,
                                                        float* __restrict__ params,
                                                        const float* __restrict__ dparams,
                                                        float* __restrict__ m,
                                                        float* __restrict__ v,
                                                        const float* __restrict__ noise) {
  const int r = blockIdx.y;
  const int64_t row4 = int64_t(r) * (n / 4);
  const float step = rows.step_size[r];
  const uint8_t kind = rows.kind[r];
  const int64_t j = int64_t(blockIdx.x) * 256 + threadIdx.x;   // float4 index in the row
  if (j >= n / 4) return;
  float4 p = load_stream(reinterpret_cast<const float4*>(params) + row4 + j);
  const float4 g = load_stream(reinterpret_cast<const float4*>(dparams) + row4 + j);
  float4 mm = load_stream(reinterpret_cast<const float4*>(m) + row4 + j);
  float4 vv = load_stream(reinterpret_cast<const float4*>(v) + row4 + j);
  p.x = adam_one(p.x, g.x, mm.x, vv.x, step, kind, a);
  p.y = adam_one(p.y, g.y, mm.y, vv.y, step, kind, a);
  p.z = adam_one(p.z, g.z, mm.z, vv.z, step, kind, a);
  p.w = adam_one(p.w, g.w, mm.w, vv.w, step, kind, a);
  if (kind == kRegNoise && a.has_noise) {
    const float4 e = load_stream(reinterpret_cast<const float4*>(noise) + row4 + j);
    p.x += a.lambda_eps * e.x;
    p.y += a.lambda_eps * e.y;
    p.z += a.lambda_eps * e.z;
    p.w += a.lambda_eps * e.w;
  }
  store_stream(reinterpret_cast<float4*>(params) + row4 + j, p);
  store_stream(reinterpret_cast<float4*>(m) + row4 + j, mm);
  store_stream(reinterpret_cast<float4*>(v) + row4 + j, vv);
}

}  // namespace ubs

using namespace ubs;

static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

extern "C" ubs_status ubs_adam_step(const ubs_adam* cfg, int32_t dim, int32_t rot, int64_t n,
                                    float* params, const float* dparams, float* m, float* v,
                                    const float* noise, void* stream) {
  if (!cfg) return UBS_ERR_ARG;
  if (dim < 3 || dim > kMaxDim || (rot != UBS_ROT_QUAT && rot != UBS_ROT_SKEW) || n < 0)
    return UBS_ERR_ARG;
  if (!dim_ok(dim)) return UBS_ERR_UNSUPPORTED;
  if (cfg->step < 1 || !(cfg->beta1 >= 0.0f && cfg->beta1 < 1.0f) ||
      !(cfg->beta2 >= 0.0f && cfg->beta2 < 1.0f) || !(cfg->eps >= 0.0f))
    return UBS_ERR_ARG;
  if (n == 0) return UBS_OK;
  if (!params || !dparams || !m || !v) return UBS_ERR_ARG;
  const ParamRows pr = param_rows(dim - 3, rot);
  if (pr.F > kAdamMaxRows) return UBS_ERR_UNSUPPORTED;
  AdamRows rows{};
  const double bc1 = 1.0 - std::pow(double(cfg->beta1), double(cfg->step));
  const double bc2 = 1.0 - std::pow(double(cfg->beta2), double(cfg->step));
  for (int r = 0; r < pr.F; ++r) {
    float lr = cfg->lr_other;
    uint8_t kind = kRegNone;
    if (r >= pr.mu_x && r < pr.mu_x + 3) { lr = cfg->lr_mu_x; kind = kRegNoise; }
    if (r >= pr.log_s && r < pr.log_s + 3) { lr = cfg->lr_scale; kind = kRegScale; }
    if (r == pr.o) { lr = cfg->lr_opacity; kind = kRegOpacity; }
    rows.step_size[r] = float(double(lr) / bc1);
    rows.kind[r] = kind;
  }
  AdamScalars a{};
  a.beta1 = cfg->beta1;
  a.beta2 = cfg->beta2;
  a.eps = cfg->eps;
  a.inv_sqrt_bc2 = float(1.0 / std::sqrt(bc2));
  a.lambda_o = cfg->lambda_o;
  a.lambda_s = cfg->lambda_s;
  a.lambda_eps = cfg->lambda_eps;
  a.has_noise = noise != nullptr ? 1 : 0;
  const bool vec4 = n % 4 == 0 && aligned16(params) && aligned16(dparams) && aligned16(m) &&
                    aligned16(v) && (!noise || aligned16(noise));
  const int64_t per_block = vec4 ? 256 * 4 : 256 * kAdamItems;
  const int64_t blocks = (n + per_block - 1) / per_block;
  if (blocks > 0x7fffffff) return UBS_ERR_UNSUPPORTED;
  if (vec4)
    hipLaunchKernelGGL(adam_kernel_vec4, dim3(unsigned(blocks), unsigned(pr.F)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), rows, a, n, params, dparams, m, v, noise);
  else
    hipLaunchKernelGGL(adam_kernel, dim3(unsigned(blocks), unsigned(pr.F)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), rows, a, n, params, dparams, m, v, noise);
  return hipGetLastError() == hipSuccess ? UBS_OK : UBS_ERR_HIP;
}
