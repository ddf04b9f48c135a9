// Per-tile rasterisation: front-to-back compositing and its adjoint.
//
// One workgroup per tile, one lane per pixel.  The tile's sorted records are
// staged through LDS in batches (one record per lane per batch); every lane
// then walks the batch.  The forward pass stops a pixel before the first
// record that would take its transmittance below 1e-4, and the workgroup
// stops when all its pixels have stopped.  The backward pass walks each
// tile back to front from the last contributor, recovers the transmittance
// in front of each record by division, reduces the per-record gradients
// over each wavefront and accumulates them with one atomic per component.
//
// Both passes take every per-pixel decision (support test, skip, stop)
// through the same inline functions, so the backward pass visits exactly
// the contributors the forward pass used.
#include "ubs_internal.hpp"

namespace ubs {

// Hardware base-2 exponential and logarithm (v_exp_f32 / v_log_f32).
__device__ __forceinline__ float hw_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float hw_log2(float x) { return __builtin_amdgcn_logf(x); }

// Record fields as staged in LDS.
struct Staged {
  float4 g0;  // mx, my, a, 2b
  float4 g1;  // c, rho, log2(o), beta
  float4 g2;  // r, g, b, (record index as bits)
};

__device__ __forceinline__ Staged stage_record(const float* __restrict__ records, uint32_t rec) {
  const float4* rp = reinterpret_cast<const float4*>(records + size_t(rec) * kRecFloats);
  const float4 a = rp[0], b = rp[1], c = rp[2];
  Staged s;
  s.g0 = make_float4(a.x, a.y, a.z, 2.0f * a.w);
  s.g1 = make_float4(b.x, b.y, hw_log2(b.z), b.w);
  s.g2 = make_float4(c.x, c.y, c.z, __uint_as_float(rec));
  return s;
}

// r = a dx^2 + 2 b dx dy + c dy^2 (squared Mahalanobis distance).
__device__ __forceinline__ float eval_r(const float4 g0, float c, float dx, float dy) {
  return dx * (g0.z * dx + g0.w * dy) + c * dy * dy;
}

// sigma = o (1 - r)^beta = exp2(log2 o + beta log2(1 - r)); alpha = min(0.99, sigma).
__device__ __forceinline__ float eval_sigma(float r, float lo, float beta, float* l2) {
  const float l = hw_log2(1.0f - r);
  *l2 = l;
  return hw_exp2(lo + beta * l);
}

__device__ __forceinline__ int view_of_tile(const DevView* __restrict__ views, int n_views,
                                            uint32_t tile) {
  int lo = 0, hi = n_views - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (views[mid].tile_base <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <int TW, int TH>
__global__ void __launch_bounds__(TW * TH) raster_fwd_kernel(
    const float* __restrict__ records, const uint32_t* __restrict__ values,
    const uint32_t* __restrict__ ranges, const DevView* __restrict__ views, int n_views,
    float* __restrict__ image, float* __restrict__ t_ws, float* __restrict__ t_user,
    uint32_t* __restrict__ ncontrib) {
  constexpr int NT = TW * TH;
  __shared__ float4 s0[NT], s1[NT], s2[NT];
  const uint32_t tile = blockIdx.x;
  const int vi = view_of_tile(views, n_views, tile);
  const DevView& V = views[vi];
  const uint32_t lt = tile - V.tile_base;
  const int ty = int(lt) / V.tiles_x, tx = int(lt) - ty * V.tiles_x;
  const int px = tx * TW + int(threadIdx.x) % TW, py = ty * TH + int(threadIdx.x) / TW;
  const bool inside = px < V.W && py < V.H;
  const float fx = float(px) + 0.5f, fy = float(py) + 0.5f;
  const uint32_t start = ranges[2 * size_t(tile)], end = ranges[2 * size_t(tile) + 1];
  float T = 1.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f;
  uint32_t last = 0;
  bool done = !inside;
  for (uint32_t b0 = start; b0 < end; b0 += NT) {
    if (__syncthreads_count(done) == NT) break;
    const uint32_t idx = b0 + threadIdx.x;
    if (idx < end) {
      const Staged st = stage_record(records, values[idx]);
      s0[threadIdx.x] = st.g0;
      s1[threadIdx.x] = st.g1;
      s2[threadIdx.x] = st.g2;
    }
    __syncthreads();
    if (!done) {
      const int nb = int(min(uint32_t(NT), end - b0));
      for (int j = 0; j < nb; ++j) {
        const float4 g0 = s0[j], g1 = s1[j];
        const float dx = fx - g0.x, dy = fy - g0.y;
        const float r = eval_r(g0, g1.x, dx, dy);
        if (!(r <= g1.y)) continue;
        float l2;
        const float sigma = eval_sigma(r, g1.z, g1.w, &l2);
        const float alpha = fminf(kAlphaMax, sigma);
        if (alpha < kAlphaMin) continue;
        const float test = T * (1.0f - alpha);
        if (test < kTStop) { done = true; break; }
        const float4 g2 = s2[j];
        const float w = alpha * T;
        cr += g2.x * w;
        cg += g2.y * w;
        cb += g2.z * w;
        T = test;
        last = b0 - start + uint32_t(j) + 1u;
      }
    }
  }
  if (inside) {
    const size_t pix = size_t(V.pix_base) + size_t(py) * V.W + px;
    image[3 * pix] = cr;
    image[3 * pix + 1] = cg;
    image[3 * pix + 2] = cb;
    t_ws[pix] = T;
    if (t_user) t_user[pix] = T;
    ncontrib[pix] = last;
  }
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <int TW, int TH>
__global__ void __launch_bounds__(TW * TH) raster_bwd_kernel(
    const float* __restrict__ records, const uint32_t* __restrict__ values,
    const uint32_t* __restrict__ ranges, const DevView* __restrict__ views, int n_views,
    const float* __restrict__ t_ws, const uint32_t* __restrict__ ncontrib,
    const float* __restrict__ d_image, const float* __restrict__ d_tfinal,
    const float* __restrict__ l1_image, const float* __restrict__ l1_target, float l1_scale,
    float* __restrict__ grad2d) {
  constexpr int NT = TW * TH;
  __shared__ float4 s0[NT], s1[NT], s2[NT];
  __shared__ uint32_t s_max;
  const uint32_t tile = blockIdx.x;
  const int vi = view_of_tile(views, n_views, tile);
  const DevView& V = views[vi];
  const uint32_t lt = tile - V.tile_base;
  const int ty = int(lt) / V.tiles_x, tx = int(lt) - ty * V.tiles_x;
  const int px = tx * TW + int(threadIdx.x) % TW, py = ty * TH + int(threadIdx.x) / TW;
  const bool inside = px < V.W && py < V.H;
  const float fx = float(px) + 0.5f, fy = float(py) + 0.5f;
  const uint32_t start = ranges[2 * size_t(tile)], end = ranges[2 * size_t(tile) + 1];
  if (threadIdx.x == 0) s_max = 0;
  float Tf = 1.0f, gR = 0.0f, gG = 0.0f, gB = 0.0f, gT = 0.0f;
  uint32_t last = 0;
  if (inside) {
    const size_t pix = size_t(V.pix_base) + size_t(py) * V.W + px;
    Tf = t_ws[pix];
    last = ncontrib[pix];
    if (d_image) {
      gR = d_image[3 * pix];
      gG = d_image[3 * pix + 1];
      gB = d_image[3 * pix + 2];
      if (d_tfinal) gT = d_tfinal[pix];
    } else {
      const float e0 = l1_image[3 * pix] - l1_target[3 * pix];
      const float e1 = l1_image[3 * pix + 1] - l1_target[3 * pix + 1];
      const float e2 = l1_image[3 * pix + 2] - l1_target[3 * pix + 2];
      gR = e0 > 0.0f ? l1_scale : (e0 < 0.0f ? -l1_scale : 0.0f);
      gG = e1 > 0.0f ? l1_scale : (e1 < 0.0f ? -l1_scale : 0.0f);
      gB = e2 > 0.0f ? l1_scale : (e2 < 0.0f ? -l1_scale : 0.0f);
    }
  }
  __syncthreads();
  if (last > 0) atomicMax(&s_max, last);
  __syncthreads();
  const uint32_t span = s_max;
  float T = Tf;                       // transmittance behind the current record
  float Sr = 0.0f, Sg = 0.0f, Sb = 0.0f;  // colour accumulated behind it
  const int lane = threadIdx.x & 63;
  for (uint32_t hi = span; hi > 0;) {
    const uint32_t lo = hi > uint32_t(NT) ? hi - uint32_t(NT) : 0u;
    const uint32_t cnt = hi - lo;
    __syncthreads();
    if (threadIdx.x < cnt) {
      const Staged st = stage_record(records, values[start + lo + threadIdx.x]);
      s0[threadIdx.x] = st.g0;
      s1[threadIdx.x] = st.g1;
      s2[threadIdx.x] = st.g2;
    }
    __syncthreads();
    for (int j = int(cnt) - 1; j >= 0; --j) {
      const uint32_t pos = lo + uint32_t(j);
      float gv[kGradFloats];
#pragma unroll
      for (int k = 0; k < kGradFloats; ++k) gv[k] = 0.0f;
      bool contrib = false;
      if (pos < last) {
        const float4 g0 = s0[j], g1 = s1[j];
        const float dx = fx - g0.x, dy = fy - g0.y;
        const float r = eval_r(g0, g1.x, dx, dy);
        if (r <= g1.y) {
          float l2;
          const float sigma = eval_sigma(r, g1.z, g1.w, &l2);
          const float alpha = fminf(kAlphaMax, sigma);
          if (alpha >= kAlphaMin) {
            contrib = true;
            const float4 g2 = s2[j];
            const float oma = 1.0f - alpha;
            const float Ti = T / oma;
            const float w = alpha * Ti;
            gv[7] = gR * w;
            gv[8] = gG * w;
            gv[9] = gB * w;
            const float dalpha = Ti * (gR * (g2.x - Sr) + gG * (g2.y - Sg) + gB * (g2.z - Sb)) -
                                 gT * Tf / oma;
            Sr = alpha * g2.x + oma * Sr;
            Sg = alpha * g2.y + oma * Sg;
            Sb = alpha * g2.z + oma * Sb;
            T = Ti;
            if (sigma < kAlphaMax) {
              const float base = 1.0f - r;
              gv[5] = dalpha * hw_exp2(g1.w * l2);                  // d sigma / d o = (1-r)^beta
              gv[6] = dalpha * sigma * l2 * 0.69314718f;            // d sigma / d beta
              const float dr = -dalpha * g1.w * sigma / base;       // d sigma / d r
              const float b = 0.5f * g0.w;
              gv[0] = -2.0f * dr * (g0.z * dx + b * dy);
              gv[1] = -2.0f * dr * (b * dx + g1.x * dy);
              gv[2] = dr * dx * dx;
              gv[3] = 2.0f * dr * dx * dy;
              gv[4] = dr * dy * dy;
            }
          }
        }
      }
      if (__ballot(contrib) != 0ull) {
        const uint32_t rec = __float_as_uint(s2[j].w);
        float* gp = grad2d + size_t(rec) * kGradFloats;
#pragma unroll
        for (int k = 0; k < kGradFloats; ++k) {
          const float s = wave_sum(gv[k]);
          if (lane == 0 && s != 0.0f) atomicAdd(gp + k, s);
        }
      }
    }
    hi = lo;
  }
}

template <int TW, int TH>
static hipError_t raster_fwd_t(const float* records, const uint32_t* values, const uint32_t* ranges,
                               const DevView* views, int n_views, uint32_t n_tiles, float* image,
                               float* t_ws, float* t_user, uint32_t* ncontrib, hipStream_t st) {
  hipLaunchKernelGGL((raster_fwd_kernel<TW, TH>), dim3(n_tiles), dim3(TW * TH), 0, st, records,
                     values, ranges, views, n_views, image, t_ws, t_user, ncontrib);
  return hipGetLastError();
}

template <int TW, int TH>
static hipError_t raster_bwd_t(const float* records, const uint32_t* values, const uint32_t* ranges,
                               const DevView* views, int n_views, uint32_t n_tiles,
                               const float* t_ws, const uint32_t* ncontrib, const float* d_image,
                               const float* d_tfinal, const float* l1_image,
                               const float* l1_target, float l1_scale, float* grad2d,
                               hipStream_t st) {
  hipLaunchKernelGGL((raster_bwd_kernel<TW, TH>), dim3(n_tiles), dim3(TW * TH), 0, st, records,
                     values, ranges, views, n_views, t_ws, ncontrib, d_image, d_tfinal, l1_image,
                     l1_target, l1_scale, grad2d);
  return hipGetLastError();
}

hipError_t launch_raster_fwd(int tw, int th, const float* records, const uint32_t* values,
                             const uint32_t* ranges, const DevView* views, int n_views,
                             uint32_t n_tiles, float* image, float* t_ws, float* t_user,
                             uint32_t* ncontrib, hipStream_t st) {
  if (n_tiles == 0) return hipSuccess;
  if (tw == 16 && th == 16)
    return raster_fwd_t<16, 16>(records, values, ranges, views, n_views, n_tiles, image, t_ws, t_user, ncontrib, st);
  if (tw == 16 && th == 8)
    return raster_fwd_t<16, 8>(records, values, ranges, views, n_views, n_tiles, image, t_ws, t_user, ncontrib, st);
  if (tw == 8 && th == 8)
    return raster_fwd_t<8, 8>(records, values, ranges, views, n_views, n_tiles, image, t_ws, t_user, ncontrib, st);
  if (tw == 32 && th == 16)
    return raster_fwd_t<32, 16>(records, values, ranges, views, n_views, n_tiles, image, t_ws, t_user, ncontrib, st);
  return hipErrorInvalidValue;
}

hipError_t launch_raster_bwd(int tw, int th, const float* records, const uint32_t* values,
                             const uint32_t* ranges, const DevView* views, int n_views,
                             uint32_t n_tiles, const float* t_ws, const uint32_t* ncontrib,
                             const float* d_image, const float* d_tfinal, const float* l1_image,
                             const float* l1_target, float l1_scale, float* grad2d,
                             hipStream_t st) {
  if (n_tiles == 0) return hipSuccess;
  if (tw == 16 && th == 16)
    return raster_bwd_t<16, 16>(records, values, ranges, views, n_views, n_tiles, t_ws, ncontrib, d_image, d_tfinal, l1_image, l1_target, l1_scale, grad2d, st);
  if (tw == 16 && th == 8)
    return raster_bwd_t<16, 8>(records, values, ranges, views, n_views, n_tiles, t_ws, ncontrib, d_image, d_tfinal, l1_image, l1_target, l1_scale, grad2d, st);
  if (tw == 8 && th == 8)
    return raster_bwd_t<8, 8>(records, values, ranges, views, n_views, n_tiles, t_ws, ncontrib, d_image, d_tfinal, l1_image, l1_target, l1_scale, grad2d, st);
  if (tw == 32 && th == 16)
    return raster_bwd_t<32, 16>(records, values, ranges, views, n_views, n_tiles, t_ws, ncontrib, d_image, d_tfinal, l1_image, l1_target, l1_scale, grad2d, st);
  return hipErrorInvalidValue;
}

}  // namespace ubs
