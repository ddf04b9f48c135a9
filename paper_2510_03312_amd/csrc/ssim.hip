// The loss of Sec. 4.5, (1 - lambda) L1 + lambda (1 - mean SSIM), and its
// image gradient, over every view of a frame (images concatenated).
//
// SSIM per pixel and channel from local statistics under an 11 x 11
// Gaussian window (sigma 1.5, zero padding outside the view): means m_x,
// m_y and second moments s_xx, s_yy, s_xy;
//   S = (2 m_x m_y + C1)(2 (s_xy - m_x m_y) + C2)
//       / ((m_x^2 + m_y^2 + C1)((s_xx - m_x^2) + (s_yy - m_y^2) + C2)).
// The gradient of the mean of S with respect to the image is the window
// applied once more, to the per-pixel partials of S with respect to m_x,
// s_xx and s_xy:
//   dS/dx(p) = sum_q G(q - p) [dS/dm_x(q) + 2 x(p) dS/ds_xx(q) + y(p) dS/ds_xy(q)].
// Two stencil kernels, each over 16 x 16 tiles with an LDS patch of
// (16 + 10)^2 pixels per channel and separable passes:
//   ssim_fwd  statistics, S, the three partials (times -lambda / n) to the
//             workspace (nine planes of all pixels: partial k of channel c
//             in plane 3 c + k, so the backward's patch rows are contiguous),
//             per-tile sums of S and |x - y|
//   ssim_bwd  the window over the partials, the L1 term, d_image
// and one workgroup adds the per-tile sums into the loss.
#include <cmath>
#include <vector>

#include "ubs_internal.hpp"

namespace ubs {

constexpr int kSsimTile = 16;
constexpr int kSsimR = 5;                        // window half-width
constexpr int kSsimP = kSsimTile + 2 * kSsimR;   // 26
constexpr float kC1 = 0.01f * 0.01f;
constexpr float kC2 = 0.03f * 0.03f;
constexpr int kSsimViewChunk = 64;
constexpr int kSsimTmpW = kSsimTile + 1;   // padded row of the row-pass buffer (LDS banks)

struct SsimView {
  int32_t W, H, tiles_x;
  uint32_t tile_base, pix_base;
  uint32_t _pad[3];
};

struct SsimViewChunk {
  SsimView v[kSsimViewChunk];
  int32_t first, count;
};

__global__ void ssim_upload_kernel(SsimViewChunk c, SsimView* __restrict__ dst) {
  const int k = threadIdx.x;
  if (k < c.count) dst[c.first + k] = c.v[k];
}

// Normalised taps of the 11-tap Gaussian (sigma 1.5), filled by the host.
struct SsimTaps {
  float g[2 * kSsimR + 1];
};

__device__ __forceinline__ int ssim_view_of_tile(const SsimView* __restrict__ views, int n_views,
                                                 uint32_t tile) {
  int lo = 0, hi = n_views - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (views[mid].tile_base <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Separable window over an LDS patch, NQ quantities at once: rows first
// (kSsimP rows x 16 columns into tmp), then columns (16 x 16, left in
// in[q][r][c] for r, c < 16, from where each thread reads its pixel).  A
// thread computes 8 consecutive outputs from 18 consecutive inputs held in
// registers (a sliding window), so each output costs about 2.3 LDS reads
// instead of 11.  in[q][kSsimP][kSsimP], tmp[q][kSsimP][kSsimTmpW].
constexpr int kSsimRun = 8;                       // outputs per thread and pass
constexpr int kSsimSpan = kSsimRun + 2 * kSsimR;  // 18 inputs per run

template <int NQ>
__device__ __forceinline__ void window_16x16(float (*in)[kSsimP][kSsimP],
                                             float (*tmp)[kSsimP][kSsimTmpW], const SsimTaps& t,
                                             float* out) {
  const int tid = threadIdx.x;
  constexpr int kRuns = kSsimTile / kSsimRun;     // 2 runs per row or column
  // rows: task = (q, r, run)
  for (int task = tid; task < NQ * kSsimP * kRuns; task += 256) {
    const int q = task / (kSsimP * kRuns), rem = task % (kSsimP * kRuns);
    const int r = rem / kRuns, c0 = (rem % kRuns) * kSsimRun;
    float v[kSsimSpan];
#pragma unroll
    for (int k = 0; k < kSsimSpan; ++k) v[k] = in[q][r][c0 + k];
#pragma unroll
    for (int o = 0; o < kSsimRun; ++o) {
      float acc = 0.0f;
#pragma unroll
      for (int k = 0; k <= 2 * kSsimR; ++k) acc += t.g[k] * v[o + k];
      tmp[q][r][c0 + o] = acc;
    }
  }
  __syncthreads();
  // columns: task = (q, c, run), results into in[q][r][c]
  for (int task = tid; task < NQ * kSsimTile * kRuns; task += 256) {
    const int q = task / (kSsimTile * kRuns), rem = task % (kSsimTile * kRuns);
    const int c = rem % kSsimTile, r0 = (rem / kSsimTile) * kSsimRun;
    float v[kSsimSpan];
#pragma unroll
    for (int k = 0; k < kSsimSpan; ++k) v[k] = tmp[q][r0 + k][c];
#pragma unroll
    for (int o = 0; o < kSsimRun; ++o) {
      float acc = 0.0f;
#pragma unroll
      for (int k = 0; k <= 2 * kSsimR; ++k) acc += t.g[k] * v[o + k];
      in[q][r0 + o][c] = acc;
    }
  }
  __syncthreads();
  const int r = tid / kSsimTile, c = tid % kSsimTile;
#pragma unroll
  for (int q = 0; q < NQ; ++q) out[q] = in[q][r][c];
}

__global__ void __launch_bounds__(256) ssim_fwd_kernel(
    const SsimView* __restrict__ views, int n_views, const float* __restrict__ image,
    const float* __restrict__ target, SsimTaps taps, float scale,
    float* __restrict__ dstat, uint32_t n_pixels, double* __restrict__ tile_sums) {
  __shared__ float s_in[5][kSsimP][kSsimP];      // x, y, xx, yy, xy
  __shared__ float s_tmp[5][kSsimP][kSsimTmpW];
  __shared__ float s_px[2][kSsimP * kSsimP][3];  // the patch of image and target, RGB
  __shared__ double s_red[2][4];
  const uint32_t tile = blockIdx.x;
  const SsimView& V = views[ssim_view_of_tile(views, n_views, tile)];
  const int lt = int(tile - V.tile_base);
  const int ty = lt / V.tiles_x, tx = lt - ty * V.tiles_x;
  const int x0 = tx * kSsimTile - kSsimR, y0 = ty * kSsimTile - kSsimR;
  const int tid = threadIdx.x;
  const int px = tx * kSsimTile + tid % kSsimTile, py = ty * kSsimTile + tid / kSsimTile;
  const bool inside = px < V.W && py < V.H;
  const size_t pix = size_t(V.pix_base) + size_t(py) * V.W + px;
  // the patch's three channels at once (one 12-byte pixel per lane)
  for (int e = tid; e < kSsimP * kSsimP; e += 256) {
    const int r = e / kSsimP, c = e % kSsimP;
    const int gx = x0 + c, gy = y0 + r;
    float a[3] = {0.0f, 0.0f, 0.0f}, b[3] = {0.0f, 0.0f, 0.0f};
    if (gx >= 0 && gx < V.W && gy >= 0 && gy < V.H) {
      const size_t q = size_t(V.pix_base) + size_t(gy) * V.W + gx;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        a[ch] = image[3 * q + ch];
        b[ch] = target[3 * q + ch];
      }
    }
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      s_px[0][e][ch] = a[ch];
      s_px[1][e][ch] = b[ch];
    }
  }
  double s_sum = 0.0, l1_sum = 0.0;
  for (int ch = 0; ch < 3; ++ch) {
    __syncthreads();
    for (int e = tid; e < kSsimP * kSsimP; e += 256) {
      const int r = e / kSsimP, c = e % kSsimP;
      const float a = s_px[0][e][ch], b = s_px[1][e][ch];
      s_in[0][r][c] = a;
      s_in[1][r][c] = b;
      s_in[2][r][c] = a * a;
      s_in[3][r][c] = b * b;
      s_in[4][r][c] = a * b;
    }
    __syncthreads();
    float st[5];
    window_16x16<5>(s_in, s_tmp, taps, st);
    if (inside) {
      const float mx = st[0], my = st[1];
      const float a1 = 2.0f * mx * my + kC1;
      const float a2 = 2.0f * (st[4] - mx * my) + kC2;
      const float b1 = mx * mx + my * my + kC1;
      const float b2 = (st[2] - mx * mx) + (st[3] - my * my) + kC2;
      const float ib = 1.0f / (b1 * b2);
      const float S = a1 * a2 * ib;
      const float d_m = 2.0f * my * (a2 - a1) * ib - 2.0f * mx * S * (1.0f / b1 - 1.0f / b2);
      const float d_sxx = -S / b2;
      const float d_sxy = 2.0f * a1 * ib;
      float* d = dstat + size_t(3 * ch) * n_pixels + pix;
      d[0] = scale * d_m;
      d[n_pixels] = scale * d_sxx;
      d[2 * size_t(n_pixels)] = scale * d_sxy;
      s_sum += S;
      const int e = (tid / kSsimTile + kSsimR) * kSsimP + tid % kSsimTile + kSsimR;
      l1_sum += fabsf(s_px[0][e][ch] - s_px[1][e][ch]);
    }
  }
  // tile sums of S and |x - y|
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    s_sum += __shfl_xor(s_sum, o, 64);
    l1_sum += __shfl_xor(l1_sum, o, 64);
  }
  if ((tid & 63) == 0) {
    s_red[0][tid >> 6] = s_sum;
    s_red[1][tid >> 6] = l1_sum;
  }
  __syncthreads();
  if (tid == 0) {
    tile_sums[2 * size_t(tile)] = (s_red[0][0] + s_red[0][1]) + (s_red[0][2] + s_red[0][3]);
    tile_sums[2 * size_t(tile) + 1] = (s_red[1][0] + s_red[1][1]) + (s_red[1][2] + s_red[1][3]);
  }
}

__global__ void __launch_bounds__(256) ssim_bwd_kernel(
    const SsimView* __restrict__ views, int n_views, const float* __restrict__ image,
    const float* __restrict__ target, SsimTaps taps, float l1_weight,
    const float* __restrict__ dstat, uint32_t n_pixels, float* __restrict__ d_image) {
  __shared__ float s_in[3][kSsimP][kSsimP];      // d/dm, d/dsxx, d/dsxy
  __shared__ float s_tmp[3][kSsimP][kSsimTmpW];
  const uint32_t tile = blockIdx.x;
  const SsimView& V = views[ssim_view_of_tile(views, n_views, tile)];
  const int lt = int(tile - V.tile_base);
  const int ty = lt / V.tiles_x, tx = lt - ty * V.tiles_x;
  const int x0 = tx * kSsimTile - kSsimR, y0 = ty * kSsimTile - kSsimR;
  const int tid = threadIdx.x;
  const int px = tx * kSsimTile + tid % kSsimTile, py = ty * kSsimTile + tid / kSsimTile;
  const bool inside = px < V.W && py < V.H;
  const size_t pix = size_t(V.pix_base) + size_t(py) * V.W + px;
  for (int ch = 0; ch < 3; ++ch) {
    __syncthreads();
    for (int e = tid; e < kSsimP * kSsimP; e += 256) {
      const int r = e / kSsimP, c = e % kSsimP;
      const int gx = x0 + c, gy = y0 + r;
      float a = 0.0f, b = 0.0f, d = 0.0f;
      if (gx >= 0 && gx < V.W && gy >= 0 && gy < V.H) {
        const float* q = dstat + size_t(3 * ch) * n_pixels + size_t(V.pix_base) + size_t(gy) * V.W + gx;
        a = q[0];
        b = q[n_pixels];
        d = q[2 * size_t(n_pixels)];
      }
      s_in[0][r][c] = a;
      s_in[1][r][c] = b;
      s_in[2][r][c] = d;
    }
    __syncthreads();
    float w[3];
    window_16x16<3>(s_in, s_tmp, taps, w);
    if (inside) {
      const float x = image[3 * pix + ch], y = target[3 * pix + ch];
      const float diff = x - y;
      const float sgn = diff > 0.0f ? 1.0f : (diff < 0.0f ? -1.0f : 0.0f);
      d_image[3 * pix + ch] = w[0] + 2.0f * x * w[1] + y * w[2] + l1_weight * sgn;
    }
  }
}

// loss = (1 - lambda) sum|x - y| / n + lambda (1 - sum S / n)
__global__ void __launch_bounds__(256) ssim_loss_kernel(const double* __restrict__ tile_sums,
                                                        uint32_t n_tiles, double n_entries,
                                                        double lambda, double* __restrict__ loss) {
  __shared__ double s_red[2][4];
  double s = 0.0, l = 0.0;
  for (uint32_t k = threadIdx.x; k < n_tiles; k += 256) {
    s += tile_sums[2 * size_t(k)];
    l += tile_sums[2 * size_t(k) + 1];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    s += __shfl_xor(s, o, 64);
    l += __shfl_xor(l, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    s_red[0][threadIdx.x >> 6] = s;
    s_red[1][threadIdx.x >> 6] = l;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double S = (s_red[0][0] + s_red[0][1]) + (s_red[0][2] + s_red[0][3]);
    const double L1 = (s_red[1][0] + s_red[1][1]) + (s_red[1][2] + s_red[1][3]);
    *loss = (1.0 - lambda) * L1 / n_entries + lambda * (1.0 - S / n_entries);
  }
}

}  // namespace ubs

using namespace ubs;

static uint64_t ssim_align(uint64_t x) { return (x + 255) & ~uint64_t(255); }

extern "C" ubs_status ubs_ssim_loss(int32_t n_views, const int32_t* sizes, const float* image,
                                    const float* target, float lambda_ssim, float* d_image,
                                    double* loss, void* ws, uint64_t ws_bytes,
                                    uint64_t* ws_bytes_needed, void* stream) {
  if (n_views < 0 || n_views > UBS_MAX_VIEWS || (n_views > 0 && !sizes)) return UBS_ERR_ARG;
  if (!(lambda_ssim >= 0.0f && lambda_ssim <= 1.0f)) return UBS_ERR_ARG;
  std::vector<SsimView> vs(size_t(n_views > 0 ? n_views : 0));
  uint64_t tiles = 0, pixels = 0;
  for (int v = 0; v < n_views; ++v) {
    const int W = sizes[2 * v], H = sizes[2 * v + 1];
    if (W < 1 || H < 1 || W > 16384 || H > 16384) return UBS_ERR_ARG;
    SsimView s{};
    s.W = W;
    s.H = H;
    s.tiles_x = (W + kSsimTile - 1) / kSsimTile;
    s.tile_base = uint32_t(tiles);
    s.pix_base = uint32_t(pixels);
    tiles += uint64_t(s.tiles_x) * uint64_t((H + kSsimTile - 1) / kSsimTile);
    pixels += uint64_t(W) * uint64_t(H);
    if (pixels > 0x7fffffffull) return UBS_ERR_UNSUPPORTED;
    vs[size_t(v)] = s;
  }
  const uint64_t off_views = 0;
  const uint64_t off_sums = ssim_align(off_views + sizeof(SsimView) * uint64_t(n_views > 0 ? n_views : 1));
  const uint64_t off_dstat = ssim_align(off_sums + 16 * (tiles > 0 ? tiles : 1));
  const uint64_t need = ssim_align(off_dstat + 36 * pixels);
  if (!ws) {
    if (!ws_bytes_needed) return UBS_ERR_ARG;
    *ws_bytes_needed = need;
    return UBS_OK;
  }
  if (ws_bytes < need) return UBS_ERR_CAPACITY;
  if (pixels > 0 && (!image || !target || !d_image)) return UBS_ERR_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  SsimView* dviews = reinterpret_cast<SsimView*>(base + off_views);
  double* sums = reinterpret_cast<double*>(base + off_sums);
  float* dstat = reinterpret_cast<float*>(base + off_dstat);
  for (int first = 0; first < n_views; first += kSsimViewChunk) {
    SsimViewChunk c{};
    c.first = first;
    c.count = n_views - first < kSsimViewChunk ? n_views - first : kSsimViewChunk;
    for (int k = 0; k < c.count; ++k) c.v[k] = vs[size_t(first + k)];
    hipLaunchKernelGGL(ssim_upload_kernel, dim3(1), dim3(64), 0, st, c, dviews);
  }
  SsimTaps taps{};
  {
    double g[2 * kSsimR + 1], tot = 0.0;
    for (int k = 0; k <= 2 * kSsimR; ++k) {
      const double x = double(k - kSsimR);
      g[k] = std::exp(-x * x / (2.0 * 1.5 * 1.5));
      tot += g[k];
    }
    for (int k = 0; k <= 2 * kSsimR; ++k) taps.g[k] = float(g[k] / tot);
  }
  const double n_entries = 3.0 * double(pixels);
  if (tiles > 0) {
    const float scale = float(-double(lambda_ssim) / n_entries);
    const float l1_weight = float((1.0 - double(lambda_ssim)) / n_entries);
    hipLaunchKernelGGL(ssim_fwd_kernel, dim3(unsigned(tiles)), dim3(256), 0, st, dviews, n_views,
                       image, target, taps, scale, dstat, uint32_t(pixels), sums);
    hipLaunchKernelGGL(ssim_bwd_kernel, dim3(unsigned(tiles)), dim3(256), 0, st, dviews, n_views,
                       image, target, taps, l1_weight, dstat, uint32_t(pixels), d_image);
  }
  if (loss && tiles > 0)
    hipLaunchKernelGGL(ssim_loss_kernel, dim3(1), dim3(256), 0, st, sums, uint32_t(tiles),
                       n_entries, double(lambda_ssim), loss);
  return hipGetLastError() == hipSuccess ? UBS_OK : UBS_ERR_HIP;
}
