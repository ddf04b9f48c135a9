// Per-primitive kernels: forward preprocess (parameters -> screen-space
// records for every view of the primitive's scene) and its adjoint
// (gradients of the records, summed over views -> gradients of every
// parameter).  One lane per primitive; a lane reads its parameters once
// (component-major rows, so a wavefront's loads of one row are contiguous)
// and loops over the views of its scene.  The forward pass also copies the
// parameter rows of the primitives some view kept to a compacted copy laid
// out like the adjoint's work lists, so that the adjoint reads dense rows
// instead of gathering a fifth of every line of the parameter array.
#include "prim_math.hpp"

namespace ubs {

template <typename T, int C, int ROT>
__global__ void __launch_bounds__(256) preprocess_fwd_kernel(DevScene S, int scene,
                                                             const DevView* __restrict__ views,
                                                             int n_views, float* __restrict__ records,
                                                             LiveOut kept,
                                                             uint32_t* __restrict__ partial,
                                                             uint32_t partial_stride) {
  constexpr int F = param_rows(C, ROT).F;
  // the workgroup's parameters, kept for the copy of its kept primitives
  __shared__ float s_par[F][256];
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  const bool active = i < S.n;
  bool finite = true;
  Raw<C, ROT> r;
  Geo<T, C, ROT> g;
  if (active) {
    load_raw_rows<C, ROT>(
        [&](int k) {
          const float x = __builtin_nontemporal_load(&S.params[int64_t(k) * S.n + i]);
          s_par[k][threadIdx.x] = x;
          return x;
        },
        r);
    finite = r.finite;
    geo_forward<T, C, ROT>(r, g, S.variant);
  }
  uint32_t visible = 0;
  for (int v = 0; v < n_views; ++v) {
    const DevView& V = views[v];
    if (V.scene != scene) continue;
    if (!active) continue;
    ViewState<T, C> s;
    view_forward<T, C, ROT>(r, g, V, s);
    bool live = s.live && finite;
    float4 o0, o1, o2;
    if (live) {
      o0 = make_float4(float(s.mx), float(s.my), float(s.ca), float(s.cb));
      o1 = make_float4(float(s.cc), float(s.rho), float(s.oq), float(s.beta));
      o2 = make_float4(r.rgb[0], r.rgb[1], r.rgb[2], float(s.p[2]));
      if (!isfinite(o0.x) || !isfinite(o0.y) || !isfinite(o0.z) || !isfinite(o0.w) ||
          !isfinite(o1.x) || !isfinite(o1.y) || !isfinite(o1.z) || !isfinite(o1.w) ||
          !(o1.y > 0.0f)) {
        live = false;
      }
    }
    // a culled record is marked only: its fields are not written
    const size_t rec = size_t(V.rec_base) + size_t(i);
    kept.rec_live[rec] = live ? 1u : 0u;
    if (live) {
      ++visible;
      float4* rp = reinterpret_cast<float4*>(records + rec * kRecFloats);
      store_stream(&rp[0], o0);
      store_stream(&rp[1], o1);
      store_stream(&rp[2], o2);
    }
  }
  const bool keep = active && visible > 0;
  if (active) kept.flags[i] = keep ? 1u : 0u;
  // per-workgroup counts (no atomics on a shared word per wavefront: those
  // serialise across the chip); the binning's first kernel adds them into
  // the status block.  The kept primitives go to the adjoint's list: one
  // atomic per workgroup reserves their run (ascending inside it), and each
  // wavefront then lists its own kept primitives and copies their parameter
  // rows (from LDS) to their columns of the compacted copy.
  __shared__ uint32_t s_cnt[2], s_run;
  __shared__ unsigned long long s_keep[4];
  if (threadIdx.x == 0) { s_cnt[0] = 0; s_cnt[1] = 0; }
  __syncthreads();
  const unsigned long long nf = __ballot(active && !finite);
  const unsigned long long km = __ballot(keep);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t vis = visible;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) vis += __shfl_xor(vis, o, 64);
  if (lane == 0) {
    if (nf) atomicAdd(&s_cnt[0], uint32_t(__popcll(nf)));
    if (vis) atomicAdd(&s_cnt[1], vis);
    s_keep[wave] = km;
  }
  __syncthreads();
  const unsigned long long m0 = s_keep[0], m1 = s_keep[1], m2 = s_keep[2], m3 = s_keep[3];
  const uint32_t which = blockIdx.x % kKeptLists;
  if (threadIdx.x == 0) {
    const uint32_t n_keep = uint32_t(__popcll(m0) + __popcll(m1) + __popcll(m2) + __popcll(m3));
    partial[blockIdx.x] = s_cnt[1];
    partial[partial_stride + blockIdx.x] = s_cnt[0];
    s_run = n_keep ? atomicAdd(&kept.count[which], n_keep) : 0u;
  }
  __syncthreads();
  if (!keep) return;
  // entry q of the run: the kept primitives in thread order
  uint32_t q = uint32_t(__popcll(km & ((1ull << lane) - 1ull)));
  if (wave > 0) q += uint32_t(__popcll(m0));
  if (wave > 1) q += uint32_t(__popcll(m1));
  if (wave > 2) q += uint32_t(__popcll(m2));
  const uint32_t p = s_run + q;
  kept.list[size_t(which) * kept.cap + p] = uint32_t(i);
  kept.pos[i] = p;
  float* par = kept.par + size_t(which) * kept.cap + p;
  const int64_t par_stride = int64_t(kKeptLists) * kept.cap;
#pragma unroll
  for (int k = 0; k < F; ++k) par[k * par_stride] = s_par[k][threadIdx.x];
}

// The backward raster leaves per record the pixel sums of
//   P = sum dx s', Q = sum dy s', U = sum dx^2 s', V = sum dx dy s',
//   E = sum dy^2 s', with s' = sigma (d loss / d alpha) / (1 - r),
//   A_o = sum sigma d loss / d alpha, A_b = sum that times log2(1 - r),
// and the colour sums (dx, dy: pixel centre minus projected mean).  With
// d sigma / d r = -beta sigma / (1 - r), r = a dx^2 + 2 b dx dy + c dy^2,
// d sigma / d o = sigma / o and d sigma / d beta = sigma ln(1 - r), the
// record-field gradients are
//   d/d mx = 2 beta (a P + b Q), d/d my = 2 beta (b P + c Q),
//   d/d a = -beta U, d/d b = -2 beta V, d/d c = -beta E,
//   d/d o = A_o / o, d/d beta = ln 2 A_b
// (in place; rf: fields 2-7 of the record as the raster used it).
__device__ __forceinline__ void record_gradient_from_sums(const float* rf, float* g) {
  const float a = rf[0], b = rf[1], c = rf[2], o = rf[4], beta = rf[5];
  const float P = g[0], Q = g[1], U = g[2], V = g[3], E = g[4];
  g[0] = 2.0f * beta * (a * P + b * Q);
  g[1] = 2.0f * beta * (b * P + c * Q);
  g[2] = -beta * U;
  g[3] = -2.0f * beta * V;
  g[4] = -beta * E;
  g[5] = g[5] / o;
  g[6] = g[6] * 0.69314718f;
}

// One thread per entry of the kept lists: the adjoint of the primitive at
// entry e of list l, its parameters read from column t = l cap + e of the
// compacted copy and its gradient written to column t of the compacted
// [F][kKeptLists cap] buffer (both coalesced); scatter_dparams_kernel moves
// it to the primitive's column.
template <typename T, int C, int ROT>
__global__ void __launch_bounds__(256) preprocess_bwd_kernel(DevScene S, int scene,
                                                             const DevView* __restrict__ views,
                                                             int n_views,
                                                             const float* __restrict__ records,
                                                             float* __restrict__ grad2d,
                                                             LiveIn kept,
                                                             float* __restrict__ compact) {
  // workgroup b takes entries 256 (b / kKeptLists) + [0, 256) of kept list
  // b mod kKeptLists (cap is a multiple of 256), so the workgroups holding
  // entries come first in the grid whatever the lists' counts; thread t =
  // list cap + entry writes compacted column t
  const uint32_t lo = blockIdx.x % kKeptLists;
  const uint32_t pos = (blockIdx.x / kKeptLists) * 256u + threadIdx.x;
  const uint32_t t = lo * kept.cap + pos;
  if (pos >= kept.count[lo]) return;
  const int64_t i = kept.list[t];
  const int64_t stride = int64_t(kKeptLists) * kept.cap;
  Raw<C, ROT> r;
  // (dense rows of the compacted copy the preprocess wrote)
  load_raw<C, ROT>(kept.par, stride, t, r);
  Geo<T, C, ROT> g;
  geo_forward<T, C, ROT>(r, g, S.variant);
  GeoGrad<T, C> G;
  geograd_zero<T, C>(G);
  for (int v = 0; v < n_views; ++v) {
    const DevView& V = views[v];
    if (V.scene != scene) continue;
    const size_t rec = size_t(V.rec_base) + size_t(i);
    // the record's sums and fields are read together with its live flag
    // (every row lies inside the workspace; a culled record's are unused)
    const bool live = kept.rec_live[rec] != 0;
    const float* rp = records + rec * kRecFloats;
    float gr[kGradFloats], rf[6];
    float* gp = grad2d + rec * kGradFloats;
#pragma unroll
    for (int k = 0; k < kGradFloats; ++k) gr[k] = gp[k];
#pragma unroll
    for (int k = 0; k < 6; ++k) rf[k] = rp[2 + k];
    // (the loads stay ahead of the branch: one wait for all three)
#pragma unroll
    for (int k = 0; k < kGradFloats; ++k) asm volatile("" : "+v"(gr[k]));
#pragma unroll
    for (int k = 0; k < 6; ++k) asm volatile("" : "+v"(rf[k]));
    if (!live) continue;
    record_gradient_from_sums(rf, gr);
#pragma unroll
    for (int k = 0; k < 7; ++k) gp[k] = gr[k];
    ViewState<T, C> s;
    view_forward<T, C, ROT>(r, g, V, s);
    view_backward<T, C, ROT>(r, g, V, s, gr, G);
  }
  constexpr int F = param_rows(C, ROT).F;
  float out[F];
  geo_backward<T, C, ROT>(r, g, G, out);
#pragma unroll
  for (int k = 0; k < F; ++k) compact[int64_t(k) * stride + t] = out[k];
}

// dparams[k, i] = compact[k, j(i)] for kept primitives (j: the column of
// their kept-list entry), 0 otherwise.  VEC primitives per thread (4: one
// 16-byte store per row, for rows that start 16-byte aligned); the rows go
// in chunks whose loads are all issued before their stores, so a wavefront
// waits for memory once per chunk rather than once per row.
constexpr int kScatterChunk = 9;

template <int VEC>
__global__ void __launch_bounds__(256) scatter_dparams_kernel(DevScene S, LiveIn kept,
                                                              const float* __restrict__ compact) {
  const int64_t i0 = (int64_t(blockIdx.x) * 256 + threadIdx.x) * VEC;
  if (i0 >= S.n) return;
  const int64_t stride = int64_t(kKeptLists) * kept.cap;
  // (a primitive's list: that of its preprocess workgroup of 256; the VEC
  // primitives of a thread share it)
  const int64_t list_base = int64_t((i0 / 256) % kKeptLists) * kept.cap;
  bool live[VEC];
  int64_t j[VEC];
#pragma unroll
  for (int q = 0; q < VEC; ++q) {
    live[q] = i0 + q < S.n && kept.flags[i0 + q] != 0;
    j[q] = live[q] ? list_base + int64_t(kept.pos[i0 + q]) : 0;
  }
  for (int k0 = 0; k0 < S.F; k0 += kScatterChunk) {
    float v[kScatterChunk][VEC];
#pragma unroll
    for (int c = 0; c < kScatterChunk; ++c)
#pragma unroll
      for (int q = 0; q < VEC; ++q)
        v[c][q] = (live[q] && k0 + c < S.F) ? compact[int64_t(k0 + c) * stride + j[q]] : 0.0f;
#pragma unroll
    for (int c = 0; c < kScatterChunk; ++c) {
      if (k0 + c >= S.F) break;
      float* row = S.dparams + int64_t(k0 + c) * S.n;
      if constexpr (VEC == 4)
        store_stream(reinterpret_cast<float4*>(row + i0), make_float4(v[c][0], v[c][1], v[c][2], v[c][3]));
      else
        store_stream(row + i0, v[c][0]);
    }
  }
}

template <typename T, int C, int ROT>
static hipError_t pre_fwd_t(const DevScene& S, int scene, const DevView* views, int n_views,
                            float* records, LiveOut live, uint32_t* partial, uint32_t stride,
                            hipStream_t st) {
  const unsigned blocks = unsigned((S.n + 255) / 256);
  hipLaunchKernelGGL((preprocess_fwd_kernel<T, C, ROT>), dim3(blocks), dim3(256), 0, st, S, scene,
                     views, n_views, records, live, partial, stride);
  return hipGetLastError();
}

template <typename T, int C, int ROT>
static hipError_t pre_bwd_t(const DevScene& S, int scene, const DevView* views, int n_views,
                            const float* records, float* grad2d, LiveIn kept, float* compact,
                            hipStream_t st) {
  // one thread per entry of the kKeptLists lists of cap entries
  const unsigned blocks = unsigned(uint64_t(kKeptLists) * kept.cap / 256);
  hipLaunchKernelGGL((preprocess_bwd_kernel<T, C, ROT>), dim3(blocks), dim3(256), 0, st, S, scene,
                     views, n_views, records, grad2d, kept, compact);
  // 16-byte stores when every row of dparams starts 16-byte aligned
  if (S.n % 4 == 0 && reinterpret_cast<uintptr_t>(S.dparams) % 16 == 0)
    hipLaunchKernelGGL(scatter_dparams_kernel<4>, dim3(unsigned((S.n / 4 + 255) / 256)), dim3(256),
                       0, st, S, kept, compact);
  else
    hipLaunchKernelGGL(scatter_dparams_kernel<1>, dim3(unsigned((S.n + 255) / 256)), dim3(256), 0,
                       st, S, kept, compact);
  return hipGetLastError();
}

template <typename T>
static hipError_t pre_fwd_dispatch(const DevScene& S, int scene, const DevView* views, int n_views,
                                   float* records, LiveOut live, uint32_t* partial,
                                   uint32_t stride, hipStream_t st) {
  const int C = S.dim - 3;
  if (S.rot == UBS_ROT_QUAT) {
    if (C == 0) return pre_fwd_t<T, 0, 0>(S, scene, views, n_views, records, live, partial, stride, st);
    if (C == 3) return pre_fwd_t<T, 3, 0>(S, scene, views, n_views, records, live, partial, stride, st);
    if (C == 4) return pre_fwd_t<T, 4, 0>(S, scene, views, n_views, records, live, partial, stride, st);
    if (C == 5) return pre_fwd_t<T, 5, 0>(S, scene, views, n_views, records, live, partial, stride, st);
    if (C == 6) return pre_fwd_t<T, 6, 0>(S, scene, views, n_views, records, live, partial, stride, st);
    if (C == 7) return pre_fwd_t<T, 7, 0>(S, scene, views, n_views, records, live, partial, stride, st);
  } else {
    if (C == 0) return pre_fwd_t<T, 0, 1>(S, scene, views, n_views, records, live, partial, stride, st);
    if (C == 3) return pre_fwd_t<T, 3, 1>(S, scene, views, n_views, records, live, partial, stride, st);
    if (C == 4) return pre_fwd_t<T, 4, 1>(S, scene, views, n_views, records, live, partial, stride, st);
    if (C == 5) return pre_fwd_t<T, 5, 1>(S, scene, views, n_views, records, live, partial, stride, st);
    if (C == 6) return pre_fwd_t<T, 6, 1>(S, scene, views, n_views, records, live, partial, stride, st);
    if (C == 7) return pre_fwd_t<T, 7, 1>(S, scene, views, n_views, records, live, partial, stride, st);
  }
  return hipErrorInvalidValue;
}

template <typename T>
static hipError_t pre_bwd_dispatch(const DevScene& S, int scene, const DevView* views, int n_views,
                                   const float* records, float* grad2d, LiveIn kept,
                                   float* compact, hipStream_t st) {
  const int C = S.dim - 3;
  if (S.rot == UBS_ROT_QUAT) {
    if (C == 0) return pre_bwd_t<T, 0, 0>(S, scene, views, n_views, records, grad2d, kept, compact, st);
    if (C == 3) return pre_bwd_t<T, 3, 0>(S, scene, views, n_views, records, grad2d, kept, compact, st);
    if (C == 4) return pre_bwd_t<T, 4, 0>(S, scene, views, n_views, records, grad2d, kept, compact, st);
    if (C == 5) return pre_bwd_t<T, 5, 0>(S, scene, views, n_views, records, grad2d, kept, compact, st);
    if (C == 6) return pre_bwd_t<T, 6, 0>(S, scene, views, n_views, records, grad2d, kept, compact, st);
    if (C == 7) return pre_bwd_t<T, 7, 0>(S, scene, views, n_views, records, grad2d, kept, compact, st);
  } else {
    if (C == 0) return pre_bwd_t<T, 0, 1>(S, scene, views, n_views, records, grad2d, kept, compact, st);
    if (C == 3) return pre_bwd_t<T, 3, 1>(S, scene, views, n_views, records, grad2d, kept, compact, st);
    if (C == 4) return pre_bwd_t<T, 4, 1>(S, scene, views, n_views, records, grad2d, kept, compact, st);
    if (C == 5) return pre_bwd_t<T, 5, 1>(S, scene, views, n_views, records, grad2d, kept, compact, st);
    if (C == 6) return pre_bwd_t<T, 6, 1>(S, scene, views, n_views, records, grad2d, kept, compact, st);
    if (C == 7) return pre_bwd_t<T, 7, 1>(S, scene, views, n_views, records, grad2d, kept, compact, st);
  }
  return hipErrorInvalidValue;
}

// partial: this launch's slice of the per-workgroup counts (visible records
// at partial[b], non-finite primitives at partial[stride + b]).
hipError_t launch_preprocess_fwd(bool fp64, const DevScene& S, int scene, const DevView* views,
                                 int n_views, float* records, LiveOut live, uint32_t* partial,
                                 uint32_t stride, hipStream_t st) {
  if (S.n == 0) return hipSuccess;
  return fp64 ? pre_fwd_dispatch<double>(S, scene, views, n_views, records, live, partial, stride, st)
              : pre_fwd_dispatch<float>(S, scene, views, n_views, records, live, partial, stride, st);
}

hipError_t launch_preprocess_bwd(bool fp64, const DevScene& S, int scene, const DevView* views,
                                 int n_views, const float* records, float* grad2d, LiveIn kept,
                                 float* compact, hipStream_t st) {
  if (S.n == 0) return hipSuccess;
  return fp64 ? pre_bwd_dispatch<double>(S, scene, views, n_views, records, grad2d, kept, compact, st)
              : pre_bwd_dispatch<float>(S, scene, views, n_views, records, grad2d, kept, compact, st);
}

}  // namespace ubs
