// Relocation of dead primitives (Sec. 4.5 cloning rule with the MCMC
// primitive management the paper adopts): every primitive whose opacity is
// below o_min (or whose parameters are not finite) copies a live primitive
// picked with probability proportional to opacity, and the N copies of a
// picked primitive (itself included) share o' = 1 - (1 - o)^(1/N).
//
//   weights   per primitive: w = o if live else 0, the dead flag, o kept
//   cdf       inclusive float64 scan of w (exact: live opacities are
//             float32 values >= o_min, so every partial sum is a multiple
//             of 2^-31 below 2^22 for n < 2^22; the order of the additions
//             does not matter)
//   dead      exclusive scan of the dead flags and compaction: the dead
//             slots in index order
//   sample    slot k: first j with cdf[j] > u_k * total (float64), one
//             atomic per slot on the copy count of j
//   apply     row by row: a dead primitive takes its pick's row (or o'), a
//             picked one gets o', the moments of both are zeroed
#include <cmath>
#include <mutex>

#include "ubs_internal.hpp"

namespace ubs {

hipError_t launch_scan_compact(const uint32_t* flags, uint32_t n, uint32_t* tile_sums,
                               uint32_t* offsets, uint32_t* list, hipStream_t st,
                               unsigned long long* total_out);

constexpr int kRelThreads = 256;
constexpr int kRelItems = 16;
constexpr int kRelTile = kRelThreads * kRelItems;

struct RelocLayout {
  uint64_t cdf, o_keep, dead, offs, list, targets, counts, sums_u32, sums_f64, n_dead, bytes;
  uint32_t n_tiles;
};

constexpr uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

constexpr RelocLayout reloc_layout(int64_t n) {
  RelocLayout L{};
  const uint64_t un = uint64_t(n);
  L.n_tiles = uint32_t((un + kRelTile - 1) / kRelTile);
  uint64_t off = 0;
  L.cdf = off;      off = align256(off + 8 * un);
  L.o_keep = off;   off = align256(off + 4 * un);
  L.dead = off;     off = align256(off + 4 * un);
  L.offs = off;     off = align256(off + 4 * un);
  L.list = off;     off = align256(off + 4 * un);
  L.targets = off;  off = align256(off + 4 * un);
  L.counts = off;   off = align256(off + 4 * un);
  L.sums_u32 = off; off = align256(off + 4 * (uint64_t(L.n_tiles) + 1));
  L.sums_f64 = off; off = align256(off + 8 * (uint64_t(L.n_tiles) + 1));
  L.n_dead = off;   off = align256(off + 8);
  L.bytes = off;
  return L;
}

// Workspace of ubs_relocate_noalloc: a relocation of up to
// UBS_RELOCATE_NOALLOC_MAX_N primitives, one copy per GPU, kept for the
// life of the process.  Every word a call reads is first written by that
// call (weights, counts, scans), so nothing needs clearing between calls.
constexpr uint64_t kNoallocBytes = reloc_layout(UBS_RELOCATE_NOALLOC_MAX_N).bytes;
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

__global__ void __launch_bounds__(kRelThreads) reloc_weights_kernel(
    const float* __restrict__ params, int64_t n, int F, int o_row, float o_min,
    double* __restrict__ w, float* __restrict__ o_keep, uint32_t* __restrict__ dead,
    uint32_t* __restrict__ counts) {
  const int64_t i = int64_t(blockIdx.x) * kRelThreads + threadIdx.x;
  if (i >= n) return;
  bool finite = true;
  for (int r = 0; r < F; ++r) finite = finite && isfinite(params[int64_t(r) * n + i]);
  const float o = params[int64_t(o_row) * n + i];
  const bool live = finite && o >= o_min;
  w[i] = live ? double(o) : 0.0;
  o_keep[i] = o;
  dead[i] = live ? 0u : 1u;
  counts[i] = 0u;
}

// Inclusive float64 scan: per-tile sums, one workgroup scans them, apply.
__device__ __forceinline__ double wg_inclusive_scan_f64(double v, double* lds4, double* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const double y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) lds4[wave] = x;
  __syncthreads();
  double base = 0.0, tot = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (k < wave) base += lds4[k];
    tot += lds4[k];
  }
  __syncthreads();
  *total = tot;
  return base + x;
}

__global__ void __launch_bounds__(kRelThreads) cdf_tile_sums_kernel(const double* __restrict__ w,
                                                                    int64_t n,
                                                                    double* __restrict__ sums) {
  __shared__ double lds4[4];
  const int64_t base = int64_t(blockIdx.x) * kRelTile + int64_t(threadIdx.x) * kRelItems;
  double s = 0.0;
  for (int k = 0; k < kRelItems; ++k)
    if (base + k < n) s += w[base + k];
  double tot;
  wg_inclusive_scan_f64(s, lds4, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kRelThreads) cdf_sums_scan_kernel(double* __restrict__ sums,
                                                                    uint32_t n_tiles) {
  __shared__ double lds4[4];
  double carry = 0.0;
  for (uint32_t b = 0; b < n_tiles; b += kRelThreads) {
    const uint32_t i = b + threadIdx.x;
    const double v = i < n_tiles ? sums[i] : 0.0;
    double tot;
    const double incl = wg_inclusive_scan_f64(v, lds4, &tot);
    if (i < n_tiles) sums[i] = carry + incl - v;   // exclusive
    carry += tot;
  }
}

__global__ void __launch_bounds__(kRelThreads) cdf_apply_kernel(double* __restrict__ w, int64_t n,
                                                                const double* __restrict__ sums) {
  __shared__ double lds4[4];
  const int64_t base = int64_t(blockIdx.x) * kRelTile + int64_t(threadIdx.x) * kRelItems;
  double vals[kRelItems];
  double s = 0.0;
  for (int k = 0; k < kRelItems; ++k) {
    vals[k] = base + k < n ? w[base + k] : 0.0;
    s += vals[k];
  }
  double tot;
  double run = sums[blockIdx.x] + wg_inclusive_scan_f64(s, lds4, &tot) - s;
  for (int k = 0; k < kRelItems; ++k) {
    run += vals[k];
    if (base + k < n) w[base + k] = run;
  }
}

// First index j with cdf[j] > x (strict) or >= x, cdf non-decreasing; n if none.
template <bool STRICT>
__device__ __forceinline__ int64_t first_index(const double* __restrict__ cdf, int64_t n, double x) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = lo + ((hi - lo) >> 1);
    const bool past = STRICT ? cdf[mid] > x : cdf[mid] >= x;
    if (past) hi = mid; else lo = mid + 1;
  }
  return lo;
}

// Dead slot k picks the first j with cdf[j] > u_k * total; when the product
// rounds to the total itself (u within an ulp of 1) there is none, and the
// pick is the last live primitive (the first j with cdf[j] >= total).
__global__ void __launch_bounds__(kRelThreads) reloc_sample_kernel(
    const double* __restrict__ cdf, int64_t n, const unsigned long long* __restrict__ n_dead,
    const double* __restrict__ uniforms, uint32_t* __restrict__ targets,
    uint32_t* __restrict__ counts, uint32_t* __restrict__ targets_out) {
  const int64_t k = int64_t(blockIdx.x) * kRelThreads + threadIdx.x;
  const double total = cdf[n - 1];
  if (k >= int64_t(*n_dead) || !(total > 0.0)) return;
  int64_t j = first_index<true>(cdf, n, uniforms[k] * total);
  if (j >= n) j = first_index<false>(cdf, n, total);
  targets[k] = uint32_t(j);
  if (targets_out) targets_out[k] = uint32_t(j);
  atomicAdd(&counts[j], 1u);
}

__global__ void copy_count_kernel(const unsigned long long* __restrict__ src,
                                  uint64_t* __restrict__ dst) {
  if (threadIdx.x == 0) *dst = *src;
}

// One (row, primitive) pair per thread, rows along blockIdx.y, so that the
// accesses of a wavefront to one row are consecutive: a dead primitive i
// takes row r of its pick j = targets[offs[i]] (or the cloned opacity), a
// picked primitive gets the cloned opacity, and both have their moments
// zeroed.  Picks are never dead, so no thread reads what another writes.
__global__ void __launch_bounds__(kRelThreads) reloc_apply_kernel(
    float* __restrict__ params, float* __restrict__ m, float* __restrict__ v, int64_t n,
    int o_row, const double* __restrict__ cdf, const float* __restrict__ o_keep,
    const uint32_t* __restrict__ dead, const uint32_t* __restrict__ offs,
    const uint32_t* __restrict__ targets, const uint32_t* __restrict__ counts) {
  const int64_t i = int64_t(blockIdx.x) * kRelThreads + threadIdx.x;
  if (i >= n || !(cdf[n - 1] > 0.0)) return;
  const int r = blockIdx.y;
  const int64_t row = int64_t(r) * n;
  if (dead[i]) {
    const int64_t j = targets[offs[i]];
    float val;
    if (r == o_row)
      val = float(1.0 - pow(1.0 - double(o_keep[j]), 1.0 / (double(counts[j]) + 1.0)));
    else
      val = params[row + j];
    store_stream(params + row + i, val);
    store_stream(m + row + i, 0.0f);
    store_stream(v + row + i, 0.0f);
  } else if (counts[i] > 0u) {
    if (r == o_row)
      params[row + i] = float(1.0 - pow(1.0 - double(o_keep[i]), 1.0 / (double(counts[i]) + 1.0)));
    store_stream(m + row + i, 0.0f);
    store_stream(v + row + i, 0.0f);
  }
}

// Device address of `scratch` on the current device, looked up once per
// device (each GPU holds its own copy of the array at its own address).
static ubs_status noalloc_scratch(char** out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* ptr[kMaxDevices] = {};
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return UBS_ERR_HIP;
  if (dev < 0 || dev >= kMaxDevices) return UBS_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return UBS_ERR_HIP;
    ptr[dev] = p;
  }
  *out = static_cast<char*>(ptr[dev]);
  return UBS_OK;
}

static ubs_status relocate_args(int32_t dim, int32_t rot, int64_t n, float o_min) {
  if (dim < 3 || dim > kMaxDim || (rot != UBS_ROT_QUAT && rot != UBS_ROT_SKEW) || n < 0)
    return UBS_ERR_ARG;
  if (!dim_ok(dim)) return UBS_ERR_UNSUPPORTED;
  if (n > (int64_t(1) << 31) - 1) return UBS_ERR_UNSUPPORTED;
  if (!(o_min >= 0.0f)) return UBS_ERR_ARG;
  return UBS_OK;
}

// The relocation's launches over a workspace at `base` laid out by L.
static ubs_status relocate_run(int32_t dim, int32_t rot, int64_t n, float* params, float* m,
                               float* v, const double* uniforms, float o_min, char* base,
                               const RelocLayout& L, uint32_t* targets_out,
                               uint64_t* n_dead_out, void* stream) {
  const ParamRows pr = param_rows(dim - 3, rot);
  hipStream_t st = static_cast<hipStream_t>(stream);
  double* cdf = reinterpret_cast<double*>(base + L.cdf);
  float* o_keep = reinterpret_cast<float*>(base + L.o_keep);
  uint32_t* dead = reinterpret_cast<uint32_t*>(base + L.dead);
  uint32_t* offs = reinterpret_cast<uint32_t*>(base + L.offs);
  uint32_t* list = reinterpret_cast<uint32_t*>(base + L.list);
  uint32_t* targets = reinterpret_cast<uint32_t*>(base + L.targets);
  uint32_t* counts = reinterpret_cast<uint32_t*>(base + L.counts);
  double* sums = reinterpret_cast<double*>(base + L.sums_f64);
  unsigned long long* n_dead = reinterpret_cast<unsigned long long*>(base + L.n_dead);
  const unsigned blocks = unsigned((n + kRelThreads - 1) / kRelThreads);
  hipLaunchKernelGGL(reloc_weights_kernel, dim3(blocks), dim3(kRelThreads), 0, st, params, n,
                     pr.F, pr.o, o_min, cdf, o_keep, dead, counts);
  hipLaunchKernelGGL(cdf_tile_sums_kernel, dim3(L.n_tiles), dim3(kRelThreads), 0, st, cdf, n, sums);
  hipLaunchKernelGGL(cdf_sums_scan_kernel, dim3(1), dim3(kRelThreads), 0, st, sums, L.n_tiles);
  hipLaunchKernelGGL(cdf_apply_kernel, dim3(L.n_tiles), dim3(kRelThreads), 0, st, cdf, n, sums);
  if (launch_scan_compact(dead, uint32_t(n), reinterpret_cast<uint32_t*>(base + L.sums_u32), offs,
                          list, st, n_dead) != hipSuccess)
    return UBS_ERR_HIP;
  hipLaunchKernelGGL(reloc_sample_kernel, dim3(blocks), dim3(kRelThreads), 0, st, cdf, n, n_dead,
                     uniforms, targets, counts, targets_out);
  hipLaunchKernelGGL(reloc_apply_kernel, dim3(blocks, unsigned(pr.F)), dim3(kRelThreads), 0, st,
                     params, m, v, n, pr.o, cdf, o_keep, dead, offs, targets, counts);
  if (n_dead_out)
    hipLaunchKernelGGL(copy_count_kernel, dim3(1), dim3(64), 0, st, n_dead, n_dead_out);
  return hipGetLastError() == hipSuccess ? UBS_OK : UBS_ERR_HIP;
}

}  // namespace ubs

using namespace ubs;

extern "C" ubs_status ubs_relocate(int32_t dim, int32_t rot, int64_t n, float* params, float* m,
                                   float* v, const double* uniforms, float o_min, void* ws,
                                   uint64_t ws_bytes, uint64_t* ws_bytes_needed,
                                   uint32_t* targets_out, uint64_t* n_dead_out, void* stream) {
  const ubs_status a = relocate_args(dim, rot, n, o_min);
  if (a != UBS_OK) return a;
  const RelocLayout L = reloc_layout(n);
  if (!ws) {
    if (!ws_bytes_needed) return UBS_ERR_ARG;
    *ws_bytes_needed = L.bytes;
    return UBS_OK;
  }
  if (ws_bytes < L.bytes) return UBS_ERR_CAPACITY;
  if (n == 0) return UBS_OK;
  if (!params || !m || !v || !uniforms) return UBS_ERR_ARG;
  return relocate_run(dim, rot, n, params, m, v, uniforms, o_min, static_cast<char*>(ws), L,
                      targets_out, n_dead_out, stream);
}

extern "C" ubs_status ubs_relocate_noalloc(int32_t dim, int32_t rot, int64_t n, float* params,
                                           float* m, float* v, const double* uniforms,
                                           float o_min, uint32_t* targets_out,
                                           uint64_t* n_dead_out, void* stream) {
  const ubs_status a = relocate_args(dim, rot, n, o_min);
  if (a != UBS_OK) return a;
  if (n > UBS_RELOCATE_NOALLOC_MAX_N) return UBS_ERR_CAPACITY;
  if (n == 0) return UBS_OK;
  if (!params || !m || !v || !uniforms) return UBS_ERR_ARG;
  char* base = nullptr;
  const ubs_status sc = noalloc_scratch(&base);
  if (sc != UBS_OK) return sc;
  return relocate_run(dim, rot, n, params, m, v, uniforms, o_min, base, reloc_layout(n),
                      targets_out, n_dead_out, stream);
}
