// Device-wide LSD radix sort of (uint64 key, uint32 value) pairs.
//
// One pass per digit: (1) per-block digit histograms, (2) exclusive scan of
// the digit-major histogram matrix, (3) stable scatter.  The element count
// is read from the status block on the device (so the passes need no host
// synchronisation and can be captured in a graph); blocks past the count
// contribute empty histograms.
//
// Stable ranking inside a block: each wave takes 64 consecutive keys per
// step; lanes with equal digits are found with one ballot per digit bit, a
// lane's rank is the popcount of equal-digit lanes below it, and a per-wave
// LDS counter carries the running count across steps.  Ranks therefore
// follow the input order, which makes every pass stable.
#include "ubs_internal.hpp"

namespace ubs {

hipError_t launch_scan(const uint32_t* in, uint32_t n, uint32_t* tile_sums, uint32_t* out,
                       DevStatus* status, unsigned long long capacity, hipStream_t st);

__device__ __forceinline__ unsigned long long sort_count(const DevStatus* __restrict__ status) {
  return status->overflow ? 0ull : status->pairs_needed;
}

template <int BITS>
__global__ void __launch_bounds__(kSortThreads) radix_hist_kernel(
    const unsigned long long* __restrict__ keys, const DevStatus* __restrict__ status, int shift,
    uint32_t* __restrict__ hist, uint32_t n_blocks) {
  constexpr int R = 1 << BITS;
  __shared__ uint32_t cnt[R];
  for (int d = threadIdx.x; d < R; d += kSortThreads) cnt[d] = 0;
  __syncthreads();
  const unsigned long long K = sort_count(status);
  const unsigned long long base = (unsigned long long)blockIdx.x * kSortTile;
  if (base < K) {
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
      const unsigned long long idx = base + (unsigned long long)j * kSortThreads + threadIdx.x;
      if (idx < K) {
        const uint32_t d = uint32_t(keys[idx] >> shift) & (R - 1);
        atomicAdd(&cnt[d], 1u);
      }
    }
  }
  __syncthreads();
  for (int d = threadIdx.x; d < R; d += kSortThreads) hist[size_t(d) * n_blocks + blockIdx.x] = cnt[d];
}

template <int BITS>
__global__ void __launch_bounds__(kSortThreads) radix_scatter_kernel(
    const unsigned long long* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
    unsigned long long* __restrict__ keys_out, uint32_t* __restrict__ vals_out,
    const DevStatus* __restrict__ status, int shift, const uint32_t* __restrict__ hist_scan,
    uint32_t n_blocks) {
  constexpr int R = 1 << BITS;
  constexpr int kWaves = kSortThreads / 64;
  __shared__ uint32_t wcnt[kWaves][R];
  __shared__ uint32_t gbase[R];
  const unsigned long long K = sort_count(status);
  const unsigned long long base = (unsigned long long)blockIdx.x * kSortTile;
  if (base >= K) return;   // uniform per block
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int d = threadIdx.x; d < kWaves * R; d += kSortThreads) (&wcnt[0][0])[d] = 0;
  for (int d = threadIdx.x; d < R; d += kSortThreads) gbase[d] = hist_scan[size_t(d) * n_blocks + blockIdx.x];
  __syncthreads();
  const unsigned long long lt_mask = (1ull << lane) - 1ull;
  unsigned long long key[kSortItems];
  uint32_t val[kSortItems];
  uint32_t rank[kSortItems];
  uint32_t dig[kSortItems];
  const unsigned long long wbase = base + (unsigned long long)wave * (64 * kSortItems);
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const unsigned long long idx = wbase + (unsigned long long)j * 64 + lane;
    const bool valid = idx < K;
    key[j] = valid ? keys_in[idx] : 0ull;
    val[j] = valid ? vals_in[idx] : 0u;
    const uint32_t d = uint32_t(key[j] >> shift) & (R - 1);
    dig[j] = valid ? d : 0xFFFFFFFFu;
    unsigned long long m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
      const bool bit = (d >> b) & 1u;
      const unsigned long long bb = __ballot(bit);
      m &= bit ? bb : ~bb;
    }
    rank[j] = 0;
    if (valid) {
      const uint32_t below = __popcll(m & lt_mask);
      rank[j] = wcnt[wave][d] + below;
      // the lowest lane of each equal-digit group advances the wave counter
      if (below == 0) wcnt[wave][d] += uint32_t(__popcll(m));
    }
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  // per-digit exclusive offsets across the waves of the block
  for (int d = threadIdx.x; d < R; d += kSortThreads) {
    uint32_t run = gbase[d];
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      const uint32_t c = wcnt[w][d];
      wcnt[w][d] = run;
      run += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    if (dig[j] != 0xFFFFFFFFu) {
      const uint32_t pos = wcnt[wave][dig[j]] + rank[j];
      keys_out[pos] = key[j];
      vals_out[pos] = val[j];
    }
  }
}

template <int BITS>
static hipError_t sort_pass(const unsigned long long* kin, const uint32_t* vin,
                            unsigned long long* kout, uint32_t* vout, const DevStatus* status,
                            int shift, uint32_t* hist, uint32_t* tile_sums, uint32_t n_blocks,
                            hipStream_t st) {
  constexpr int R = 1 << BITS;
  hipLaunchKernelGGL(radix_hist_kernel<BITS>, dim3(n_blocks), dim3(kSortThreads), 0, st, kin,
                     status, shift, hist, n_blocks);
  hipError_t e = launch_scan(hist, uint32_t(R) * n_blocks, tile_sums, hist, nullptr, 0ull, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(radix_scatter_kernel<BITS>, dim3(n_blocks), dim3(kSortThreads), 0, st, kin,
                     vin, kout, vout, status, shift, hist, n_blocks);
  return hipGetLastError();
}

// Sorts bits [0, key_bits) with digit_bits-wide digits, ping-ponging between
// buffer 0 (input) and buffer 1.  After an odd number of passes the result
// is in buffer 1.
hipError_t launch_radix_sort(unsigned long long* k0, uint32_t* v0, unsigned long long* k1,
                             uint32_t* v1, const DevStatus* status, int key_bits, int digit_bits,
                             uint32_t* hist, uint32_t* tile_sums, uint32_t n_blocks,
                             hipStream_t st) {
  if (n_blocks == 0) return hipSuccess;
  unsigned long long* kin = k0;
  uint32_t* vin = v0;
  unsigned long long* kout = k1;
  uint32_t* vout = v1;
  for (int shift = 0; shift < key_bits; shift += digit_bits) {
    const int bits = (key_bits - shift) < digit_bits ? (key_bits - shift) : digit_bits;
    hipError_t e;
    switch (bits) {
      case 1: e = sort_pass<1>(kin, vin, kout, vout, status, shift, hist, tile_sums, n_blocks, st); break;
      case 2: e = sort_pass<2>(kin, vin, kout, vout, status, shift, hist, tile_sums, n_blocks, st); break;
      case 3: e = sort_pass<3>(kin, vin, kout, vout, status, shift, hist, tile_sums, n_blocks, st); break;
      case 4: e = sort_pass<4>(kin, vin, kout, vout, status, shift, hist, tile_sums, n_blocks, st); break;
      case 5: e = sort_pass<5>(kin, vin, kout, vout, status, shift, hist, tile_sums, n_blocks, st); break;
      case 6: e = sort_pass<6>(kin, vin, kout, vout, status, shift, hist, tile_sums, n_blocks, st); break;
      case 7: e = sort_pass<7>(kin, vin, kout, vout, status, shift, hist, tile_sums, n_blocks, st); break;
      default: e = sort_pass<8>(kin, vin, kout, vout, status, shift, hist, tile_sums, n_blocks, st); break;
    }
    if (e != hipSuccess) return e;
    unsigned long long* tk = kin; kin = kout; kout = tk;
    uint32_t* tv = vin; vin = vout; vout = tv;
  }
  return hipSuccess;
}

}  // namespace ubs
