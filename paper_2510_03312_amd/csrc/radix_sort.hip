// Device-wide LSD radix sort of (uint64 key, uint32 value) pairs.
//
// Structure (one read of the keys for the histograms, one kernel per digit):
//  1. radix_hist_all_kernel counts the digits of every pass at once into a
//     global histogram [pass][digit].
//  2. radix_onesweep_kernel<BITS>, one launch per pass: each workgroup takes
//     the next tile of 2048 keys (dynamic tile id from an atomic counter, so
//     a tile's predecessors were all taken by workgroups already running),
//     ranks its keys stably, publishes the tile's per-digit counts, then
//     walks back over the preceding tiles' published counts until it meets
//     an inclusive prefix (decoupled look-back), publishes its own inclusive
//     prefix and scatters.  Every workgroup publishes its counts before it
//     waits on anyone, so waits always end; the wait is also bounded and
//     sets an error flag instead of spinning forever.
// The element count is read from the status block on the device: no host
// synchronisation, safe to capture in a graph.
//
// Stable ranking inside a tile: each wave takes 64 consecutive keys per step;
// lanes with equal digits are found with one ballot per digit bit, a lane's
// rank is the popcount of equal-digit lanes below it, and a per-wave LDS
// counter carries the running count across steps.
#include "ubs_internal.hpp"

namespace ubs {

constexpr uint32_t kFlagAgg = 1u << 30;   // published: the tile's own count
constexpr uint32_t kFlagIncl = 2u << 30;  // published: count of this and all earlier tiles
constexpr uint32_t kValMask = (1u << 30) - 1u;
constexpr uint32_t kSpinLimit = 1u << 20;

__device__ __forceinline__ unsigned long long sort_count(const DevStatus* __restrict__ status) {
  return status->overflow ? 0ull : status->pairs_needed;
}

// Exclusive scan over the 256 threads of a workgroup (4 waves).
__device__ __forceinline__ uint32_t block_exclusive_scan256(uint32_t v, uint32_t* lds4) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) lds4[wave] = x;
  __syncthreads();
  uint32_t wb = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) wb += w < wave ? lds4[w] : 0u;
  return wb + x - v;
}

__global__ void __launch_bounds__(kSortThreads) radix_hist_all_kernel(
    const unsigned long long* __restrict__ keys, const DevStatus* __restrict__ status,
    int key_bits, int digit_bits, SortState* __restrict__ state) {
  __shared__ uint32_t cnt[kSortPassMax * 256];
  const int n_pass = (key_bits + digit_bits - 1) / digit_bits;
  for (int d = threadIdx.x; d < n_pass * 256; d += kSortThreads) cnt[d] = 0;
  __syncthreads();
  const unsigned long long K = sort_count(status);
  const unsigned mask = (1u << digit_bits) - 1u;
  for (unsigned long long i = (unsigned long long)blockIdx.x * kSortThreads + threadIdx.x; i < K;
       i += (unsigned long long)gridDim.x * kSortThreads) {
    const unsigned long long k = keys[i];
    for (int p = 0; p < n_pass; ++p)
      atomicAdd(&cnt[p * 256 + (uint32_t(k >> (p * digit_bits)) & mask)], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < n_pass * 256; d += kSortThreads)
    if (cnt[d]) atomicAdd(&state->hist[d], cnt[d]);
}

template <int BITS>
__global__ void __launch_bounds__(kSortThreads) radix_onesweep_kernel(
    const unsigned long long* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
    unsigned long long* __restrict__ keys_out, uint32_t* __restrict__ vals_out,
    DevStatus* __restrict__ status, int pass, int shift, SortState* __restrict__ state,
    uint32_t* __restrict__ lookback, uint32_t max_tiles) {
  constexpr int R = 1 << BITS;
  constexpr int kWaves = kSortThreads / 64;
  static_assert(R <= kSortThreads, "one thread per digit");
  __shared__ uint32_t wcnt[kWaves][R];
  __shared__ uint32_t gbase[R];
  __shared__ uint32_t s_tile;
  __shared__ uint32_t s_scan[4];
  const unsigned long long K = sort_count(status);
  if (threadIdx.x == 0) s_tile = atomicAdd(&state->tile_counter[pass], 1u);
  for (int d = threadIdx.x; d < kWaves * R; d += kSortThreads) (&wcnt[0][0])[d] = 0;
  __syncthreads();
  const uint32_t tile = s_tile;
  const unsigned long long base = (unsigned long long)tile * kSortTile;
  if (base >= K) return;   // uniform per workgroup; no later tile waits on it
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
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
  uint32_t* pass_lb = lookback + size_t(pass) * max_tiles * 256;
  const int d = threadIdx.x;   // one thread per digit
  uint32_t excl = 0;
  if (d < R) {
    // the tile's count of digit d; waves' exclusive offsets inside the tile
    uint32_t total = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      const uint32_t c = wcnt[w][d];
      wcnt[w][d] = total;
      total += c;
    }
    uint32_t* my_lb = pass_lb + size_t(tile) * 256 + d;
    __hip_atomic_store(my_lb, kFlagAgg | total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // look back over earlier tiles until an inclusive prefix
    bool stalled = false;
    for (int64_t j = int64_t(tile) - 1; j >= 0 && !stalled; --j) {
      const uint32_t* lb = pass_lb + size_t(j) * 256 + d;
      uint32_t v = __hip_atomic_load(lb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      uint32_t spins = 0;
      while ((v & ~kValMask) == 0u) {
        if (++spins > kSpinLimit) {
          stalled = true;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
        v = __hip_atomic_load(lb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      if (stalled) break;
      excl += v & kValMask;
      if ((v & ~kValMask) == kFlagIncl) break;
    }
    if (stalled) atomicOr(&status->sort_stalled, 1u);
    __hip_atomic_store(my_lb, kFlagIncl | (excl + total), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
  // global offset of digit d: all smaller digits of this pass, then earlier tiles
  const uint32_t hd = d < R ? state->hist[pass * 256 + d] : 0u;
  const uint32_t below_d = block_exclusive_scan256(hd, s_scan);
  if (d < R) gbase[d] = below_d + excl;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    if (dig[j] != 0xFFFFFFFFu) {
      const uint32_t pos = gbase[dig[j]] + wcnt[wave][dig[j]] + rank[j];
      keys_out[pos] = key[j];
      vals_out[pos] = val[j];
    }
  }
}

// Clears the sort state and, for each pass, the look-back words of the tiles
// the sort will use (a prefix whose length follows from the device-side
// element count).
__global__ void __launch_bounds__(256) radix_prepare_kernel(const DevStatus* __restrict__ status,
                                                            SortState* __restrict__ state,
                                                            uint32_t* __restrict__ lookback,
                                                            int n_pass, uint32_t max_tiles) {
  const unsigned long long K = sort_count(status);
  const size_t n_tiles = size_t((K + kSortTile - 1) / kSortTile);
  const size_t words = n_tiles * 256;
  const size_t i0 = size_t(blockIdx.x) * 256 + threadIdx.x;
  const size_t stride = size_t(gridDim.x) * 256;
  for (int p = 0; p < n_pass; ++p) {
    uint32_t* lb = lookback + size_t(p) * max_tiles * 256;
    for (size_t i = i0; i < words; i += stride) lb[i] = 0u;
  }
  if (blockIdx.x == 0) {
    uint32_t* s = reinterpret_cast<uint32_t*>(state);
    for (size_t i = threadIdx.x; i < sizeof(SortState) / 4; i += 256) s[i] = 0u;
  }
}

template <int BITS>
static hipError_t onesweep_pass(const unsigned long long* kin, const uint32_t* vin,
                                unsigned long long* kout, uint32_t* vout, DevStatus* status,
                                int pass, int shift, SortState* state, uint32_t* lookback,
                                uint32_t n_blocks, hipStream_t st) {
  hipLaunchKernelGGL(radix_onesweep_kernel<BITS>, dim3(n_blocks), dim3(kSortThreads), 0, st, kin,
                     vin, kout, vout, status, pass, shift, state, lookback, n_blocks);
  return hipGetLastError();
}

// Sorts bits [0, key_bits) with digit_bits-wide digits, ping-ponging between
// buffer 0 (input) and buffer 1.  After an odd number of passes the result
// is in buffer 1.  n_blocks = tiles of the capacity.
hipError_t launch_radix_sort(unsigned long long* k0, uint32_t* v0, unsigned long long* k1,
                             uint32_t* v1, DevStatus* status, int key_bits, int digit_bits,
                             SortState* state, uint32_t* lookback, uint32_t n_blocks,
                             hipStream_t st) {
  if (n_blocks == 0) return hipSuccess;
  const int n_pass = (key_bits + digit_bits - 1) / digit_bits;
  if (n_pass > kSortPassMax) return hipErrorInvalidValue;
  unsigned prep = n_blocks;
  if (prep > 1024u) prep = 1024u;
  hipLaunchKernelGGL(radix_prepare_kernel, dim3(prep), dim3(256), 0, st, status, state, lookback,
                     n_pass, n_blocks);
  unsigned hist_blocks = n_blocks < 512u ? n_blocks : 512u;
  hipLaunchKernelGGL(radix_hist_all_kernel, dim3(hist_blocks), dim3(kSortThreads), 0, st, k0,
                     status, key_bits, digit_bits, state);
  unsigned long long* kin = k0;
  uint32_t* vin = v0;
  unsigned long long* kout = k1;
  uint32_t* vout = v1;
  int pass = 0;
  for (int shift = 0; shift < key_bits; shift += digit_bits, ++pass) {
    const int bits = (key_bits - shift) < digit_bits ? (key_bits - shift) : digit_bits;
    hipError_t e;
    switch (bits) {
      case 1: e = onesweep_pass<1>(kin, vin, kout, vout, status, pass, shift, state, lookback, n_blocks, st); break;
      case 2: e = onesweep_pass<2>(kin, vin, kout, vout, status, pass, shift, state, lookback, n_blocks, st); break;
      case 3: e = onesweep_pass<3>(kin, vin, kout, vout, status, pass, shift, state, lookback, n_blocks, st); break;
      case 4: e = onesweep_pass<4>(kin, vin, kout, vout, status, pass, shift, state, lookback, n_blocks, st); break;
      case 5: e = onesweep_pass<5>(kin, vin, kout, vout, status, pass, shift, state, lookback, n_blocks, st); break;
      case 6: e = onesweep_pass<6>(kin, vin, kout, vout, status, pass, shift, state, lookback, n_blocks, st); break;
      case 7: e = onesweep_pass<7>(kin, vin, kout, vout, status, pass, shift, state, lookback, n_blocks, st); break;
      default: e = onesweep_pass<8>(kin, vin, kout, vout, status, pass, shift, state, lookback, n_blocks, st); break;
    }
    if (e != hipSuccess) return e;
    unsigned long long* tk = kin; kin = kout; kout = tk;
    uint32_t* tv = vin; vin = vout; vout = tv;
  }
  return hipSuccess;
}

}  // namespace ubs
