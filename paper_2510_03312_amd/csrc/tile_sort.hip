// Per-tile ordering of the (tile, record) pairs.
//
// Binning counts the pairs of every tile (one atomic per pair) and stores
// the 64-bit key (depth bits << 32 | record) of each in the tile's block of
// tuning.tile_slots slots, in no particular order; an exclusive scan of the counts
// gives every tile a contiguous segment of the output.  If some tile has
// more pairs than slots (the spill flag), a second binning pass appends
// every key to its tile's segment of `comp` through a per-tile cursor
// instead, and the sort reads from there.  The key is unique within a tile
// (a record meets a tile at most once), so sorting a tile's keys yields
// exactly the order of a stable sort of (tile, depth) keys emitted in record
// order: depth first, equal depths in record order.
//
// tile_sort_small_kernel: one wavefront per tile (grid-stride over tiles);
//   writes every tile's range and sorts the tiles of at most kSmallSort
//   pairs by rank (each key's position is the number of smaller keys in the
//   tile, LDS broadcast reads); larger tiles go to a list for
// tile_sort_kernel: one workgroup per listed tile.
//   n <= kLdsSortMax  bitonic sort in LDS, padded to a power of two;
//   larger            LSD radix sort of the segment in global memory by the
//                     workgroup alone (each wavefront owns a contiguous
//                     quarter, so the scatter is stable without barriers),
//                     ping-ponging with the segment's slice of the output
//                     key buffer; digits that are constant over the segment
//                     are skipped.
// It also writes the tile's [start, end) range ((0, 0) for an empty tile and
// for every tile after an overflow).
#include "ubs_internal.hpp"

namespace ubs {

constexpr int kTileSortThreads = 256;
constexpr int kLdsSortMax = 4096;   // keys held in LDS (32 KiB)
constexpr uint32_t kSmallSort = 256;
static_assert(kSmallSort == 256, "the rank sort counts for up to four 64-key slots");
static_assert(kMaxTileSlots <= uint32_t(kLdsSortMax),
              "a slot block always fits the LDS sort: the radix sort runs after a spill only");

__device__ __forceinline__ void write_sorted(unsigned long long key, uint32_t tile, size_t pos,
                                             unsigned long long* __restrict__ keys_out,
                                             uint32_t* __restrict__ vals_out) {
  keys_out[pos] = ((unsigned long long)tile << 32) | (key >> 32);
  vals_out[pos] = uint32_t(key);
}

// Exclusive scan over 256 threads (4 waves); lds4 holds 4 words.
__device__ __forceinline__ uint32_t wg_exclusive_scan(uint32_t v, uint32_t* lds4) {
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
  __syncthreads();
  return wb + x - v;
}

// LSD radix sort of seg[0, n) by one workgroup, using alt[0, n) as the second
// buffer.  Sorts the bits [0, rec_bits) and [32, 64).  Returns the buffer
// holding the result.
__device__ unsigned long long* wg_radix_sort(unsigned long long* seg, unsigned long long* alt,
                                             uint32_t n, int digit_bits, int rec_bits,
                                             uint32_t (*hist)[256], uint32_t* lds4,
                                             uint32_t* s_flag) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned long long lt_mask = (1ull << lane) - 1ull;
  const uint32_t R = 1u << digit_bits, mask = R - 1u;
  const uint32_t quarter = (n + 3u) / 4u;
  const uint32_t q0 = min(n, uint32_t(wave) * quarter), q1 = min(n, q0 + quarter);
  unsigned long long* src = seg;
  unsigned long long* dst = alt;
  for (int shift = 0; shift < 64; shift += digit_bits) {
    if (shift >= rec_bits && shift + digit_bits <= 32) continue;   // always zero
    for (uint32_t d = threadIdx.x; d < 4u * 256u; d += kTileSortThreads) (&hist[0][0])[d] = 0u;
    if (threadIdx.x == 0) *s_flag = 0u;
    __syncthreads();
    for (uint32_t i = q0 + lane; i < q1; i += 64)
      atomicAdd(&hist[wave][uint32_t(src[i] >> shift) & mask], 1u);
    __syncthreads();
    const uint32_t d = threadIdx.x;
    uint32_t c[4] = {0u, 0u, 0u, 0u}, tot = 0u;
    if (d < R) {
#pragma unroll
      for (int w = 0; w < 4; ++w) { c[w] = hist[w][d]; tot += c[w]; }
      if (tot == n) *s_flag = 1u;   // one digit value only: the pass is the identity
    }
    const uint32_t excl = wg_exclusive_scan(d < R ? tot : 0u, lds4);
    if (d < R) {
      uint32_t run = excl;
#pragma unroll
      for (int w = 0; w < 4; ++w) { hist[w][d] = run; run += c[w]; }
    }
    __syncthreads();
    const bool identity = *s_flag != 0u;
    __syncthreads();   // every thread has read the flag before the next pass resets it
    if (identity) continue;
    // stable scatter of the wave's quarter, 64 keys at a time
    for (uint32_t b = q0; b < q1; b += 64) {
      const uint32_t i = b + lane;
      const bool valid = i < q1;
      const unsigned long long k = valid ? src[i] : 0ull;
      const uint32_t dg = uint32_t(k >> shift) & mask;
      unsigned long long m = __ballot(valid);
      for (int bit = 0; bit < digit_bits; ++bit) {
        const bool on = (dg >> bit) & 1u;
        const unsigned long long bb = __ballot(on);
        m &= on ? bb : ~bb;
      }
      if (valid) {
        const uint32_t below = uint32_t(__popcll(m & lt_mask));
        dst[hist[wave][dg] + below] = k;
        if (below == 0) hist[wave][dg] += uint32_t(__popcll(m));
      }
      __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    unsigned long long* t = src; src = dst; dst = t;
  }
  return src;
}

// rank[q] += number of keys in s_keys[0, n) below k[q], for the first NQ slots
template <int NQ>
__device__ __forceinline__ void count_smaller(const unsigned long long* s_keys, uint32_t n,
                                              const unsigned long long* k, uint32_t* rank) {
  for (uint32_t j = 0; j < n; ++j) {
    const unsigned long long kj = s_keys[j];
#pragma unroll
    for (int q = 0; q < NQ; ++q) rank[q] += kj < k[q] ? 1u : 0u;
  }
}

__global__ void __launch_bounds__(64) tile_sort_small_kernel(
    const unsigned long long* __restrict__ comp, const unsigned long long* __restrict__ slots,
    uint32_t slot_cap, const uint32_t* __restrict__ tile_counts,
    const uint32_t* __restrict__ tile_cursor, const DevStatus* __restrict__ status,
    unsigned long long* __restrict__ keys_out, uint32_t* __restrict__ vals_out,
    uint32_t* __restrict__ ranges, uint32_t n_tiles, const uint32_t* __restrict__ order,
    uint32_t* __restrict__ big_tiles, uint32_t* __restrict__ n_big_tiles) {
  __shared__ unsigned long long s_keys[kSmallSort];
  constexpr int Q = int(kSmallSort / 64);
  const uint32_t lane = threadIdx.x;
  const bool overflow = status->overflow != 0u;
  const bool spill = status->spill != 0u;
  for (uint32_t q = blockIdx.x; q < n_tiles; q += gridDim.x) {
    const uint32_t t = order[q];   // (longest tiles first)
    const uint32_t n = overflow ? 0u : tile_counts[t];
    // the cursor is the segment start, or its end once the spill pass ran
    const uint32_t start = n ? (spill ? tile_cursor[t] - n : tile_cursor[t]) : 0u;
    const uint32_t end = start + n;   // an empty tile's range is (0, 0)
    const unsigned long long* src = spill ? comp + start : slots + size_t(t) * slot_cap;
    if (lane == 0) {
      ranges[2 * size_t(t)] = start;
      ranges[2 * size_t(t) + 1] = end;
    }
    if (n == 0) continue;
    if (n > kSmallSort) {
      if (lane == 0) big_tiles[atomicAdd(n_big_tiles, 1u)] = t;
      continue;
    }
    unsigned long long k[Q];
    uint32_t rank[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const uint32_t i = lane + 64u * uint32_t(q);
      k[q] = i < n ? src[i] : ~0ull;
      if (i < n) s_keys[i] = k[q];
      rank[q] = 0u;
    }
    __syncthreads();
    // only the slots holding keys count (n <= 64 * nq)
    switch ((n + 63u) / 64u) {
      case 1: count_smaller<1>(s_keys, n, k, rank); break;
      case 2: count_smaller<2>(s_keys, n, k, rank); break;
      case 3: count_smaller<3>(s_keys, n, k, rank); break;
      default: count_smaller<4>(s_keys, n, k, rank); break;
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const uint32_t i = lane + 64u * uint32_t(q);
      if (i < n) write_sorted(k[q], t, size_t(start) + rank[q], keys_out, vals_out);
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kTileSortThreads) tile_sort_kernel(
    unsigned long long* __restrict__ comp, const unsigned long long* __restrict__ slots,
    uint32_t slot_cap, const uint32_t* __restrict__ tile_counts,
    const uint32_t* __restrict__ tile_cursor, const DevStatus* __restrict__ status,
    const uint32_t* __restrict__ big_tiles, const uint32_t* __restrict__ n_big_tiles,
    unsigned long long* __restrict__ keys_out, uint32_t* __restrict__ vals_out, int digit_bits,
    int rec_bits) {
  __shared__ unsigned long long s_keys[kLdsSortMax];
  __shared__ uint32_t s_hist[4][256];
  __shared__ uint32_t s_lds4[4];
  __shared__ uint32_t s_flag;
  const uint32_t n_big = *n_big_tiles;
  const bool spill = status->spill != 0u;
  for (uint32_t bt = blockIdx.x; bt < n_big; bt += gridDim.x) {
    const uint32_t t = big_tiles[bt];
    const uint32_t n = tile_counts[t];
    // the cursor is the segment start, or its end once the spill pass ran;
    // without a spill the keys are in the tile's slot block (n <= slot_cap)
    const uint32_t start = spill ? tile_cursor[t] - n : tile_cursor[t];
    const unsigned long long* src = spill ? comp + start : slots + size_t(t) * slot_cap;
    if (n <= uint32_t(kLdsSortMax)) {
      uint32_t P = 512;
      while (P < n) P <<= 1;
      for (uint32_t i = threadIdx.x; i < P; i += kTileSortThreads)
        s_keys[i] = i < n ? src[i] : ~0ull;
      __syncthreads();
      for (uint32_t k = 2; k <= P; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
          for (uint32_t i = threadIdx.x; i < P / 2; i += kTileSortThreads) {
            const uint32_t lo = 2 * i - (i & (j - 1));
            const uint32_t hi = lo + j;
            const unsigned long long a = s_keys[lo], b = s_keys[hi];
            const bool up = (lo & k) == 0;
            if ((a > b) == up) {
              s_keys[lo] = b;
              s_keys[hi] = a;
            }
          }
          __syncthreads();
        }
      }
      for (uint32_t i = threadIdx.x; i < n; i += kTileSortThreads)
        write_sorted(s_keys[i], t, size_t(start) + i, keys_out, vals_out);
      __syncthreads();
    } else {
      // the segment's slice of the output key buffer is the second buffer
      unsigned long long* res = wg_radix_sort(comp + start, keys_out + start, n, digit_bits,
                                              rec_bits, s_hist, s_lds4, &s_flag);
      for (uint32_t i = threadIdx.x; i < n; i += kTileSortThreads) {
        const unsigned long long k = res[i];   // read before the same thread overwrites slot i
        write_sorted(k, t, size_t(start) + i, keys_out, vals_out);
      }
      __syncthreads();
    }
  }
}

// big_tiles: n_tiles words; n_big_tiles must be zero; order: the tiles
// longest first (the scan's order).
hipError_t launch_tile_sort(unsigned long long* comp, const unsigned long long* slots,
                            uint32_t slot_cap, const uint32_t* tile_counts,
                            const uint32_t* tile_cursor,
                            const DevStatus* status, unsigned long long* keys_out,
                            uint32_t* vals_out, uint32_t* ranges, uint32_t n_tiles,
                            int digit_bits, int rec_bits, uint32_t* big_tiles,
                            uint32_t* n_big_tiles, const uint32_t* order, hipStream_t st) {
  if (n_tiles == 0) return hipSuccess;
  const uint32_t grid = n_tiles < 65536u ? n_tiles : 65536u;
  hipLaunchKernelGGL(tile_sort_small_kernel, dim3(grid), dim3(64), 0, st, comp, slots,
                     slot_cap, tile_counts, tile_cursor, status, keys_out, vals_out, ranges,
                     n_tiles, order, big_tiles, n_big_tiles);
  // up to four workgroups per CU (the LDS sort takes 37 KiB of the 160)
  const uint32_t big_grid = n_tiles < 1024u ? n_tiles : 1024u;
  hipLaunchKernelGGL(tile_sort_kernel, dim3(big_grid), dim3(kTileSortThreads), 0, st, comp,
                     slots, slot_cap, tile_counts, tile_cursor, status, big_tiles, n_big_tiles,
                     keys_out, vals_out, digit_bits, rec_bits);
  return hipGetLastError();
}

}  // namespace ubs
