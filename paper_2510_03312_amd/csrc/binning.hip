// Tile binning: per-tile pair counts, with every (tile, record) key stored
// in the tile's block of slots (tuning.tile_slots) in the same pass; for a
// frame where some tile outgrows its block, a second pass emits every pair
// into its tile's segment (the segments come from an exclusive scan of the
// counts).  The order inside a tile is fixed afterwards by tile_sort.hip.
//
// A record overlaps a tile iff the minimum of its quadratic form
// r(p) = a dx^2 + 2 b dx dy + c dy^2 over the rectangle spanned by the
// tile's pixel centres (clipped to the image) is at most rho (1 + 2^-10).
// The test is evaluated in float64, round-to-nearest, with no contraction
// and in a fixed operation order, so that the decision is reproducible
// bit for bit by any IEEE-754 implementation of the same expression.
#include "tile_box.hpp"
#include "ubs_internal.hpp"

namespace ubs {

#pragma clang fp contract(off)
__device__ __noinline__ bool tile_overlap_exact(double mx, double my, double a, double b, double c,
                                                double rho, double x0, double x1, double y0,
                                                double y1) {
  const double rb = rho * (1.0 + 0x1p-10);
  if (mx >= x0 && mx <= x1 && my >= y0 && my <= y1) return true;
  const double det = a * c - b * b;
  const double dy0 = y0 - my, dy1 = y1 - my;
  const double dx0 = x0 - mx, dx1 = x1 - mx;
  // vertical edges: dx fixed, minimiser dy* = -b dx / c clamped to [dy0, dy1]
  for (int e = 0; e < 2; ++e) {
    const double dx = e == 0 ? dx0 : dx1;
    const double t = -(b * dx);
    const double lo = c * dy0, hi = c * dy1;
    if (t >= lo && t <= hi) {
      if ((det * dx) * dx <= rb * c) return true;
    } else {
      const double dy = (t < lo) ? dy0 : dy1;
      const double q = ((a * dx) * dx + ((2.0 * b) * dx) * dy) + (c * dy) * dy;
      if (q <= rb) return true;
    }
  }
  // horizontal edges: dy fixed, minimiser dx* = -b dy / a clamped to [dx0, dx1]
  for (int e = 0; e < 2; ++e) {
    const double dy = e == 0 ? dy0 : dy1;
    const double t = -(b * dy);
    const double lo = a * dx0, hi = a * dx1;
    if (t >= lo && t <= hi) {
      if ((det * dy) * dy <= rb * a) return true;
    } else {
      const double dx = (t < lo) ? dx0 : dx1;
      const double q = ((a * dx) * dx + ((2.0 * b) * dx) * dy) + (c * dy) * dy;
      if (q <= rb) return true;
    }
  }
  return false;
}
#pragma clang fp contract(on)

// View of a record: views are laid out with ascending rec_base.
__device__ __forceinline__ int view_of_record(const DevView* __restrict__ views, int n_views,
                                              uint32_t rec) {
  int lo = 0, hi = n_views - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (views[mid].rec_base <= rec) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Conservative tile box of {r <= rho (1 + 2^-10)} (tile_box.hpp).
__device__ __forceinline__ TileBox record_tile_box(const float4 r0, const float4 r1,
                                                   const DevView& V) {
  return tile_box_of(r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, V.W, V.H, V.tile_w, V.tile_h);
}

__device__ __forceinline__ bool record_hits_tile(const float4 r0, const float4 r1, const DevView& V,
                                                 int tx, int ty) {
  const int px0 = tx * V.tile_w, py0 = ty * V.tile_h;
  const int px1 = min(px0 + V.tile_w - 1, V.W - 1), py1 = min(py0 + V.tile_h - 1, V.H - 1);
  return tile_overlap_exact(double(r0.x), double(r0.y), double(r0.z), double(r0.w), double(r1.x),
                            double(r1.y), double(px0) + 0.5, double(px1) + 0.5, double(py0) + 0.5,
                            double(py1) + 0.5);
}

// Records whose conservative tile box holds at most kSmallBox candidate tiles
// go through their wavefront's flat candidate list, their hits kept as one
// bit per candidate; larger ones are binned by their whole workgroup.
constexpr int kSmallBox = 32;
static_assert(kSmallBox <= 32, "hit masks are 32 bits");

struct BinRec {
  float4 r0, r1;
  float depth;
  int view;
  TileBox box;
  int n_cand;
};

__device__ __forceinline__ int bcast_i(int v, int src) { return __builtin_amdgcn_readlane(v, src); }
__device__ __forceinline__ float bcast_f(float v, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}

__device__ __forceinline__ BinRec bcast_rec(const BinRec& b, int src) {
  BinRec o;
  o.r0 = make_float4(bcast_f(b.r0.x, src), bcast_f(b.r0.y, src), bcast_f(b.r0.z, src), bcast_f(b.r0.w, src));
  o.r1 = make_float4(bcast_f(b.r1.x, src), bcast_f(b.r1.y, src), bcast_f(b.r1.z, src), bcast_f(b.r1.w, src));
  o.depth = bcast_f(b.depth, src);
  o.view = bcast_i(b.view, src);
  o.box.tx0 = bcast_i(b.box.tx0, src);
  o.box.tx1 = bcast_i(b.box.tx1, src);
  o.box.ty0 = bcast_i(b.box.ty0, src);
  o.box.ty1 = bcast_i(b.box.ty1, src);
  o.n_cand = bcast_i(b.n_cand, src);
  return o;
}

__device__ __forceinline__ BinRec load_bin_rec(const float* __restrict__ records,
                                               const DevView* __restrict__ views, int n_views,
                                               uint32_t rec, bool active) {
  BinRec b;
  b.r0 = make_float4(0.f, 0.f, 0.f, 0.f);
  b.r1 = b.r0;
  b.depth = 0.f;
  b.view = 0;
  b.box = TileBox{1, 0, 1, 0};
  b.n_cand = 0;
  if (active) {
    const float4* rp = reinterpret_cast<const float4*>(records + size_t(rec) * kRecFloats);
    b.r0 = rp[0];
    b.r1 = rp[1];
    b.depth = records[size_t(rec) * kRecFloats + 11];
    b.view = view_of_record(views, n_views, rec);
    b.box = record_tile_box(b.r0, b.r1, views[b.view]);
    if (b.box.tx0 <= b.box.tx1 && b.box.ty0 <= b.box.ty1)
      b.n_cand = (b.box.tx1 - b.box.tx0 + 1) * (b.box.ty1 - b.box.ty0 + 1);
  }
  return b;
}

__device__ __forceinline__ uint32_t global_tile(const DevView& V, int tx, int ty) {
  return V.tile_base + uint32_t(ty * V.tiles_x + tx);
}

// Each wavefront takes RPW consecutive records and first packs the indices
// of the live ones (live flag set) into a per-wave LDS list, so that its
// lanes then work only on live records (after culling, typically a fifth of
// them).  The counting pass takes RPW = 64 for frames of up to
// kBinSmallFrame records (more, smaller wavefronts hide more of the counting
// atomics' latency: 42.1 -> 39.0 us at 1M records) and 256 beyond (there the
// many nearly empty wavefronts of 64 records cost more: 8M records 0.30 ->
// 0.36 ms); the spill pass always 256.
constexpr int kBinRecPerWave = 256;
constexpr int kBinRecPerWaveSmall = 64;
constexpr uint32_t kBinSmallFrame = 1u << 21;
constexpr int kBinWaves = 4;   // 256-thread workgroups

template <int RPW>
__device__ __forceinline__ uint32_t gather_live(const uint8_t* __restrict__ live,
                                                uint32_t n_records, uint32_t* __restrict__ list) {
  const int lane = threadIdx.x & 63;
  const uint32_t wave_global = blockIdx.x * kBinWaves + (threadIdx.x >> 6);
  const uint32_t base = wave_global * RPW;
  const unsigned long long lt_mask = (1ull << lane) - 1ull;
  uint32_t cnt = 0;
#pragma unroll
  for (int m = 0; m < RPW / 64; ++m) {
    const uint32_t rec = base + uint32_t(m * 64 + lane);
    const bool vis = rec < n_records && live[rec] != 0;
    const unsigned long long mask = __ballot(vis);
    if (vis) list[cnt + uint32_t(__popcll(mask & lt_mask))] = rec;
    cnt += uint32_t(__popcll(mask));
  }
  __builtin_amdgcn_wave_barrier();
  return cnt;
}

// Position of flat index f in a wavefront's work list: the last slot j whose
// exclusive prefix excl[j] is <= f (slots holding no work share their
// successor's prefix, so the last such slot is the one f belongs to).
__device__ __forceinline__ int owner_slot(const uint32_t* excl, uint32_t f) {
  int j = 0;
#pragma unroll
  for (int step = 32; step > 0; step >>= 1)
    if (excl[j + step] <= f) j += step;
  return j;
}

// Inclusive sum over the 64 lanes of a wavefront.
__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(v, o, 64);
    if (lane >= o) v += y;
  }
  return v;
}

// Counts one pair of `tile` and stores its key in the tile's block of `cap`
// slots while the block has room; the first pair beyond it raises the spill
// flag.
__device__ __forceinline__ void store_slot(uint32_t tile, unsigned long long key,
                                           uint32_t* __restrict__ tile_counts,
                                           unsigned long long* __restrict__ slots, uint32_t cap,
                                           DevStatus* __restrict__ status) {
  const uint32_t slot = atomicAdd(&tile_counts[tile], 1u);
  if (slot < cap)
    slots[size_t(tile) * cap + slot] = key;
  else if (slot == cap)
    status->spill = 1u;
}

// One atomic increment of tile_counts per (tile, record) pair, the key
// stored in the tile's slot block.  Records with at most kSmallBox candidate
// tiles are binned 64 at a time by the whole wavefront: their candidates form
// one flat list (record order, row-major candidates) that the lanes take in
// turns, so a wavefront runs as many rounds of tile tests as it has
// candidates / 64 rather than as its largest record has candidates.  The
// hits of each record (bit k: candidate k) are kept as a mask for the spill
// pass.  Larger records are binned at the end by the whole workgroup, one at
// a time, and appended to big_list for the spill pass.
template <int RPW>
__global__ void __launch_bounds__(256) bin_count_kernel(const float* __restrict__ records,
                                                        const uint8_t* __restrict__ live,
                                                        const DevView* __restrict__ views,
                                                        int n_views, uint32_t n_records,
                                                        uint32_t* __restrict__ tile_counts,
                                                        uint32_t* __restrict__ hit_mask,
                                                        uint32_t* __restrict__ big_list,
                                                        uint32_t* __restrict__ big_count,
                                                        unsigned long long* __restrict__ slots,
                                                        uint32_t slot_cap,
                                                        DevStatus* __restrict__ status,
                                                        float* __restrict__ grad2d) {
  __shared__ uint32_t s_list[kBinWaves][RPW];
  __shared__ uint32_t s_excl[kBinWaves][65];
  __shared__ unsigned long long s_key[kBinWaves][64];
  __shared__ float4 s_r0[kBinWaves][64];
  __shared__ float2 s_r1[kBinWaves][64];
  __shared__ int4 s_box[kBinWaves][64];     // tx0, ty0, box width, view
  __shared__ uint32_t s_mask[kBinWaves][64];
  __shared__ uint32_t s_big[kBinWaves * RPW];   // the workgroup's big records
  __shared__ uint32_t s_nbig;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const unsigned long long lt_mask = (1ull << lane) - 1ull;
  if (threadIdx.x == 0) s_nbig = 0u;
  __syncthreads();
  uint32_t* list = s_list[w];
  const uint32_t cnt = gather_live<RPW>(live, n_records, list);
  for (uint32_t c0 = 0; c0 < cnt; c0 += 64) {
    const bool active = c0 + lane < cnt;
    const uint32_t rec = active ? list[c0 + lane] : 0u;
    // the backward raster accumulates into the gradient rows of exactly
    // these records: they start at zero (the rows of culled records are
    // never read)
    if (active) {
      float2* gp = reinterpret_cast<float2*>(grad2d + size_t(rec) * kGradFloats);
#pragma unroll
      for (int q = 0; q < kGradFloats / 2; ++q) gp[q] = make_float2(0.0f, 0.0f);
    }
    const BinRec b = load_bin_rec(records, views, n_views, rec, active);
    const bool small = b.n_cand > 0 && b.n_cand <= kSmallBox;
    const uint32_t nc = small ? uint32_t(b.n_cand) : 0u;
    const uint32_t incl = wave_inclusive_sum(nc);
    const uint32_t total = uint32_t(__shfl(int(incl), 63, 64));
    s_excl[w][lane] = incl - nc;
    if (lane == 0) s_excl[w][64] = 0xffffffffu;
    s_key[w][lane] = ((unsigned long long)__float_as_uint(b.depth) << 32) | rec;
    s_r0[w][lane] = b.r0;
    s_r1[w][lane] = make_float2(b.r1.x, b.r1.y);
    s_box[w][lane] = make_int4(b.box.tx0, b.box.ty0, b.box.tx1 - b.box.tx0 + 1, b.view);
    s_mask[w][lane] = 0u;
    __builtin_amdgcn_wave_barrier();
    for (uint32_t f = lane; f < total; f += 64) {
      const int j = owner_slot(s_excl[w], f);
      const int k = int(f - s_excl[w][j]);
      const int4 bx = s_box[w][j];
      const DevView& V = views[bx.w];
      const int tx = bx.x + k % bx.z, ty = bx.y + k / bx.z;
      const float2 r1 = s_r1[w][j];
      if (record_hits_tile(s_r0[w][j], make_float4(r1.x, r1.y, 0.f, 0.f), V, tx, ty)) {
        store_slot(global_tile(V, tx, ty), s_key[w][j], tile_counts, slots, slot_cap, status);
        atomicOr(&s_mask[w][j], 1u << k);
      }
    }
    __builtin_amdgcn_wave_barrier();
    if (small) hit_mask[rec] = s_mask[w][lane];
    const bool big = b.n_cand > kSmallBox;
    const unsigned long long bm = __ballot(big);
    if (bm) {
      // listed for the workgroup below, and globally for the spill pass
      uint32_t base = 0, lbase = 0;
      if (lane == 0) {
        base = atomicAdd(big_count, uint32_t(__popcll(bm)));
        lbase = atomicAdd(&s_nbig, uint32_t(__popcll(bm)));
      }
      base = uint32_t(__shfl(int(base), 0, 64));
      lbase = uint32_t(__shfl(int(lbase), 0, 64));
      const uint32_t below = uint32_t(__popcll(bm & lt_mask));
      if (big) {
        big_list[base + below] = rec;
        s_big[lbase + below] = rec;
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
  // the records with more than kSmallBox candidates: the whole workgroup
  // tests the candidates of one at a time
  __syncthreads();
  const uint32_t nb = s_nbig;
  for (uint32_t bi = 0; bi < nb; ++bi) {
    const uint32_t rec = s_big[bi];
    const BinRec o = load_bin_rec(records, views, n_views, rec, true);
    const DevView& V = views[o.view];
    const int bw = o.box.tx1 - o.box.tx0 + 1;
    const unsigned long long key = ((unsigned long long)__float_as_uint(o.depth) << 32) | rec;
    for (int k = int(threadIdx.x); k < o.n_cand; k += 256) {
      const int tx = o.box.tx0 + k % bw, ty = o.box.ty0 + k / bw;
      if (record_hits_tile(o.r0, o.r1, V, tx, ty))
        store_slot(global_tile(V, tx, ty), key, tile_counts, slots, slot_cap, status);
    }
  }
}

// Spill pass, records with more than kSmallBox candidate tiles: a workgroup
// per record (grid-stride over big_list; workgroup `block` of `n_blocks`
// takes records block, block + n_blocks, ...), its threads testing
// consecutive candidates and appending the hits to the tile segments.
__device__ __forceinline__ void emit_big_records(uint32_t block, uint32_t n_blocks,
                                                 const float* __restrict__ records,
                                                 const DevView* __restrict__ views, int n_views,
                                                 const uint32_t* __restrict__ big_list,
                                                 const uint32_t* __restrict__ big_count,
                                                 uint32_t* __restrict__ tile_cursor,
                                                 unsigned long long* __restrict__ comp) {
  const uint32_t nb = *big_count;
  for (uint32_t bi = block; bi < nb; bi += n_blocks) {
    const uint32_t rec = big_list[bi];
    const BinRec o = load_bin_rec(records, views, n_views, rec, true);
    const DevView& V = views[o.view];
    const int bw = o.box.tx1 - o.box.tx0 + 1;
    const unsigned long long key = ((unsigned long long)__float_as_uint(o.depth) << 32) | rec;
    for (int k = int(threadIdx.x); k < o.n_cand; k += 256) {
      const int tx = o.box.tx0 + k % bw, ty = o.box.ty0 + k / bw;
      if (record_hits_tile(o.r0, o.r1, V, tx, ty))
        comp[atomicAdd(&tile_cursor[global_tile(V, tx, ty)], 1u)] = key;
    }
  }
}

// Spill pass: appends (depth bits << 32 | record) of every pair to its
// tile's segment.  The first n_small_blocks workgroups replay bin_count's hit
// masks of the records with at most kSmallBox candidates as one flat list of
// hits per 64 records (one round of independent cursor atomics per 64 hits);
// the others test the big records' candidates again.  tile_cursor starts at
// each segment's first slot and ends one past its last.  Without a spill
// every workgroup returns at once.
__global__ void __launch_bounds__(256) bin_emit_kernel(const float* __restrict__ records,
                                                       const uint8_t* __restrict__ live,
                                                       const DevView* __restrict__ views,
                                                       int n_views, uint32_t n_records,
                                                       const uint32_t* __restrict__ hit_mask,
                                                       const uint32_t* __restrict__ big_list,
                                                       const uint32_t* __restrict__ big_count,
                                                       uint32_t n_small_blocks,
                                                       uint32_t* __restrict__ tile_cursor,
                                                       DevStatus* __restrict__ status,
                                                       unsigned long long* __restrict__ comp) {
  if (status->overflow || !status->spill) return;
  if (blockIdx.x >= n_small_blocks) {
    emit_big_records(blockIdx.x - n_small_blocks, gridDim.x - n_small_blocks, records, views,
                     n_views, big_list, big_count, tile_cursor, comp);
    return;
  }
  __shared__ uint32_t s_list[kBinWaves][kBinRecPerWave];
  __shared__ uint32_t s_excl[kBinWaves][65];
  __shared__ unsigned long long s_key[kBinWaves][64];
  __shared__ int4 s_box[kBinWaves][64];     // tx0, ty0, box width, view
  __shared__ uint32_t s_bits[kBinWaves][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t* list = s_list[w];
  const uint32_t cnt = gather_live<kBinRecPerWave>(live, n_records, list);
  for (uint32_t c0 = 0; c0 < cnt; c0 += 64) {
    const bool active = c0 + lane < cnt;
    const uint32_t rec = active ? list[c0 + lane] : 0u;
    const BinRec b = load_bin_rec(records, views, n_views, rec, active);
    const bool small = b.n_cand > 0 && b.n_cand <= kSmallBox;
    const uint32_t bits = small ? hit_mask[rec] : 0u;
    const uint32_t nh = uint32_t(__popc(bits));
    const uint32_t incl = wave_inclusive_sum(nh);
    const uint32_t total = uint32_t(__shfl(int(incl), 63, 64));
    s_excl[w][lane] = incl - nh;
    if (lane == 0) s_excl[w][64] = 0xffffffffu;
    s_key[w][lane] = ((unsigned long long)__float_as_uint(b.depth) << 32) | rec;
    s_box[w][lane] = make_int4(b.box.tx0, b.box.ty0, b.box.tx1 - b.box.tx0 + 1, b.view);
    s_bits[w][lane] = bits;
    __builtin_amdgcn_wave_barrier();
    for (uint32_t f = lane; f < total; f += 64) {
      const int j = owner_slot(s_excl[w], f);
      uint32_t m = f - s_excl[w][j];
      uint32_t bb = s_bits[w][j];
      while (m--) bb &= bb - 1u;           // drop the hits before the m-th
      const int k = __ffs(int(bb)) - 1;
      const int4 bx = s_box[w][j];
      const DevView& V = views[bx.w];
      const int tx = bx.x + k % bx.z, ty = bx.y + k / bx.z;
      comp[atomicAdd(&tile_cursor[global_tile(V, tx, ty)], 1u)] = s_key[w][j];
    }
    __builtin_amdgcn_wave_barrier();
  }
}


// ---------------------------------------------------------------------------
// Exclusive scan of uint32 counts (three phases: tile sums, scan of the tile
// sums in one block, tile-local scan plus the tile's base).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t block_exclusive_scan_u32(uint32_t v, uint32_t* lds,
                                                             uint32_t* total) {
  // 256 threads = 4 waves of 64
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) lds[wave] = x;
  __syncthreads();
  uint32_t wbase = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    uint32_t s = lds[w];
    if (w < wave) wbase += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return wbase + x - v;
}

// Sum over the 256 threads of a workgroup in 64 bits (a count total must not
// wrap: it decides the overflow flag).
__device__ __forceinline__ unsigned long long block_sum_u64(unsigned long long v,
                                                            unsigned long long* lds4) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) lds4[threadIdx.x >> 6] = v;
  __syncthreads();
  const unsigned long long t = lds4[0] + lds4[1] + lds4[2] + lds4[3];
  __syncthreads();
  return t;
}

// Per-block totals, saturated at 2^32 - 1 (a saturated total makes the
// grand total exceed any capacity, so the overflow flag is still raised).
__global__ void __launch_bounds__(kScanThreads) scan_tile_sums_kernel(
    const uint32_t* __restrict__ in, uint32_t n, uint32_t* __restrict__ tile_sums) {
  __shared__ unsigned long long lds4[4];
  const size_t base = size_t(blockIdx.x) * kScanTile + size_t(threadIdx.x) * kScanItems;
  unsigned long long s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < n) s += in[base + k];
  const unsigned long long tot = block_sum_u64(s, lds4);
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = tot > 0xffffffffull ? 0xffffffffu : uint32_t(tot);
}

// One block scans all tile sums in place (exclusive) and writes the total
// (and, for the pair scan, the overflow flag of the status block).
__global__ void __launch_bounds__(kScanThreads) scan_tile_sums_scan_kernel(
    uint32_t* __restrict__ tile_sums, uint32_t n_tiles, DevStatus* __restrict__ status,
    unsigned long long capacity, unsigned long long* __restrict__ total_out) {
  __shared__ uint32_t lds[8];
  unsigned long long carry = 0;
  for (uint32_t base = 0; base < n_tiles; base += kScanThreads) {
    const uint32_t i = base + threadIdx.x;
    const uint32_t v = i < n_tiles ? tile_sums[i] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan_u32(v, lds, &tot);
    if (i < n_tiles) tile_sums[i] = uint32_t(carry + ex);
    carry += tot;
  }
  if (threadIdx.x == 0 && status != nullptr) {
    status->pairs_needed = carry;
    status->overflow = carry > capacity ? 1u : 0u;
  }
  if (threadIdx.x == 0 && total_out != nullptr) *total_out = carry;
}

// With `list` (0/1 inputs only), also the compaction: list[out[i]] = i for
// every set in[i].
__global__ void __launch_bounds__(kScanThreads) scan_apply_kernel(
    const uint32_t* __restrict__ in, uint32_t n, const uint32_t* __restrict__ tile_sums,
    uint32_t* __restrict__ out, uint32_t* __restrict__ list) {
  __shared__ uint32_t lds[8];
  const size_t base = size_t(blockIdx.x) * kScanTile + size_t(threadIdx.x) * kScanItems;
  uint32_t vals[kScanItems];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    vals[k] = base + k < n ? in[base + k] : 0u;
    s += vals[k];
  }
  uint32_t tot;
  uint32_t run = block_exclusive_scan_u32(s, lds, &tot) + tile_sums[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) {
      out[base + k] = run;
      if (list != nullptr && vals[k] != 0u) list[run] = uint32_t(base + k);
    }
    run += vals[k];
  }
}

__global__ void fill_u32_kernel(uint32_t* __restrict__ p, size_t n, uint32_t v) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t k = i; k < n; k += stride) p[k] = v;
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static unsigned bin_blocks(uint32_t n_records, uint32_t rpw = kBinRecPerWave) {
  const uint32_t per_block = uint32_t(kBinWaves) * rpw;
  return unsigned((uint64_t(n_records) + per_block - 1) / per_block);
}

constexpr unsigned kBigBlocks = 1024;

// tile_counts and *big_count must be zero.
hipError_t launch_bin_count(const float* records, const uint8_t* live, const DevView* views,
                            int n_views,
                            uint32_t n_records, uint32_t* tile_counts, uint32_t* hit_mask,
                            uint32_t* big_list, uint32_t* big_count, unsigned long long* slots,
                            uint32_t slot_cap, DevStatus* status, float* grad2d, hipStream_t st) {
  if (n_records == 0) return hipSuccess;
  if (n_records <= kBinSmallFrame)
    hipLaunchKernelGGL(bin_count_kernel<kBinRecPerWaveSmall>,
                       dim3(bin_blocks(n_records, kBinRecPerWaveSmall)), dim3(256), 0, st, records,
                       live, views, n_views, n_records, tile_counts, hit_mask, big_list, big_count,
                       slots, slot_cap, status, grad2d);
  else
    hipLaunchKernelGGL(bin_count_kernel<kBinRecPerWave>, dim3(bin_blocks(n_records)), dim3(256),
                       0, st, records, live, views, n_views, n_records, tile_counts, hit_mask,
                       big_list, big_count, slots, slot_cap, status, grad2d);
  return hipGetLastError();
}

// Exclusive scan of up to kSingleScanMax values by one workgroup of 1024
// threads, 8192 values per step with a running carry (one launch instead of
// three); same outputs as the three-kernel scan.
constexpr uint32_t kSingleScanMax = 16u * kScanTile;
constexpr int kSingleThreads = 1024;

// Order in which the rasters take the tiles: by pair count, largest first
// (ties in no particular order), so that the last tiles a launch hands out
// are small ones and the SIMDs finish together.  A counting sort of the
// tiles on min(count, kOrderBins - 1), here by one workgroup of kOrderBins
// threads for up to kOrderBins * kOrderPer tiles (each tile's rank in its
// bin kept from its counting atomic).
constexpr int kOrderBins = 1024;
constexpr int kOrderPer = 8;

__device__ __forceinline__ uint32_t order_bin(uint32_t count) {
  // ascending bins put the longest tiles first
  return uint32_t(kOrderBins - 1) - min(count, uint32_t(kOrderBins - 1));
}

__device__ __forceinline__ void order_tiles_by_count(const uint32_t* __restrict__ counts,
                                                     uint32_t n, uint32_t* __restrict__ order,
                                                     uint32_t* bins, uint32_t* wave_tot) {
  const uint32_t tid = threadIdx.x;
  uint32_t b[kOrderPer], rank[kOrderPer];
  bins[tid] = 0u;
  __syncthreads();
  {
    uint32_t c[kOrderPer];
#pragma unroll
    for (int q = 0; q < kOrderPer; ++q) {
      const uint32_t t = uint32_t(q) * kOrderBins + tid;
      c[q] = t < n ? counts[t] : 0u;
    }
#pragma unroll
    for (int q = 0; q < kOrderPer; ++q) {
      b[q] = order_bin(c[q]);
      rank[q] = uint32_t(q) * kOrderBins + tid < n ? atomicAdd(&bins[b[q]], 1u) : 0u;
    }
  }
  __syncthreads();
  // exclusive scan of the bins: within wavefronts, then over their totals
  const int lane = int(tid & 63), wave = int(tid >> 6);
  const uint32_t c = bins[tid];
  uint32_t x = c;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wave_tot[wave] = x;
  __syncthreads();
  uint32_t wbase = 0;
  for (int w = 0; w < wave; ++w) wbase += wave_tot[w];
  bins[tid] = wbase + x - c;
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kOrderPer; ++q) {
    const uint32_t t = uint32_t(q) * kOrderBins + tid;
    if (t < n) order[bins[b[q]] + rank[q]] = t;
  }
}

constexpr uint32_t kOrderOneRound = uint32_t(kOrderBins * kOrderPer);

// Frames of more than kOrderOneRound tiles: the same counting sort by
// workgroups of kOrderGroupTiles tiles (bin counts per workgroup, one
// workgroup turning them into each workgroup's offsets bin by bin, then the
// scatter), so that no one workgroup walks every tile.
constexpr uint32_t kOrderGroupTiles = 2048;   // 256 threads x 8

__global__ void __launch_bounds__(256) tile_order_hist_kernel(const uint32_t* __restrict__ counts,
                                                              uint32_t n,
                                                              uint32_t* __restrict__ hist) {
  __shared__ uint32_t bins[kOrderBins];
  for (int i = int(threadIdx.x); i < kOrderBins; i += 256) bins[i] = 0u;
  __syncthreads();
  const uint32_t t0 = blockIdx.x * kOrderGroupTiles + threadIdx.x;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const uint32_t t = t0 + uint32_t(q) * 256u;
    if (t < n) atomicAdd(&bins[order_bin(counts[t])], 1u);
  }
  __syncthreads();
  for (int i = int(threadIdx.x); i < kOrderBins; i += 256)
    hist[size_t(blockIdx.x) * kOrderBins + i] = bins[i];
}

// hist[g][b] becomes the position of workgroup g's first tile of bin b:
// bins in ascending order, workgroups in order within a bin.
__global__ void __launch_bounds__(kOrderBins) tile_order_offsets_kernel(uint32_t* __restrict__ hist,
                                                                        uint32_t groups) {
  __shared__ uint32_t wave_tot[kOrderBins / 64];
  const uint32_t b = threadIdx.x;
  uint32_t c = 0;
  // (eight workgroups' counts loaded at a time)
  for (uint32_t g0 = 0; g0 < groups; g0 += 8) {
    uint32_t h[8];
#pragma unroll
    for (int q = 0; q < 8; ++q)
      h[q] = g0 + q < groups ? hist[size_t(g0 + q) * kOrderBins + b] : 0u;
#pragma unroll
    for (int q = 0; q < 8; ++q) c += h[q];
  }
  const int lane = int(b & 63), wave = int(b >> 6);
  uint32_t x = c;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wave_tot[wave] = x;
  __syncthreads();
  uint32_t run = x - c;
  for (int w = 0; w < wave; ++w) run += wave_tot[w];
  for (uint32_t g0 = 0; g0 < groups; g0 += 8) {
    uint32_t h[8];
#pragma unroll
    for (int q = 0; q < 8; ++q)
      h[q] = g0 + q < groups ? hist[size_t(g0 + q) * kOrderBins + b] : 0u;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (g0 + q < groups) hist[size_t(g0 + q) * kOrderBins + b] = run;
      run += h[q];
    }
  }
}

__global__ void __launch_bounds__(256) tile_order_scatter_kernel(const uint32_t* __restrict__ counts,
                                                                 uint32_t n,
                                                                 const uint32_t* __restrict__ hist,
                                                                 uint32_t* __restrict__ order) {
  __shared__ uint32_t bins[kOrderBins];
  for (int i = int(threadIdx.x); i < kOrderBins; i += 256)
    bins[i] = hist[size_t(blockIdx.x) * kOrderBins + i];
  __syncthreads();
  const uint32_t t0 = blockIdx.x * kOrderGroupTiles + threadIdx.x;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const uint32_t t = t0 + uint32_t(q) * 256u;
    if (t < n) order[atomicAdd(&bins[order_bin(counts[t])], 1u)] = t;
  }
}

constexpr int kSingleItems = 8;
static_assert(kSingleItems == 8, "the vector path loads and stores two uint4 per thread");
constexpr uint32_t kSingleChunk = uint32_t(kSingleThreads * kSingleItems);

// (order: also the tile order of the counts in `in`, when not null)
__global__ void __launch_bounds__(kSingleThreads) scan_single_kernel(
    const uint32_t* __restrict__ in, uint32_t n, uint32_t* __restrict__ out,
    uint32_t* __restrict__ list, DevStatus* __restrict__ status, unsigned long long capacity,
    unsigned long long* __restrict__ total_out, uint32_t* __restrict__ order) {
  static_assert(kSingleThreads == kOrderBins, "the tile order takes the scan's workgroup");
  constexpr int W = kSingleThreads / 64;
  __shared__ uint32_t s_wave[W];
  __shared__ unsigned long long s_wave64[W];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool vec = ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15u) == 0;
  uint32_t carry = 0;
  unsigned long long total = 0;
  for (uint32_t c0 = 0; c0 < n; c0 += kSingleChunk) {
    const uint32_t base = c0 + threadIdx.x * kSingleItems;
    uint32_t vals[kSingleItems];
    uint32_t sum = 0;
    unsigned long long sum64 = 0;
    if (vec && base + kSingleItems <= n) {
      // two 16-byte loads (in is 16-byte aligned, base a multiple of 8)
      const uint4 v0 = *reinterpret_cast<const uint4*>(in + base);
      const uint4 v1 = *reinterpret_cast<const uint4*>(in + base + 4);
      vals[0] = v0.x; vals[1] = v0.y; vals[2] = v0.z; vals[3] = v0.w;
      vals[4] = v1.x; vals[5] = v1.y; vals[6] = v1.z; vals[7] = v1.w;
    } else {
#pragma unroll
      for (int k = 0; k < kSingleItems; ++k) vals[k] = base + k < n ? in[base + k] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kSingleItems; ++k) {
      sum += vals[k];
      sum64 += vals[k];
    }
    // inclusive scan of the thread sums within the wavefront, and its total
    // in 64 bits (a chunk's 32-bit sum may wrap; the 64-bit total may not)
    uint32_t x = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) sum64 += __shfl_xor(sum64, o, 64);
    if (lane == 63) s_wave[wave] = x;
    if (lane == 0) s_wave64[wave] = sum64;
    __syncthreads();
    uint32_t before = 0, chunk = 0;
    unsigned long long chunk64 = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const uint32_t t = s_wave[w];
      before += w < wave ? t : 0u;
      chunk += t;
      chunk64 += s_wave64[w];
    }
    __syncthreads();
    uint32_t run = carry + before + x - sum;
    if (vec && list == nullptr && base + kSingleItems <= n) {
      uint32_t o[kSingleItems];
#pragma unroll
      for (int k = 0; k < kSingleItems; ++k) { o[k] = run; run += vals[k]; }
      *reinterpret_cast<uint4*>(out + base) = make_uint4(o[0], o[1], o[2], o[3]);
      *reinterpret_cast<uint4*>(out + base + 4) = make_uint4(o[4], o[5], o[6], o[7]);
    } else {
#pragma unroll
      for (int k = 0; k < kSingleItems; ++k) {
        if (base + k < n) {
          out[base + k] = run;
          if (list != nullptr && vals[k] != 0u) list[run] = base + k;
        }
        run += vals[k];
      }
    }
    carry += chunk;
    total += chunk64;
  }
  if (threadIdx.x == 0 && status != nullptr) {
    status->pairs_needed = total;
    status->overflow = total > capacity ? 1u : 0u;
  }
  if (threadIdx.x == 0 && total_out != nullptr) *total_out = total;
  if (order != nullptr) {
    __shared__ uint32_t s_bins[kOrderBins];
    __shared__ uint32_t s_tot[kOrderBins / 64];
    order_tiles_by_count(in, n, order, s_bins, s_tot);
  }
}

static hipError_t scan_impl(const uint32_t* in, uint32_t n, uint32_t* tile_sums, uint32_t* out,
                            uint32_t* list, DevStatus* status, unsigned long long capacity,
                            hipStream_t st, unsigned long long* total_out,
                            uint32_t* order = nullptr, uint32_t* order_hist = nullptr) {
  // the tile order: by the scan's own workgroup up to kOrderOneRound tiles,
  // else by its kernels
  if (order != nullptr && n > kOrderOneRound) {
    const uint32_t groups = (n + kOrderGroupTiles - 1) / kOrderGroupTiles;
    hipLaunchKernelGGL(tile_order_hist_kernel, dim3(groups), dim3(256), 0, st, in, n, order_hist);
    hipLaunchKernelGGL(tile_order_offsets_kernel, dim3(1), dim3(kOrderBins), 0, st, order_hist,
                       groups);
    hipLaunchKernelGGL(tile_order_scatter_kernel, dim3(groups), dim3(256), 0, st, in, n,
                       order_hist, order);
    order = nullptr;
  }
  if (n <= kSingleScanMax) {
    hipLaunchKernelGGL(scan_single_kernel, dim3(1), dim3(kSingleThreads), 0, st, in, n, out,
                       list, status, capacity, total_out, order);
    return hipGetLastError();
  }
  const uint32_t n_tiles = (n + kScanTile - 1) / kScanTile;
  if (n_tiles > 0)
    hipLaunchKernelGGL(scan_tile_sums_kernel, dim3(n_tiles), dim3(kScanThreads), 0, st, in, n,
                       tile_sums);
  hipLaunchKernelGGL(scan_tile_sums_scan_kernel, dim3(1), dim3(kScanThreads), 0, st, tile_sums,
                     n_tiles, status, capacity, total_out);
  if (n_tiles > 0)
    hipLaunchKernelGGL(scan_apply_kernel, dim3(n_tiles), dim3(kScanThreads), 0, st, in, n,
                       tile_sums, out, list);
  return hipGetLastError();
}

// order (when not null): the rasters' tile order, longest tiles first;
// order_hist: order_hist_words(n) words for it.
hipError_t launch_scan(const uint32_t* in, uint32_t n, uint32_t* tile_sums, uint32_t* out,
                       DevStatus* status, unsigned long long capacity, hipStream_t st,
                       unsigned long long* total_out, uint32_t* order, uint32_t* order_hist) {
  return scan_impl(in, n, tile_sums, out, nullptr, status, capacity, st, total_out, order,
                   order_hist);
}

uint64_t order_hist_words(uint64_t n_tiles) {
  return uint64_t(kOrderBins) * ((n_tiles + kOrderGroupTiles - 1) / kOrderGroupTiles);
}

// Exclusive scan of a 0/1 flag array and, in the same pass, the compacted
// list of its set entries (ascending); *total_out gets their number.
hipError_t launch_scan_compact(const uint32_t* flags, uint32_t n, uint32_t* tile_sums,
                               uint32_t* offsets, uint32_t* list, hipStream_t st,
                               unsigned long long* total_out) {
  return scan_impl(flags, n, tile_sums, offsets, list, nullptr, 0ull, st, total_out);
}

hipError_t launch_bin_emit(const float* records, const uint8_t* live, const DevView* views,
                           int n_views,
                           uint32_t n_records, const uint32_t* hit_mask, const uint32_t* big_list,
                           const uint32_t* big_count, uint32_t* tile_cursor,
                           DevStatus* status, unsigned long long* comp, hipStream_t st) {
  if (n_records == 0) return hipSuccess;
  const unsigned small_blocks = bin_blocks(n_records);
  hipLaunchKernelGGL(bin_emit_kernel, dim3(small_blocks + kBigBlocks), dim3(256), 0, st, records,
                     live, views, n_views, n_records, hit_mask, big_list, big_count, small_blocks,
                     tile_cursor, status, comp);
  return hipGetLastError();
}


// First kernel of the binning: zeroes the n_words counters at `words`, and
// workgroup 0 adds up the per-workgroup counts preprocess left (visible
// records at partial[k], non-finite primitives at partial[stride + k]) into
// the status block.
__global__ void __launch_bounds__(256) bin_prepare_kernel(uint32_t* __restrict__ words,
                                                          size_t n_words,
                                                          const uint32_t* __restrict__ partial,
                                                          uint32_t n_partials, uint32_t stride,
                                                          DevStatus* __restrict__ status) {
  const size_t i0 = size_t(blockIdx.x) * 256 + threadIdx.x;
  for (size_t k = i0; k < n_words; k += size_t(gridDim.x) * 256) words[k] = 0u;
  if (blockIdx.x != 0) return;
  __shared__ uint32_t s_sum[2][4];
  uint32_t vis = 0, nf = 0;
  uint32_t k0 = 0;
  if ((stride & 3u) == 0 && (reinterpret_cast<uintptr_t>(partial) & 15u) == 0) {
    // 16-byte loads over both halves (stride a multiple of 4)
    const uint4* pv = reinterpret_cast<const uint4*>(partial);
    const uint4* pn = reinterpret_cast<const uint4*>(partial + stride);
    const uint32_t n4 = n_partials / 4;
#pragma unroll 4
    for (uint32_t k = threadIdx.x; k < n4; k += 256) {
      const uint4 a = pv[k], b = pn[k];
      vis += (a.x + a.y) + (a.z + a.w);
      nf += (b.x + b.y) + (b.z + b.w);
    }
    k0 = n4 * 4;
  }
  for (uint32_t k = k0 + threadIdx.x; k < n_partials; k += 256) {
    vis += partial[k];
    nf += partial[stride + k];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    vis += __shfl_xor(vis, o, 64);
    nf += __shfl_xor(nf, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    s_sum[0][threadIdx.x >> 6] = vis;
    s_sum[1][threadIdx.x >> 6] = nf;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    status->spill = 0u;
    status->grad_dirty = 0u;
    status->n_visible = s_sum[0][0] + s_sum[0][1] + s_sum[0][2] + s_sum[0][3];
    status->n_nonfinite = s_sum[1][0] + s_sum[1][1] + s_sum[1][2] + s_sum[1][3];
  }
}

hipError_t launch_bin_prepare(uint32_t* words, size_t n_words, const uint32_t* partial,
                              uint32_t n_partials, uint32_t stride, DevStatus* status,
                              hipStream_t st) {
  size_t blocks = (n_words + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(bin_prepare_kernel, dim3(unsigned(blocks)), dim3(256), 0, st, words, n_words,
                     partial, n_partials, stride, status);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(unsigned(blocks)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

}  // namespace ubs
