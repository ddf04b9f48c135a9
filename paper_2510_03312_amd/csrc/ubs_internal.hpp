// Internal definitions shared by the HIP translation units of libubs.
// Not part of the public ABI (include/ubs.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "ubs.h"

namespace ubs {

constexpr int kRecFloats = 12;   // record: mx my a b c rho o beta r g b depth
constexpr int kGradFloats = 10;  // d mx, my, a, b, c, o, beta, r, g, b
constexpr float kNear = 0.2f;
constexpr float kDilation = 0.3f;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTStop = 1e-4f;

// Per-view constants as the kernels read them (copied into the workspace).
struct DevView {
  float R[9];
  float t[3];
  float cam[3];          // camera centre -R^T t
  float fx, fy, cx, cy;
  float time;
  float query[3];        // query values beyond [t, d] (dim 8-10)
  int32_t scene;
  int32_t W, H;
  int32_t tiles_x, tiles_y;
  int32_t tile_w, tile_h;
  uint32_t tile_base;    // first global tile of the view
  uint32_t rec_base;     // first record of the view
  uint32_t pix_base;     // first pixel of the view
  uint32_t _pad[3];
};
static_assert(sizeof(DevView) % 16 == 0, "DevView alignment");

struct DevScene {
  const float* params;
  float* dparams;
  int64_t n;
  int32_t dim, rot, F;
  uint32_t variant;    // UBS_TUNE_NO_BETA_* bits of the frame (Sec. 5.3 ablations)
  int64_t prim_base;   // first entry of this scene in per-primitive tables
  int64_t list_base;   // first entry of this scene's kept lists
  int64_t par_base;    // first float of this scene's compacted parameter copy
};

// Row offsets of the parameter format (component-major [F][n]).
struct ParamRows {
  int mu_x, mu_q, rot, log_s, lqx, lq, b_x, b_q, o, rgb, F;
};

__host__ __device__ constexpr ParamRows param_rows(int C, int rot) {
  ParamRows r{};
  int k = 0;
  r.mu_x = k; k += 3;
  r.mu_q = k; k += C;
  r.rot = k; k += (rot == UBS_ROT_QUAT ? 4 : 3);
  r.log_s = k; k += 3;
  r.lqx = k; k += 3 * C;
  r.lq = k; k += C * (C + 1) / 2;
  r.b_x = k; k += 1;
  r.b_q = k; k += C;
  r.o = k; k += 1;
  r.rgb = k; k += 3;
  r.F = k;
  return r;
}

// Streaming loads and stores (non-temporal hint): for data a launch reads or
// writes once, so that it does not displace cached data on its way to or
// from HBM.
typedef float stream_f4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void store_stream(float* p, float v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void store_stream(uint32_t* p, uint32_t v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void store_stream(float4* p, float4 v) {
  __builtin_nontemporal_store(stream_f4{v.x, v.y, v.z, v.w}, reinterpret_cast<stream_f4*>(p));
}

__device__ __forceinline__ float load_stream(const float* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ float4 load_stream(const float4* p) {
  const stream_f4 v = __builtin_nontemporal_load(reinterpret_cast<const stream_f4*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}

// Supported dimensions N: 3 (static), 6 (+ view direction), 7 (+ time) and
// 8 .. kMaxDim (+ query values given with each view).
constexpr int kMaxDim = 10;
constexpr int kMaxRows = param_rows(kMaxDim - 3, UBS_ROT_QUAT).F;
__host__ __device__ constexpr bool dim_ok(int dim) {
  return dim == 3 || (dim >= 6 && dim <= kMaxDim);
}

// Where the forward preprocess leaves the primitives some view kept, for
// the adjoint.  The kept primitives of preprocess workgroup b (256
// primitives) go to list b mod kKeptLists, each list holding up to `cap`
// entries (cap = kept_list_cap(n)), with `count` entries per list; pos is a
// kept primitive's index inside its list.  The adjoint runs one thread per
// list entry, entry e of list l being column l cap + e of its compacted
// gradient buffer (the columns past a list's count are unused); the
// preprocess also copies the kept primitive's parameter rows to that column
// of `par` ([F][kKeptLists cap], per scene), so that the adjoint reads dense
// rows instead of gathering a fifth of every line of the parameter array.
// (Several counters spread the workgroups' reserving atomics over several
// addresses.)
constexpr uint32_t kKeptLists = 64;
__host__ __device__ constexpr uint32_t kept_list_cap(int64_t n) {
  return uint32_t(((n + 255) / 256 + kKeptLists - 1) / kKeptLists) * 256u;
}
struct LiveOut {
  uint8_t* rec_live; // per record (all views), 1 if the record survived culling
  uint32_t* flags;   // per primitive, 1 if kept
  uint32_t* pos;
  uint32_t* list;    // kKeptLists lists of cap entries
  uint32_t* count;   // kKeptLists counters, zeroed before the preprocess launch
  uint32_t cap;
  float* par;        // compacted parameter copy, [F][kKeptLists cap]
};
struct LiveIn {
  const uint8_t* rec_live;
  const uint32_t* flags;
  const uint32_t* pos;
  const uint32_t* list;
  const uint32_t* count;
  uint32_t cap;
  const float* par;
};


// Status block, mirrors ubs_status_block.
struct DevStatus {
  unsigned long long pairs_needed;
  uint32_t overflow;
  uint32_t n_nonfinite;
  uint32_t n_visible;
  uint32_t sort_stalled;     // reserved (no bounded wait in the current kernels), 0
  uint32_t work_counter[3];  // persistent raster queues (fwd, bwd, spare)
  uint32_t spill;            // 1 if some tile met more records than its slot block holds
  uint32_t grad_dirty;       // 1 once a backward raster has accumulated into the record
                             // gradients since the binning zeroed the live records' rows
  uint32_t _pad[5];
};

static_assert(offsetof(DevStatus, spill) == offsetof(ubs_status_block, spill), "spill offset");
// Pairs of a tile the counting pass stores directly in the tile's slot block
// (tuning.tile_slots, default kDefaultTileSlots, at most kMaxTileSlots); a
// frame where some tile has more falls back to a second, emitting pass over
// the records.
constexpr uint32_t kDefaultTileSlots = 256;
constexpr uint32_t kMaxTileSlots = 4096;

static_assert(sizeof(DevStatus) == sizeof(ubs_status_block), "status block size");

// Full private layout of the workspace (superset of ubs_layout).
struct Layout {
  ubs_layout pub;
  uint64_t off_views, off_scenes, off_offsets, off_blocksums;
  uint64_t off_tile_counts, off_tile_cursor;  // pairs per tile (+2 counters); segment cursors
  uint64_t off_big_tiles;            // tiles sorted by a workgroup (more than 256 pairs)
  uint64_t off_hit_mask;             // per record: hits among its candidate tiles
  uint64_t off_big_list;             // records binned by a workgroup each
  uint64_t off_comp;                 // emitted (depth bits << 32 | record) per tile segment
  uint64_t off_slots;                // [n_tiles][tile_slots] keys stored by the counting pass
  uint64_t off_keys0, off_values0;   // sorted keys and values
  uint64_t off_tfinal_ws;            // final transmittance kept for the adjoint
  uint64_t off_tile_order;   // the rasters' tile order (longest first)
  uint64_t off_order_hist;   // its per-workgroup bin counts (large frames)
  uint64_t off_kept, off_live_list, off_live_count;  // per-primitive kept flags, kept lists, counts
  uint64_t off_grad_compact;         // adjoint output of live primitives, [F][n] per scene
  uint64_t off_par_compact;          // kept primitives' parameters, [F][n] for each scene
  uint64_t off_pre_partials;         // per-workgroup preprocess counts [2][n_pre_partials]
  int64_t n_pre_partials;
  int64_t n_prims;                   // sum over scenes of primitives
  int64_t n_scan_blocks;
  int32_t rec_bits, digit_bits;
  int32_t tile_w, tile_h;
  uint32_t tile_slots;
};

// Scan geometry.
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;                       // per thread
constexpr int kScanTile = kScanThreads * kScanItems; // 4096 per block

inline int ceil_log2_u64(uint64_t x) {
  int b = 0;
  while ((1ull << b) < x) ++b;
  return b;
}

}  // namespace ubs
