// extern "C" entry points of libubs: argument validation, workspace layout
// and kernel launch sequences.  See include/ubs.h for the contract.
#include <math.h>
#include <string.h>

#include <vector>

#include "ubs_internal.hpp"

namespace ubs {

hipError_t launch_preprocess_fwd(bool fp64, const DevScene& S, int scene, const DevView* views,
                                 int n_views, float* records, LiveOut live, uint32_t* partial,
                                 uint32_t stride, hipStream_t st);
hipError_t launch_bin_prepare(uint32_t* words, size_t n_words, const uint32_t* partial,
                              uint32_t n_partials, uint32_t stride, DevStatus* status,
                              hipStream_t st);
hipError_t launch_preprocess_bwd(bool fp64, const DevScene& S, int scene, const DevView* views,
                                 int n_views, const float* records, float* grad2d, LiveIn kept,
                                 float* compact, hipStream_t st);
hipError_t launch_bin_count(const float* records, const uint8_t* live, const DevView* views,
                            int n_views,
                            uint32_t n_records, uint32_t* tile_counts, uint32_t* hit_mask,
                            uint32_t* big_list, uint32_t* big_count, unsigned long long* slots,
                            uint32_t slot_cap, DevStatus* status, float* grad2d, hipStream_t st);
hipError_t launch_scan(const uint32_t* in, uint32_t n, uint32_t* tile_sums, uint32_t* out,
                       DevStatus* status, unsigned long long capacity, hipStream_t st,
                       unsigned long long* total_out, uint32_t* order, uint32_t* order_hist);
uint64_t order_hist_words(uint64_t n_tiles);
hipError_t launch_bin_emit(const float* records, const uint8_t* live, const DevView* views,
                           int n_views,
                           uint32_t n_records, const uint32_t* hit_mask, const uint32_t* big_list,
                           const uint32_t* big_count, uint32_t* tile_cursor,
                           DevStatus* status, unsigned long long* comp, hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t st);
hipError_t launch_tile_sort(unsigned long long* comp, const unsigned long long* slots,
                            uint32_t slot_cap, const uint32_t* tile_counts,
                            const uint32_t* tile_cursor, const DevStatus* status,
                            unsigned long long* keys_out, uint32_t* vals_out, uint32_t* ranges,
                            uint32_t n_tiles, int digit_bits, int rec_bits, uint32_t* big_tiles,
                            uint32_t* n_big_tiles, const uint32_t* order, hipStream_t st);
hipError_t launch_raster_fwd(int tw, int th, int batch, uint32_t persistent_blocks,
                             uint32_t* work, const float* records, const uint32_t* values,
                             const uint32_t* ranges, const uint32_t* order,
                             const DevView* views, int n_views,
                             uint32_t n_tiles, float* image, float* t_ws, float* t_user,
                             uint32_t* ncontrib, hipStream_t st);
hipError_t launch_raster_bwd(int tw, int th, int batch, uint32_t persistent_blocks,
                             uint32_t* work, uint32_t* grad_dirty, const float* records,
                             const uint32_t* values,
                             const uint32_t* ranges, const uint32_t* order,
                             const DevView* views, int n_views,
                             uint32_t n_tiles, const float* t_ws, const uint32_t* ncontrib,
                             const float* d_image, const float* d_tfinal, const float* l1_image,
                             const float* l1_target, float l1_scale, float* grad2d,
                             hipStream_t st);

// Descriptor upload: views are passed by value in chunks and written into
// the workspace by a tiny kernel (no memcpy node, graph-capture safe).
constexpr int kViewChunk = 8;
struct ViewChunk {
  DevView v[kViewChunk];
  int32_t first, count;
};

// Writes a chunk of view descriptors; the first chunk's launch also clears
// the status block (s != nullptr) and the n_scenes kept-primitive counters.
__global__ void upload_views_kernel(ViewChunk c, DevView* __restrict__ dst,
                                    DevStatus* __restrict__ s, uint32_t* __restrict__ n_kept,
                                    int n_counters) {
  const int k = threadIdx.x;
  if (k < c.count) dst[c.first + k] = c.v[k];
  if (s)
    for (int j = k; j < n_counters; j += int(blockDim.x)) n_kept[j] = 0u;
  if (s && k == 0) {
    s->pairs_needed = 0;
    s->overflow = 0;
    s->n_nonfinite = 0;
    s->n_visible = 0;
    s->sort_stalled = 0;
    s->work_counter[0] = s->work_counter[1] = s->work_counter[2] = 0;
  }
}

__global__ void fill_f32_kernel(float* __restrict__ p, size_t n) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t k = i; k < n; k += stride) store_stream(&p[k], 0.0f);
}

// Same with 16-byte stores: p 16-byte aligned; the n % 4 tail by thread 0.
__global__ void fill_f32x4_kernel(float* __restrict__ p, size_t n) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  float4* q = reinterpret_cast<float4*>(p);
  const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
  for (size_t k = i; k < n / 4; k += stride) store_stream(&q[k], z);
  if (i == 0)
    for (size_t k = n & ~size_t(3); k < n; ++k) store_stream(&p[k], 0.0f);
}

// The record gradients before a backward raster: the binning zeroed the
// rows of the live records, and the backward raster marks them dirty; only
// if a backward pass has run since the binning (a second ubs_render_bwd of
// the same frame) is every row cleared again.  A small fixed grid, so that
// the usual case costs one short launch.
__global__ void __launch_bounds__(256) grad_prepare_kernel(float* __restrict__ p, size_t n,
                                                           const DevStatus* __restrict__ status) {
  if (!status->grad_dirty) return;
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  float4* q = reinterpret_cast<float4*>(p);
  const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
  for (size_t k = i; k < n / 4; k += stride) store_stream(&q[k], z);
  if (i == 0)
    for (size_t k = n & ~size_t(3); k < n; ++k) store_stream(&p[k], 0.0f);
}

// Zeroes n floats at p (one launch; none for n == 0).
static void launch_fill_zero(float* p, size_t n, hipStream_t s) {
  if (n == 0) return;
  const bool vec = (reinterpret_cast<uintptr_t>(p) & 15u) == 0;
  const size_t items = vec ? (n + 3) / 4 : n;
  size_t blocks = (items + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (vec)
    hipLaunchKernelGGL(fill_f32x4_kernel, dim3(unsigned(blocks)), dim3(256), 0, s, p, n);
  else
    hipLaunchKernelGGL(fill_f32_kernel, dim3(unsigned(blocks)), dim3(256), 0, s, p, n);
}

// Records a stage event on the call's stream.
static void stage_mark(const ubs_frame* f, int stage, int end, hipStream_t s) {
  if (f->stage_events) {
    hipEvent_t e = static_cast<hipEvent_t>(f->stage_events[2 * stage + end]);
    if (e) (void)hipEventRecord(e, s);
  }
}

static uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

static bool finite_f(float x) { return isfinite(x) != 0; }

// Persistent raster grid: 16 single-wavefront workgroups per compute unit.
static uint32_t persistent_blocks(const ubs_frame* f) {
  if (!(f->tuning.flags & UBS_TUNE_PERSISTENT)) return 0;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return uint32_t(cus > 0 ? cus : 1) * 16u;
}

static bool batch_ok(int b) { return b == 64 || b == 128 || b == 256; }

static bool tile_ok(int tw, int th) {
  return (tw == 16 && th == 16) || (tw == 16 && th == 8) || (tw == 8 && th == 8) ||
         (tw == 32 && th == 16);
}

// Validates the frame and computes the layout and the device descriptors.
static ubs_status plan(const ubs_frame* f, Layout* L, std::vector<DevView>* dv,
                       std::vector<DevScene>* ds) {
  if (!f) return UBS_ERR_ARG;
  if (f->n_scenes < 0 || f->n_scenes > UBS_MAX_SCENES) return UBS_ERR_ARG;
  if (f->n_views < 0 || f->n_views > UBS_MAX_VIEWS) return UBS_ERR_ARG;
  if (f->n_scenes > 0 && !f->scenes) return UBS_ERR_ARG;
  if (f->n_views > 0 && !f->views) return UBS_ERR_ARG;
  const ubs_tuning& tu = f->tuning;
  if (!tile_ok(tu.tile_w, tu.tile_h)) return UBS_ERR_UNSUPPORTED;
  if (tu.digit_bits < 4 || tu.digit_bits > 8) return UBS_ERR_UNSUPPORTED;
  if (!batch_ok(tu.batch_depth)) return UBS_ERR_UNSUPPORTED;
  if (tu.tile_slots != 0 && (tu.tile_slots < int32_t(kDefaultTileSlots) ||
                             tu.tile_slots > int32_t(kMaxTileSlots) || tu.tile_slots % 64 != 0))
    return UBS_ERR_UNSUPPORTED;
  if (tu.pair_capacity < 0 || tu.pair_capacity > int64_t(1) << 30) return UBS_ERR_ARG;
  ds->clear();
  dv->clear();
  uint64_t n_prims = 0, n_grad_compact = 0, n_par_compact = 0, n_list = 0;
  for (int s = 0; s < f->n_scenes; ++s) {
    const ubs_scene& S = f->scenes[s];
    if (S.dim < 3 || S.dim > kMaxDim) return UBS_ERR_ARG;
    if (!dim_ok(S.dim)) return UBS_ERR_UNSUPPORTED;
    if (S.rot != UBS_ROT_QUAT && S.rot != UBS_ROT_SKEW) return UBS_ERR_ARG;
    if (S.n < 0 || S.n > int64_t(0x7fffffff)) return UBS_ERR_ARG;
    if (S.n > 0 && !S.params) return UBS_ERR_ARG;
    DevScene d{};
    d.params = S.params;
    d.dparams = S.dparams;
    d.n = S.n;
    d.dim = S.dim;
    d.rot = S.rot;
    d.F = param_rows(S.dim - 3, S.rot).F;
    d.variant = tu.flags & (UBS_TUNE_NO_BETA_COND | UBS_TUNE_NO_BETA_OPACITY);
    d.prim_base = int64_t(n_prims);
    d.list_base = int64_t(n_list);
    n_prims += uint64_t(S.n);
    n_list += uint64_t(kKeptLists) * kept_list_cap(S.n);
    // the adjoint's compacted gradients: F rows of one column per kept-list entry
    const uint64_t n_compact = uint64_t(d.F) * kKeptLists * kept_list_cap(S.n);
    n_grad_compact = n_grad_compact > n_compact ? n_grad_compact : n_compact;
    // and the kept primitives' parameters in the same layout, every scene's
    d.par_base = int64_t(n_par_compact);
    n_par_compact += n_compact;
    if (n_prims > 0x7fffffffull) return UBS_ERR_UNSUPPORTED;
    ds->push_back(d);
  }
  uint64_t n_rec = 0, n_tiles = 0, n_pix = 0;
  for (int v = 0; v < f->n_views; ++v) {
    const ubs_view& V = f->views[v];
    if (V.scene < 0 || V.scene >= f->n_scenes) return UBS_ERR_ARG;
    if (V.width < 1 || V.height < 1 || V.width > 16384 || V.height > 16384) return UBS_ERR_ARG;
    for (int k = 0; k < 9; ++k) if (!finite_f(V.R[k])) return UBS_ERR_ARG;
    for (int k = 0; k < 3; ++k) if (!finite_f(V.t[k])) return UBS_ERR_ARG;
    if (!(V.fx > 0.0f) || !(V.fy > 0.0f) || !finite_f(V.fx) || !finite_f(V.fy) ||
        !finite_f(V.cx) || !finite_f(V.cy) || !finite_f(V.time))
      return UBS_ERR_ARG;
    for (int k = 0; k < 3; ++k) if (!finite_f(V.query[k])) return UBS_ERR_ARG;
    DevView d{};
    memcpy(d.R, V.R, sizeof(d.R));
    memcpy(d.t, V.t, sizeof(d.t));
    for (int k = 0; k < 3; ++k)  // camera centre -R^T t
      d.cam[k] = -(double(V.R[k]) * V.t[0] + double(V.R[3 + k]) * V.t[1] + double(V.R[6 + k]) * V.t[2]);
    d.fx = V.fx; d.fy = V.fy; d.cx = V.cx; d.cy = V.cy; d.time = V.time;
    for (int k = 0; k < 3; ++k) d.query[k] = V.query[k];
    d.scene = V.scene;
    d.W = V.width; d.H = V.height;
    d.tile_w = tu.tile_w; d.tile_h = tu.tile_h;
    d.tiles_x = (V.width + tu.tile_w - 1) / tu.tile_w;
    d.tiles_y = (V.height + tu.tile_h - 1) / tu.tile_h;
    d.tile_base = uint32_t(n_tiles);
    d.rec_base = uint32_t(n_rec);
    d.pix_base = uint32_t(n_pix);
    n_rec += uint64_t(f->scenes[V.scene].n);
    n_tiles += uint64_t(d.tiles_x) * uint64_t(d.tiles_y);
    n_pix += uint64_t(V.width) * uint64_t(V.height);
    if (n_rec > 0x7fffffffull || n_tiles > 0x7fffffffull || n_pix > 0x7fffffffull)
      return UBS_ERR_UNSUPPORTED;
    dv->push_back(d);
  }
  Layout& l = *L;
  memset(&l, 0, sizeof(l));
  l.pub.n_records = int64_t(n_rec);
  l.pub.n_tiles = int64_t(n_tiles);
  l.pub.n_pixels = int64_t(n_pix);
  l.pub.pair_capacity = tu.pair_capacity;
  l.pub.n_views = f->n_views;
  l.tile_w = tu.tile_w;
  l.tile_h = tu.tile_h;
  l.digit_bits = tu.digit_bits;
  const int tile_bits = n_tiles > 1 ? ceil_log2_u64(n_tiles) : 0;
  l.pub.key_bits = 32 + tile_bits;
  l.rec_bits = n_rec > 1 ? ceil_log2_u64(n_rec) : 1;
  const uint64_t cap = uint64_t(tu.pair_capacity);
  l.n_prims = int64_t(n_prims);
  // the one scan of a frame runs over the tile counts
  l.n_scan_blocks = int64_t((n_tiles + kScanTile - 1) / kScanTile);
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) { const uint64_t o = off; off = align256(off + bytes); return o; };
  l.pub.off_status = take(sizeof(DevStatus));
  l.off_views = take(sizeof(DevView) * uint64_t(f->n_views > 0 ? f->n_views : 1));
  l.off_scenes = take(sizeof(DevScene) * uint64_t(f->n_scenes > 0 ? f->n_scenes : 1));
  l.pub.off_records = take(uint64_t(kRecFloats) * 4 * n_rec);
  l.off_tile_counts = take(4 * (n_tiles + 2));
  l.off_big_tiles = take(4 * n_tiles);
  l.off_tile_order = take(4 * n_tiles);
  l.off_order_hist = take(4 * order_hist_words(n_tiles));
  l.off_tile_cursor = take(4 * n_tiles);
  l.off_hit_mask = take(4 * n_rec);
  l.off_big_list = take(4 * n_rec);
  l.off_offsets = take(4 * n_prims);
  l.off_blocksums = take(4 * uint64_t(l.n_scan_blocks + 1));
  l.off_keys0 = take(8 * cap);
  l.off_comp = take(8 * cap);
  l.tile_slots = f->tuning.tile_slots ? uint32_t(f->tuning.tile_slots) : kDefaultTileSlots;
  l.off_slots = take(8 * uint64_t(l.tile_slots) * n_tiles);
  l.off_values0 = take(4 * cap);
  l.pub.off_ranges = take(8 * n_tiles);
  l.pub.off_ncontrib = take(4 * n_pix);
  l.pub.off_grad2d = take(uint64_t(kGradFloats) * 4 * n_rec);
  l.pub.off_live = take(n_rec);
  l.off_tfinal_ws = take(4 * n_pix);
  l.off_kept = take(4 * n_prims);
  l.off_live_list = take(4 * n_list);
  l.off_live_count = take(4 * uint64_t(kKeptLists) * uint64_t(f->n_scenes > 0 ? f->n_scenes : 1));
  l.off_grad_compact = take(4 * n_grad_compact);
  l.off_par_compact = take(4 * n_par_compact);
  // per-workgroup counts of the preprocess launches (one launch per scene)
  // a multiple of 4, so that both halves of the table are 16-byte aligned
  l.n_pre_partials = int64_t((n_prims / 256 + uint64_t(f->n_scenes) + 1 + 3) & ~uint64_t(3));
  l.off_pre_partials = take(8 * uint64_t(l.n_pre_partials));
  l.pub.bytes = off;
  l.pub.off_keys = l.off_keys0;
  l.pub.off_values = l.off_values0;
  return UBS_OK;
}

template <typename P>
static P* at(void* ws, uint64_t off) {
  return reinterpret_cast<P*>(static_cast<char*>(ws) + off);
}

#define UBS_HIP(call)                         \
  do {                                        \
    if ((call) != hipSuccess) return UBS_ERR_HIP; \
  } while (0)

struct Plan {
  Layout L;
  std::vector<DevView> dv;
  std::vector<DevScene> ds;
};

// Scenes some view renders (preprocess launches one kernel for each).
static bool scene_used(const Plan& p, int sc) {
  for (const DevView& v : p.dv)
    if (v.scene == sc) return true;
  return false;
}

// Workgroups of the preprocess launches: the per-workgroup counts they left.
static uint32_t pre_partials_used(const Plan& p) {
  uint32_t n = 0;
  for (int sc = 0; sc < int(p.ds.size()); ++sc)
    if (scene_used(p, sc) && p.ds[sc].n > 0) n += uint32_t((p.ds[sc].n + 255) / 256);
  return n;
}

static ubs_status prepare(const ubs_frame* f, void* ws, uint64_t ws_bytes, Plan* p) {
  const ubs_status st = plan(f, &p->L, &p->dv, &p->ds);
  if (st != UBS_OK) return st;
  if (!ws) return UBS_ERR_ARG;
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return UBS_ERR_ARG;
  if (ws_bytes < p->L.pub.bytes) return UBS_ERR_CAPACITY;
  return UBS_OK;
}

}  // namespace ubs

using namespace ubs;

extern "C" {

int32_t ubs_abi_version(void) { return UBS_ABI_VERSION; }

int32_t ubs_param_count(int32_t dim, int32_t rot) {
  if (!dim_ok(dim)) return 0;
  if (rot != UBS_ROT_QUAT && rot != UBS_ROT_SKEW) return 0;
  return param_rows(dim - 3, rot).F;
}

ubs_status ubs_preprocess(const ubs_frame* frame, void* ws, uint64_t ws_bytes, ubs_layout* layout,
                          void* stream) {
  Plan p;
  if (!ws) {
    const ubs_status st = plan(frame, &p.L, &p.dv, &p.ds);
    if (st != UBS_OK) return st;
    if (!layout) return UBS_ERR_ARG;
    *layout = p.L.pub;
    return UBS_OK;
  }
  const ubs_status st = prepare(frame, ws, ws_bytes, &p);
  if (st != UBS_OK) return st;
  if (layout) *layout = p.L.pub;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Layout& L = p.L;
  DevStatus* status = at<DevStatus>(ws, L.pub.off_status);
  DevView* views = at<DevView>(ws, L.off_views);
  for (int first = 0; first == 0 || first < frame->n_views; first += kViewChunk) {
    ViewChunk c{};
    c.first = first;
    c.count = frame->n_views - first < kViewChunk ? frame->n_views - first : kViewChunk;
    for (int k = 0; k < c.count; ++k) c.v[k] = p.dv[first + k];
    hipLaunchKernelGGL(upload_views_kernel, dim3(1), dim3(64), 0, s, c, views,
                       first == 0 ? status : nullptr,
                       at<uint32_t>(ws, L.off_live_count), frame->n_scenes * int(kKeptLists));
  }
  UBS_HIP(hipGetLastError());
  const bool fp64 = (frame->tuning.flags & UBS_TUNE_PRE_FP32) == 0;
  float* records = at<float>(ws, L.pub.off_records);
  stage_mark(frame, UBS_STAGE_PREPROCESS, 0, s);
  uint32_t* partial = at<uint32_t>(ws, L.off_pre_partials);
  const uint32_t stride = uint32_t(L.n_pre_partials);
  uint32_t block_base = 0;
  for (int sc = 0; sc < frame->n_scenes; ++sc) {
    bool used = false;
    for (const DevView& v : p.dv) used = used || v.scene == sc;
    if (!used || p.ds[sc].n == 0) continue;
    const LiveOut kept{at<uint8_t>(ws, L.pub.off_live),
                       at<uint32_t>(ws, L.off_kept) + p.ds[sc].prim_base,
                       at<uint32_t>(ws, L.off_offsets) + p.ds[sc].prim_base,
                       at<uint32_t>(ws, L.off_live_list) + p.ds[sc].list_base,
                       at<uint32_t>(ws, L.off_live_count) + size_t(sc) * kKeptLists,
                       kept_list_cap(p.ds[sc].n),
                       at<float>(ws, L.off_par_compact) + p.ds[sc].par_base};
    UBS_HIP(launch_preprocess_fwd(fp64, p.ds[sc], sc, views, frame->n_views, records, kept,
                                  partial + block_base, stride, s));
    block_base += uint32_t((p.ds[sc].n + 255) / 256);
  }
  stage_mark(frame, UBS_STAGE_PREPROCESS, 1, s);
  return UBS_OK;
}

ubs_status ubs_bin_sort(const ubs_frame* frame, void* ws, uint64_t ws_bytes, void* stream) {
  Plan p;
  const ubs_status st = prepare(frame, ws, ws_bytes, &p);
  if (st != UBS_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Layout& L = p.L;
  DevStatus* status = at<DevStatus>(ws, L.pub.off_status);
  const DevView* views = at<DevView>(ws, L.off_views);
  const float* records = at<float>(ws, L.pub.off_records);
  uint32_t* tile_counts = at<uint32_t>(ws, L.off_tile_counts);
  uint32_t* tile_cursor = at<uint32_t>(ws, L.off_tile_cursor);
  uint32_t* sums = at<uint32_t>(ws, L.off_blocksums);
  const uint32_t n_rec = uint32_t(L.pub.n_records);
  const uint32_t n_tiles = uint32_t(L.pub.n_tiles);
  const unsigned long long cap = (unsigned long long)L.pub.pair_capacity;
  auto* comp = at<unsigned long long>(ws, L.off_comp);
  stage_mark(frame, UBS_STAGE_BIN_COUNT, 0, s);
  // the two words after the tile counts count the records binned by
  // workgroups and the tiles sorted by workgroups
  uint32_t* big_count = tile_counts + n_tiles;
  uint32_t* n_big_tiles = tile_counts + n_tiles + 1;
  uint32_t* big_list = at<uint32_t>(ws, L.off_big_list);
  // clear the counters; also add up preprocess's per-workgroup counts
  UBS_HIP(launch_bin_prepare(tile_counts, size_t(n_tiles) + 2, at<uint32_t>(ws, L.off_pre_partials),
                             pre_partials_used(p), uint32_t(L.n_pre_partials), status, s));
  uint32_t* hit_mask = at<uint32_t>(ws, L.off_hit_mask);
  auto* slots = at<unsigned long long>(ws, L.off_slots);
  const uint8_t* live = at<uint8_t>(ws, L.pub.off_live);
  UBS_HIP(launch_bin_count(records, live, views, frame->n_views, n_rec, tile_counts, hit_mask,
                           big_list, big_count, slots, L.tile_slots, status,
                           at<float>(ws, L.pub.off_grad2d), s));
  stage_mark(frame, UBS_STAGE_BIN_COUNT, 1, s);
  stage_mark(frame, UBS_STAGE_SCAN, 0, s);
  // segment starts of the tiles; the total sets pairs_needed and overflow
  UBS_HIP(launch_scan(tile_counts, n_tiles, sums, tile_cursor, status, cap, s, nullptr,
                      at<uint32_t>(ws, L.off_tile_order), at<uint32_t>(ws, L.off_order_hist)));
  stage_mark(frame, UBS_STAGE_SCAN, 1, s);
  stage_mark(frame, UBS_STAGE_BIN_EMIT, 0, s);
  UBS_HIP(launch_bin_emit(records, live, views, frame->n_views, n_rec, hit_mask, big_list,
                          big_count, tile_cursor, status, comp, s));
  stage_mark(frame, UBS_STAGE_BIN_EMIT, 1, s);
  stage_mark(frame, UBS_STAGE_SORT, 0, s);
  UBS_HIP(launch_tile_sort(comp, slots, L.tile_slots, tile_counts, tile_cursor, status,
                           at<unsigned long long>(ws, L.pub.off_keys),
                           at<uint32_t>(ws, L.pub.off_values), at<uint32_t>(ws, L.pub.off_ranges),
                           n_tiles, L.digit_bits, L.rec_bits, at<uint32_t>(ws, L.off_big_tiles),
                           n_big_tiles, at<uint32_t>(ws, L.off_tile_order), s));
  stage_mark(frame, UBS_STAGE_SORT, 1, s);
  return UBS_OK;
}

ubs_status ubs_render_fwd(const ubs_frame* frame, void* ws, uint64_t ws_bytes, float* image,
                          float* t_final, void* stream) {
  Plan p;
  const ubs_status st = prepare(frame, ws, ws_bytes, &p);
  if (st != UBS_OK) return st;
  if (!image && p.L.pub.n_pixels > 0) return UBS_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Layout& L = p.L;
  stage_mark(frame, UBS_STAGE_RASTER_FWD, 0, s);
  DevStatus* status = at<DevStatus>(ws, L.pub.off_status);
  UBS_HIP(launch_raster_fwd(L.tile_w, L.tile_h, frame->tuning.batch_depth, persistent_blocks(frame),
                            &status->work_counter[0], at<float>(ws, L.pub.off_records),
                            at<uint32_t>(ws, L.pub.off_values), at<uint32_t>(ws, L.pub.off_ranges),
                            at<uint32_t>(ws, L.off_tile_order),
                            at<DevView>(ws, L.off_views), frame->n_views, uint32_t(L.pub.n_tiles),
                            image, at<float>(ws, L.off_tfinal_ws), t_final,
                            at<uint32_t>(ws, L.pub.off_ncontrib), s));
  stage_mark(frame, UBS_STAGE_RASTER_FWD, 1, s);
  return UBS_OK;
}

ubs_status ubs_render_bwd(const ubs_frame* frame, void* ws, uint64_t ws_bytes,
                          const float* d_image, const float* d_t_final, const float* l1_image,
                          const float* l1_target, void* stream) {
  Plan p;
  const ubs_status st = prepare(frame, ws, ws_bytes, &p);
  if (st != UBS_OK) return st;
  const bool has_d = d_image != nullptr;
  const bool has_l1 = l1_image != nullptr || l1_target != nullptr;
  if (has_d == has_l1) return UBS_ERR_ARG;
  if (has_l1 && (!l1_image || !l1_target || d_t_final)) return UBS_ERR_ARG;
  for (int sc = 0; sc < frame->n_scenes; ++sc)
    if (frame->scenes[sc].n > 0 && !frame->scenes[sc].dparams) return UBS_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Layout& L = p.L;
  float* grad2d = at<float>(ws, L.pub.off_grad2d);
  const size_t ng = size_t(L.pub.n_records) * kGradFloats;
  DevStatus* status = at<DevStatus>(ws, L.pub.off_status);
  stage_mark(frame, UBS_STAGE_GRAD_CLEAR, 0, s);
  if (ng > 0)
    hipLaunchKernelGGL(grad_prepare_kernel, dim3(512), dim3(256), 0, s, grad2d, ng, status);
  stage_mark(frame, UBS_STAGE_GRAD_CLEAR, 1, s);
  const float l1_scale = L.pub.n_pixels > 0 ? float(1.0 / (3.0 * double(L.pub.n_pixels))) : 0.0f;
  const DevView* views = at<DevView>(ws, L.off_views);
  stage_mark(frame, UBS_STAGE_RASTER_BWD, 0, s);
  UBS_HIP(launch_raster_bwd(L.tile_w, L.tile_h, frame->tuning.batch_depth, persistent_blocks(frame),
                            &status->work_counter[1], &status->grad_dirty,
                            at<float>(ws, L.pub.off_records),
                            at<uint32_t>(ws, L.pub.off_values), at<uint32_t>(ws, L.pub.off_ranges),
                            at<uint32_t>(ws, L.off_tile_order),
                            views, frame->n_views, uint32_t(L.pub.n_tiles),
                            at<float>(ws, L.off_tfinal_ws), at<uint32_t>(ws, L.pub.off_ncontrib),
                            d_image, d_t_final, l1_image, l1_target, l1_scale, grad2d, s));
  stage_mark(frame, UBS_STAGE_RASTER_BWD, 1, s);
  const bool fp64 = (frame->tuning.flags & UBS_TUNE_PRE_FP32) == 0;
  stage_mark(frame, UBS_STAGE_PRE_BWD, 0, s);
  for (int sc = 0; sc < frame->n_scenes; ++sc) {
    if (p.ds[sc].n == 0) continue;
    bool used = false;
    for (const DevView& v : p.dv) used = used || v.scene == sc;
    if (!used) {  // a scene no view sees has zero gradient
      launch_fill_zero(p.ds[sc].dparams, size_t(p.ds[sc].F) * size_t(p.ds[sc].n), s);
      continue;
    }
    // the adjoint runs only for the primitives some view kept (listed by
    // the forward preprocess)
    const LiveIn kept{at<uint8_t>(ws, L.pub.off_live),
                      at<uint32_t>(ws, L.off_kept) + p.ds[sc].prim_base,
                      at<uint32_t>(ws, L.off_offsets) + p.ds[sc].prim_base,
                      at<uint32_t>(ws, L.off_live_list) + p.ds[sc].list_base,
                      at<uint32_t>(ws, L.off_live_count) + size_t(sc) * kKeptLists,
                      kept_list_cap(p.ds[sc].n),
                      at<float>(ws, L.off_par_compact) + p.ds[sc].par_base};
    UBS_HIP(launch_preprocess_bwd(fp64, p.ds[sc], sc, views, frame->n_views,
                                  at<float>(ws, L.pub.off_records), grad2d, kept,
                                  at<float>(ws, L.off_grad_compact), s));
  }
  stage_mark(frame, UBS_STAGE_PRE_BWD, 1, s);
  UBS_HIP(hipGetLastError());
  return UBS_OK;
}

}  // extern "C"
