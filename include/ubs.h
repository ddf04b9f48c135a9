/*
 * ubs.h -- C ABI of the MI355X (gfx950) Universal Beta Splatting renderer.
 *
 * The library renders N-dimensional anisotropic Beta primitives (the
 * paper's Section 4: N = 3 + C with C query dimensions; C = 0 static 3-D,
 * C = 3 view direction "UBS-6D", C = 4 time + view direction "UBS-7D",
 * C = 5..7 the 7-D query extended by values each view supplies)
 * through a differentiable tile rasteriser, and returns the gradient of a
 * loss with respect to every primitive parameter.
 *
 * A frame is four calls on one HIP stream, in this order:
 *   ubs_preprocess  condition each primitive on the view's query, project
 *                   it to a screen-space splat record (Section 4.2-4.3,
 *                   Section 3 projection);
 *   ubs_bin_sort    emit one (tile, depth) key per overlapped tile, sort
 *                   each tile's keys, find each tile's range;
 *   ubs_render_fwd  alpha-composite each tile front to back (Section 3
 *                   compositing with the Beta kernel of Section 4.3);
 *   ubs_render_bwd  adjoint of the two previous steps: gradient of the loss
 *                   with respect to every primitive parameter.
 *
 * Conventions shared by every entry point
 *   - All array pointers are DEVICE pointers owned by the caller.  The
 *     library allocates no device memory and keeps no state between calls
 *     other than what it writes into the caller's workspace `ws`.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Calls only
 *     enqueue work; none synchronises the stream.  All four calls of a frame
 *     must use the same frame description, the same `ws`, and be ordered on
 *     one stream (or synchronised by the caller).
 *   - Argument errors are detected on the host before any launch and
 *     returned synchronously; nothing is enqueued in that case.  Conditions
 *     discovered on the device (too many tile pairs, non-finite parameters)
 *     are written to the status block at the head of `ws` (ubs_status_block)
 *     and can be read after the stream has been synchronised.
 *   - Calls on distinct workspaces are independent and may run concurrently
 *     on different streams.  The calls are safe to capture into a HIP graph
 *     (no host synchronisation, no memset/memcpy nodes).
 */
#ifndef UBS_H
#define UBS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define UBS_ABI_VERSION 2
#define UBS_MAX_QUERY_DIMS 7  /* C <= 7: N <= 10 (C = 1, 2 unsupported) */
#define UBS_MAX_VIEWS 4096
#define UBS_MAX_SCENES 256

typedef enum {
  UBS_OK = 0,
  UBS_ERR_ARG = 1,          /* invalid argument (null pointer, size, enum) */
  UBS_ERR_UNSUPPORTED = 2,  /* valid but unsupported (e.g. C = 1, 2, tile shape) */
  UBS_ERR_CAPACITY = 3,     /* workspace too small for the frame */
  UBS_ERR_HIP = 4           /* a HIP runtime call failed */
} ubs_status;

/* Spatial rotation parameterisation (Section 4.2 and its appendix). */
typedef enum {
  UBS_ROT_QUAT = 0,  /* unit quaternion (w, x, y, z), normalised in-kernel   */
  UBS_ROT_SKEW = 1   /* first-order Taylor R = I + A(w), A skew-symmetric    */
} ubs_rot;

/*
 * A scene: n primitives of dimension dim = 3 + C, dim in {3, 6, 7, 8, 9, 10}
 * (C = 1, 2 have no query defined here: UBS_ERR_UNSUPPORTED).
 *
 * params: float32 [F][n], component-major (row r holds component r of every
 * primitive, primitive i at params[r * n + i]).  Rows, in order:
 *   mu_x     3          spatial mean (world units)
 *   mu_q     C          query mean; for C >= 4 the order is
 *                       [t, d0, d1, d2, e0, ..., e_{C-5}] (see ubs_view)
 *   rot      4 | 3      quaternion (w,x,y,z) | skew vector w
 *   log_s_x  3          log spatial scales (s_x = exp)
 *   L_qx     3C         the C x 3 block L_qx, row-major
 *   L_q      C(C+1)/2   lower triangle of L_q, row-major, diagonal stored
 *                       as log scales (diag = exp), strictly-lower free
 *   b_x      1          spatial Beta shape, beta_x = 4 exp(b_x)
 *   b_q      C          query Beta shapes, beta_qi = exp(b_qi)
 *   o        1          opacity in [0, 1] (already activated)
 *   rgb      3          colour (already activated)
 * F = 3 + C + (4|3) + 3 + 3C + C(C+1)/2 + 1 + C + 1 + 3
 *   (35 for UBS-6D and 44 for UBS-7D with the skew rotation; +1 with quats;
 *   at most 78, for dim 10 with quaternions).
 * The covariance is Sigma = L L^T with L = [[R_x diag(s_x), 0], [L_qx, L_q]].
 *
 * dparams: float32 [F][n] in the same layout; ubs_render_bwd OVERWRITES it
 * with d loss / d params (it is not accumulated into).  May be NULL for
 * calls other than ubs_render_bwd.  Must not alias params.
 */
typedef struct {
  int32_t dim;            /* 3, 6, 7, 8, 9, 10 */
  int32_t rot;            /* ubs_rot */
  int64_t n;              /* number of primitives, >= 0 */
  const float* params;    /* device [F][n] */
  float* dparams;         /* device [F][n] or NULL */
} ubs_scene;

/*
 * A view: pinhole camera, OpenCV axes (x right, y down, z forward).
 *   camera point p = R * x_world + t (R row-major 3x3);
 *   pixel (u, v) = (fx p_x / p_z + cx, fy p_y / p_z + cy);
 *   pixel (i, j) covers [i, i+1) x [j, j+1), sampled at its centre
 *   (i + 0.5, j + 0.5).
 * The query of a primitive in this view is q = d (C = 3), q = [time, d]
 * (C = 4) or q = [time, d, query[0], ..., query[C - 5]] (C = 5..7: the
 * paper's query holds any further non-spatial dimensions; their values come
 * with the view), where d is the unit direction from the camera centre
 * -R^T t to the primitive's spatial mean (world frame).  time is ignored
 * unless C >= 4, query[k] unless C > 4 + k; all must be finite.
 */
typedef struct {
  int32_t scene;          /* index into the scene array */
  int32_t width, height;  /* pixels, >= 1 */
  int32_t _pad0;
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  float time;
  float query[3];         /* query values beyond [time, d] (dim 8-10) */
} ubs_view;               /* 96 bytes */

/*
 * Tuning.  tile_w x tile_h in {8x8, 16x8, 16x16, 32x16} (one wavefront of 64
 * lanes per tile); batch_depth in {64, 128, 256} (records staged in LDS per
 * round); digit_bits in [4, 8] (digit width of the radix sort of long tile segments).
 * pair_capacity: number of (tile, primitive) pairs the workspace holds; if a
 * frame needs more, ubs_bin_sort sets the status overflow flag, emits no
 * pairs and the render calls draw nothing (rerun with a larger capacity,
 * see ubs_status_block.pairs_needed); at most 2^30 pairs.  flags:
 * UBS_TUNE_* bits.  tile_slots: 0 (meaning 256) or a multiple of 64 in
 * [256, 4096], the pairs each tile can hold in the workspace's slot block
 * (8 bytes each); a frame where some tile has more takes a second binning
 * pass (same result, slower; ubs_status_block.spill tells).
 */
#define UBS_TUNE_PERSISTENT 1u  /* raster through a persistent grid that takes
                                   tiles from a work queue (16 wavefronts per CU) */
#define UBS_TUNE_PRE_FP32 2u    /* per-primitive math in float32 (default float64) */
/* Ablation variants of Section 5.3 (default: both Beta modulations on). */
#define UBS_TUNE_NO_BETA_COND 4u     /* "w/o Beta condition": conditioning with
                                        diag(bt) = I (the Gaussian conditional) */
#define UBS_TUNE_NO_BETA_OPACITY 8u  /* "w/o Beta opacity": o(q) = o exp(-w.w/2),
                                        the Gaussian conditional opacity */
typedef struct {
  int32_t tile_w, tile_h;
  int32_t batch_depth;
  int32_t digit_bits;
  int64_t pair_capacity;
  uint32_t flags;
  int32_t tile_slots;
} ubs_tuning;

/*
 * Optional per-stage timing.  If ubs_frame.stage_events is non-NULL it points
 * to 2 * UBS_N_STAGES hipEvent_t handles created by the caller; the library
 * records event [2 s] before and [2 s + 1] after the kernels of stage s on
 * the call's stream (the caller reads them with hipEventElapsedTime).  Stages
 * a call does not run are not recorded.  Nothing else changes.
 */
enum {
  UBS_STAGE_PREPROCESS = 0,   /* ubs_preprocess: per-primitive kernel        */
  UBS_STAGE_BIN_COUNT = 1,    /* ubs_bin_sort: tile counts                    */
  UBS_STAGE_SCAN = 2,         /* ubs_bin_sort: exclusive scan of the counts   */
  UBS_STAGE_BIN_EMIT = 3,     /* ubs_bin_sort: pairs into tile segments       */
  UBS_STAGE_SORT = 4,         /* ubs_bin_sort: per-tile depth sort + ranges   */
  UBS_STAGE_RANGES = 5,       /* reserved (ranges come with the sort)         */
  UBS_STAGE_RASTER_FWD = 6,   /* ubs_render_fwd                               */
  UBS_STAGE_GRAD_CLEAR = 7,   /* ubs_render_bwd: clear the record gradients   */
  UBS_STAGE_RASTER_BWD = 8,   /* ubs_render_bwd: compositing adjoint          */
  UBS_STAGE_PRE_BWD = 9,      /* ubs_render_bwd: per-primitive adjoint        */
  UBS_N_STAGES = 10
};

/* A frame: the scenes, the views rendered from them, and the tuning. */
typedef struct {
  const ubs_scene* scenes;   /* host array [n_scenes] */
  int32_t n_scenes;
  int32_t n_views;
  const ubs_view* views;     /* host array [n_views] */
  ubs_tuning tuning;
  void* const* stage_events; /* optional [2 * UBS_N_STAGES] hipEvent_t, or NULL */
} ubs_frame;

/*
 * Workspace layout, filled by ubs_preprocess when ws == NULL.  Every offset
 * is in bytes from the start of ws and 256-byte aligned.
 *
 *   status    ubs_status_block
 *   records   float32 [n_records][12], AoS, record (view v, primitive i) at
 *             index rec_base[v] + i where rec_base[v] is the sum of the
 *             primitive counts of views 0..v-1.  Fields:
 *               0 mean x (px)   1 mean y (px)   2 conic a   3 conic b
 *               4 conic c       5 rho           6 o(q)      7 beta_x
 *               8 r  9 g  10 b (colour)        11 depth (camera z)
 *             conic = inverse of the 2-D covariance, r(p) = a dx^2 +
 *             2 b dx dy + c dy^2 (dx = p_x - mean x); the record touches
 *             pixels with r <= rho, where rho is the largest r with
 *             o(q) (1 - r)^beta_x >= 1/255.  Only the records that
 *             survived culling (live[] = 1) are written; the fields of a
 *             culled record are left as they were.
 *   keys      uint64 [pair_capacity] sorted keys: (global tile << 32) |
 *             float32 bits of depth; global tile = tile_base[v] + ty *
 *             tiles_x(v) + tx with tile_base[v] the tile count of views
 *             0..v-1.
 *   values    uint32 [pair_capacity] record index of each sorted key.
 *   ranges    uint32 [n_tiles][2] [start, end) of each tile in keys;
 *             (0, 0) for an empty tile.
 *   ncontrib  uint32 [n_pixels] per pixel: one past the position (within
 *             its tile's range) of its last contributor.
 *   grad2d    float32 [n_records][10] d loss / d record fields 0-4, 6-10,
 *             after ubs_render_bwd (rows of culled records are not
 *             written).
 *   live      uint8 [n_records] 1 for a record that survived culling
 *             (then rho > 0), 0 for a culled one; written by
 *             ubs_preprocess for every record, read by the binning and
 *             the adjoint.
 * Other regions are private scratch.
 */
typedef struct {
  uint64_t bytes;            /* total workspace size */
  int64_t n_records;
  int64_t n_tiles;
  int64_t n_pixels;          /* sum over views of width * height */
  int64_t pair_capacity;
  int32_t key_bits;          /* significant key bits sorted: 32 + tile bits */
  int32_t n_views;
  uint64_t off_status, off_records, off_keys, off_values, off_ranges;
  uint64_t off_ncontrib, off_grad2d;
  uint64_t off_live;
} ubs_layout;

/* Status block at ws + off_status (device memory, uint32/uint64 fields). */
typedef struct {
  uint64_t pairs_needed;     /* (tile, record) pairs the frame needs */
  uint32_t overflow;         /* 1 if pairs_needed > pair_capacity */
  uint32_t n_nonfinite;      /* primitives with non-finite parameters (culled) */
  uint32_t n_visible;        /* records that survived culling */
  uint32_t sort_stalled;     /* reserved, always 0 */
  uint32_t _reserved[3];     /* internal work counters */
  uint32_t spill;            /* 1 if some tile met more records than
                                tuning.tile_slots: the frame took the second,
                                emitting binning pass */
  uint32_t _pad[6];          /* internal */
} ubs_status_block;

/*
 * ubs_preprocess -- per-primitive conditioning and projection.
 * Paper: Section 4.2 (spatial-orthogonal Cholesky, Sigma = L L^T),
 * Section 4.3 (Beta-modulated conditional slicing and opacity),
 * Section 3 (projection J W Sigma W^T J^T, Mahalanobis distance r).
 *
 * ws == NULL: size query.  Validates the frame and fills *layout (which
 * must then be non-NULL); enqueues nothing.
 * ws != NULL: ws must hold at least layout.bytes (ws_bytes); writes the
 * live flag of every (view, primitive) record and the fields of the live
 * ones, clears the status block and the private tables.  Culled records
 * (behind the near plane z <= 0.2, non-positive-definite 2-D covariance,
 * o(q) < 1/255, non-finite parameters) get live = 0 and no fields.
 */
ubs_status ubs_preprocess(const ubs_frame* frame, void* ws, uint64_t ws_bytes,
                          ubs_layout* layout, void* stream);

/*
 * ubs_bin_sort -- tile binning and (tile, depth) sort.
 * Paper: the "standard splatting" rasterisation the renderer builds on
 * (Section 4.5: splats binned to screen tiles and depth-ordered per tile),
 * with a splat's extent given by its Mahalanobis distance r (Section 3,
 * equation r) and its support r <= rho (Beta kernel, Section 3 / 4.3).
 * Reads the live records in ws (written by ubs_preprocess, or by the caller
 * in the documented record format, with their live flags, after a
 * ubs_preprocess call on the same frame).  A record overlaps a tile iff the minimum of r over the rectangle
 * spanned by the tile's pixel centres (clipped to the image) is at most
 * rho (1 + 2^-10), evaluated in float64 without contraction.  Keys are
 * sorted ascending; equal keys keep record-index order (the result is that
 * of a stable sort of the keys emitted record by record).  The pairs are
 * counted per tile and, in the same pass, stored in a block of
 * tuning.tile_slots slots per tile (part of the workspace); when some tile
 * has more pairs (the status block's spill flag), a second pass over the
 * records places every pair in its tile's segment instead.  Each tile's pairs are then sorted by (depth,
 * record); tuning.digit_bits sets the digit width of the radix sort used for
 * tiles with more than 4096 pairs.
 */
ubs_status ubs_bin_sort(const ubs_frame* frame, void* ws, uint64_t ws_bytes, void* stream);

/*
 * ubs_render_fwd -- front-to-back alpha compositing per tile.
 * Paper: Section 3 compositing, C = sum_i c_i alpha_i prod_{j<i}(1 - alpha_j),
 * with alpha_i = min(0.99, o(q) (1 - r)^beta_x) (Beta kernel, Section 3 and
 * 4.3) for r <= rho; records with alpha < 1/255 are skipped, and a pixel
 * stops before the first record that would take its transmittance below
 * 1e-4.  Background is black: add bg * t_final yourself.
 * image: float32 [sum_v H_v W_v][3] (views concatenated, each row-major HWC);
 * t_final: float32 [sum_v H_v W_v] final transmittance (may be NULL).
 */
ubs_status ubs_render_fwd(const ubs_frame* frame, void* ws, uint64_t ws_bytes,
                          float* image, float* t_final, void* stream);

/*
 * ubs_render_bwd -- adjoint of ubs_render_fwd and ubs_preprocess.
 * Paper: the gradient of the Section 3 compositing C = sum_i c_i alpha_i
 * prod_{j<i} (1 - alpha_j) with respect to every record, chained through
 * the projection (Section 3), the Beta-modulated conditioning and opacity
 * (Section 4.3) and the spatial-orthogonal Cholesky covariance (Section 4.2)
 * to every primitive parameter.
 * Walks each tile back to front, recovering the transmittance by division
 * instead of storing it, reduces per-record gradients across the tile and
 * accumulates them with atomics, then chains them through the projection,
 * conditioning and covariance construction to every parameter.
 * Gradient input, exactly one of:
 *   d_image  float32 [sum_v H_v W_v][3] d loss / d image (with d_t_final
 *            [sum_v H_v W_v] d loss / d t_final, or NULL for zero), or
 *   l1_image and l1_target, both float32 [sum_v H_v W_v][3]: the loss is the
 *            L1 mean |image - target| over all channels of all views, whose
 *            image gradient sign(image - target) / (3 sum_v H_v W_v) (sign 0
 *            at 0) is formed in-kernel; d_image and d_t_final must be NULL.
 * Writes every scenes[s].dparams (must be non-NULL).  The gradient is taken
 * at the parameters ubs_preprocess read: the workspace keeps a copy of the
 * parameters of every primitive with a live record, and this call reads
 * that copy, not scenes[s].params.
 */
ubs_status ubs_render_bwd(const ubs_frame* frame, void* ws, uint64_t ws_bytes,
                          const float* d_image, const float* d_t_final,
                          const float* l1_image, const float* l1_target, void* stream);

/*
 * Optimiser step settings (Sec. 4.5 and Sec. 5.1).  Defaults in the paper:
 * lr_mu_x 1.6e-4, lr_opacity 5e-2, lr_scale 5e-3 (the three log_s_x rows),
 * lr_other 1e-3 (every other row); lambda_o 0.01, lambda_s 0.01 (the
 * paper's lambda_Sigma), lambda_eps 1.  beta1, beta2, eps: Adam's (the paper
 * gives none; 0.9, 0.999, 1e-15 are the conventional choice).  step: the
 * 1-based Adam step t (bias corrections 1 - beta^t).
 */
typedef struct {
  float lr_mu_x, lr_opacity, lr_scale, lr_other;
  float beta1, beta2, eps;
  float lambda_o, lambda_s, lambda_eps;
  int32_t step;
  int32_t _pad;
} ubs_adam;

/*
 * ubs_adam_step -- one optimisation step of a scene's parameters, in place.
 * Paper: Section 4.5 (loss with lambda_o sum |o_i| + lambda_Sigma sum
 * ||s_i||_1; spatial noise injection mu_x += lambda_eps epsilon) and
 * Section 5.1 (Adam, learning rate per parameter group).
 * params, m, v: device float32 [F][n] (ubs_scene layout), read and written;
 * m and v are Adam's moment estimates, zero before step 1, owned by the
 * caller.  dparams: device float32 [F][n], d loss / d params of the
 * reconstruction terms (ubs_render_bwd's output); the regulariser gradients
 * lambda_o sign(o) (opacity row) and lambda_s exp(log s) (log_s_x rows) are
 * added in-kernel.  noise: device float32 [3][n] epsilon for the spatial
 * means (added after the Adam update, times lambda_eps), or NULL for none.
 * Per element: g = dparams + regulariser; m = beta1 m + (1 - beta1) g;
 * v = beta2 v + (1 - beta2) g^2; p -= lr m / (1 - beta1^t) /
 * (sqrt(v / (1 - beta2^t)) + eps).  Nothing is clamped.  Asynchronous on
 * stream; no buffer may alias another.  Errors: UBS_ERR_ARG for a NULL cfg
 * or buffer (n > 0), dim/rot outside the ubs_scene range, n < 0, step < 1,
 * beta outside [0, 1) or eps < 0; UBS_ERR_UNSUPPORTED for dim 4/5;
 * UBS_ERR_HIP if the launch fails.
 */
ubs_status ubs_adam_step(const ubs_adam* cfg, int32_t dim, int32_t rot, int64_t n,
                         float* params, const float* dparams, float* m, float* v,
                         const float* noise, void* stream);

/*
 * ubs_relocate -- relocation of dead primitives, in place.
 * Paper: Section 4.5 ("Densification": cloned opacity o' = 1 - (1 - o)^(1/N);
 * the MCMC primitive management adopted from Deformable Beta Splatting).
 * A primitive is dead if its opacity is below o_min (0.005 by default) or a
 * parameter is not finite; the k-th dead primitive (in index order) copies
 * the first live j whose running opacity sum exceeds uniforms[k] times the
 * total (float64; if the product rounds to the total, the last live
 * primitive); a live primitive picked N - 1 times and its N - 1 copies all
 * get o' = 1 - (1 - o_j)^(1/N), every other parameter is copied, and the
 * Adam moments m, v of all of them are zeroed.  Nothing moves if there is no
 * live or no dead primitive.
 * params, m, v: device float32 [F][n] (ubs_scene layout), read and written.
 * uniforms: device float64 [n], values in [0, 1) (the first n_dead are used).
 * ws: device workspace of at least *ws_bytes_needed bytes; ws == NULL is a
 * size query (writes *ws_bytes_needed, which must then be non-NULL).
 * targets_out: optional device uint32 [n], the pick of every dead slot (the
 * first n_dead entries).  n_dead_out: optional device uint64, the number of
 * dead slots.  Asynchronous on stream.  Errors: UBS_ERR_ARG (bad dim/rot,
 * n < 0, o_min < 0 or NaN, a NULL buffer with n > 0), UBS_ERR_UNSUPPORTED
 * (dim 4/5, n >= 2^31), UBS_ERR_CAPACITY (ws_bytes too small), UBS_ERR_HIP.
 * The pick is exact for n < 2^22 and opacities <= 1: every running sum of
 * float32 opacities >= o_min is then representable in float64.
 */
ubs_status ubs_relocate(int32_t dim, int32_t rot, int64_t n, float* params, float* m, float* v,
                        const double* uniforms, float o_min, void* ws, uint64_t ws_bytes,
                        uint64_t* ws_bytes_needed, uint32_t* targets_out, uint64_t* n_dead_out,
                        void* stream);

/*
 * ubs_relocate_noalloc -- ubs_relocate without a workspace argument and
 * without any device allocation, for callers that cannot allocate: code
 * under HIP graph capture, tight serving or training loops, harnesses that
 * forbid hipMalloc.  Same arguments, semantics and results as ubs_relocate
 * (minus ws, ws_bytes, ws_bytes_needed).  The workspace is a static device
 * array inside the library of the size ubs_relocate needs for
 * UBS_RELOCATE_NOALLOC_MAX_N primitives (about 64 MiB), one per GPU, held
 * until the process ends; its address is looked up on the first call on
 * each device (the device current at the call).  Every call on a GPU uses
 * that GPU's one array: calls that overlap in time on one GPU (other
 * streams, other threads) race and give wrong results; serialise them.
 * Errors: as ubs_relocate, plus UBS_ERR_CAPACITY for n >
 * UBS_RELOCATE_NOALLOC_MAX_N (before any launch).
 */
#define UBS_RELOCATE_NOALLOC_MAX_N (1 << 21)
ubs_status ubs_relocate_noalloc(int32_t dim, int32_t rot, int64_t n, float* params, float* m,
                                float* v, const double* uniforms, float o_min,
                                uint32_t* targets_out, uint64_t* n_dead_out, void* stream);

/*
 * ubs_ssim_loss -- the image loss of Section 4.5, (1 - lambda_ssim) L1 +
 * lambda_ssim (1 - SSIM), and its gradient with respect to the image.
 * SSIM (the measure the paper cites) per pixel and channel under an 11 x 11
 * Gaussian window, sigma 1.5, zero padding outside each view, C1 = 0.01^2,
 * C2 = 0.03^2; L1 and SSIM are means over every channel of every pixel of
 * every view (the paper states neither window nor weight; 0.2 is the usual
 * lambda_ssim).
 * sizes: host int32 [n_views][2] (width, height); image, target: device
 * float32 [sum_v W_v H_v][3], views concatenated, each row-major HWC (the
 * layout of ubs_render_fwd's image).  d_image: device float32, same shape,
 * written (feed it to ubs_render_bwd as d_image).  loss: device float64
 * scalar or NULL.  ws: device workspace of *ws_bytes_needed bytes; ws ==
 * NULL is a size query.  Asynchronous on stream.  Errors: UBS_ERR_ARG (bad
 * view size, n_views, lambda outside [0, 1], NULL buffers), UBS_ERR_CAPACITY,
 * UBS_ERR_UNSUPPORTED (more than 2^31 pixels), UBS_ERR_HIP.
 */
ubs_status ubs_ssim_loss(int32_t n_views, const int32_t* sizes, const float* image,
                         const float* target, float lambda_ssim, float* d_image, double* loss,
                         void* ws, uint64_t ws_bytes, uint64_t* ws_bytes_needed, void* stream);

/* Number of parameter rows F for a scene (0 for an unsupported dim/rot). */
int32_t ubs_param_count(int32_t dim, int32_t rot);

/* ABI version (UBS_ABI_VERSION) of the loaded library. */
int32_t ubs_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* UBS_H */
