// Per-tile rasterisation: front-to-back compositing and its adjoint.
//
// One wavefront (64 lanes) per tile.  Lane l owns the pixels of column
// l % TW in rows l / TW + k * (64 / TW), k < TW * TH / 64 (a 16x16 tile gives
// each lane a strip of 4 pixels).  The tile's sorted records are staged
// through LDS 64 at a time (one per lane); every lane then walks the batch.
// Because a lane's pixels share one column, dx = px - mx is shared and the
// quadratic form costs r = A + dy (B + c dy) per pixel with A, B per record.
//
// Forward: a pixel stops before the first record that would take its
// transmittance below 1e-4; the wavefront stops when all its pixels have.
// Backward: each tile is walked back to front from the last contributor;
// the transmittance in front of a record is recovered by division.  A lane
// first sums the gradient terms of its own pixels; the wavefront then folds
// its ten per-record sums onto fewer lanes with lane swaps, finishes them
// with DPP sums within 16-lane rows and half-rows, and ten lanes add the
// ten totals to the record's accumulator in one atomic instruction.
//
// Both passes take every per-pixel decision (support test, skip, stop)
// through the same inline functions, so the backward pass visits exactly
// the contributors the forward pass used.
#include <type_traits>

#include "ubs_internal.hpp"

namespace ubs {

// Hardware base-2 exponential and logarithm (v_exp_f32 / v_log_f32).
__device__ __forceinline__ float hw_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float hw_log2(float x) { return __builtin_amdgcn_logf(x); }

// Record fields as staged in LDS.
struct Staged {
  float4 g0;  // mx, my, a, 2b
  float4 g1;  // c, rho, log2(o), beta
  float4 g2;  // r, g, b, (record index as bits)
};

__device__ __forceinline__ Staged stage_record(const float* __restrict__ records, uint32_t rec) {
  const float4* rp = reinterpret_cast<const float4*>(records + size_t(rec) * kRecFloats);
  const float4 a = rp[0], b = rp[1], c = rp[2];
  Staged s;
  s.g0 = make_float4(a.x, a.y, a.z, 2.0f * a.w);
  s.g1 = make_float4(b.x, b.y, hw_log2(b.z), b.w);
  s.g2 = make_float4(c.x, c.y, c.z, __uint_as_float(rec));
  return s;
}

// Column terms of the quadratic form for one record and one lane:
// r = a dx^2 + 2 b dx dy + c dy^2 = A + dy (B + c dy), A = dx (a dx), B = 2b dx.
struct ColTerms {
  float A, B;
};
__device__ __forceinline__ ColTerms col_terms(const float4 g0, float dx) {
  return ColTerms{dx * (g0.z * dx), g0.w * dx};
}
__device__ __forceinline__ float eval_r(const ColTerms t, float c, float dy) {
  return t.A + dy * (t.B + c * dy);
}

// sigma = o (1 - r)^beta = exp2(log2 o + beta log2(1 - r)); alpha = min(0.99, sigma).
__device__ __forceinline__ float eval_sigma(float r, float lo, float beta, float* l2) {
  const float l = hw_log2(1.0f - r);
  *l2 = l;
  return hw_exp2(lo + beta * l);
}

__device__ __forceinline__ int view_of_tile(const DevView* __restrict__ views, int n_views,
                                            uint32_t tile) {
  int lo = 0, hi = n_views - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (views[mid].tile_base <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <int TW, int TH>
struct TileGeom {
  static constexpr int PPL = TW * TH / 64;   // pixels per lane
  static constexpr int RSTEP = 64 / TW;      // rows between a lane's pixels
  static_assert(TW * TH % 64 == 0 && 64 % TW == 0, "tile shape");
};

template <int TW, int TH, int BATCH>
__device__ __forceinline__ void raster_fwd_tile(
    uint32_t tile, float4* s0, float4* s1, float4* s2, const float* __restrict__ records,
    const uint32_t* __restrict__ values, const uint32_t* __restrict__ ranges,
    const DevView* __restrict__ views, int n_views, float* __restrict__ image,
    float* __restrict__ t_ws, float* __restrict__ t_user, uint32_t* __restrict__ ncontrib) {
  constexpr int PPL = TileGeom<TW, TH>::PPL;
  constexpr int RSTEP = TileGeom<TW, TH>::RSTEP;
  constexpr int PER_LANE = BATCH / 64;
  const int lane = threadIdx.x;
  const DevView& V = views[view_of_tile(views, n_views, tile)];
  const uint32_t lt = tile - V.tile_base;
  const int ty = int(lt) / V.tiles_x, tx = int(lt) - ty * V.tiles_x;
  const int px = tx * TW + lane % TW;
  const int py0 = ty * TH + lane / TW;
  const float fx = float(px) + 0.5f;
  // T: transmittance; a pixel that has stopped keeps it negated, so that
  // every later record fails its T (1 - alpha) >= 1e-4 test (instead of the
  // pixel's state being tested on every record); |T| is the final value
  // (pixels outside the image start stopped)
  float T[PPL], cr[PPL], cg[PPL], cb[PPL];
  uint32_t last[PPL];
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    T[k] = (px >= V.W || py0 + k * RSTEP >= V.H) ? -1.0f : 1.0f;
    cr[k] = cg[k] = cb[k] = 0.0f; last[k] = 0;
  }
  const uint32_t start = ranges[2 * size_t(tile)], end = ranges[2 * size_t(tile) + 1];
  for (uint32_t b0 = start; b0 < end; b0 += BATCH) {
    // the tile is finished once every pixel has stopped (checked per batch)
    bool running = false;
#pragma unroll
    for (int k = 0; k < PPL; ++k) running = running || T[k] >= 0.0f;
    if (__ballot(running) == 0ull) break;
    __syncthreads();
#pragma unroll
    for (int m = 0; m < PER_LANE; ++m) {
      const uint32_t idx = b0 + uint32_t(m * 64 + lane);
      if (idx < end) {
        const Staged st = stage_record(records, values[idx]);
        s0[m * 64 + lane] = st.g0;
        s1[m * 64 + lane] = st.g1;
        s2[m * 64 + lane] = st.g2;
      }
    }
    __syncthreads();
    // (wavefront-uniform: the record loop runs on scalar counters)
    const int nb = __builtin_amdgcn_readfirstlane(int(min(uint32_t(BATCH), end - b0)));
    for (int j = 0; j < nb; ++j) {
      const float4 g0 = s0[j], g1 = s1[j], g2 = s2[j];
      const ColTerms ct = col_terms(g0, fx - g0.x);
#pragma unroll
      for (int k = 0; k < PPL; ++k) {
        const float dy = float(py0 + k * RSTEP) + 0.5f - g0.y;
        const float r = eval_r(ct, g1.x, dy);
        if (!(r <= g1.y)) continue;
        // one branch per pixel: skipping (alpha below 1/255) and stopping
        // are taken by selects
        float l2;
        const float sigma = eval_sigma(r, g1.z, g1.w, &l2);
        const float alpha = fminf(kAlphaMax, sigma);
        const float test = T[k] * (1.0f - alpha);
        const bool hit = alpha >= kAlphaMin;
        const bool pass = test >= kTStop;
        const bool con = hit && pass;
        const float w = con ? alpha * T[k] : 0.0f;
        cr[k] += g2.x * w;
        cg[k] += g2.y * w;
        cb[k] += g2.z * w;
        // a hit that fails the stop test stops the pixel (T kept negated)
        const float tn = pass ? test : -fabsf(T[k]);
        T[k] = hit ? tn : T[k];
        last[k] = con ? b0 - start + uint32_t(j) + 1u : last[k];
      }
    }
  }
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    const int py = py0 + k * RSTEP;
    if (px < V.W && py < V.H) {
      const size_t pix = size_t(V.pix_base) + size_t(py) * V.W + px;
      image[3 * pix] = cr[k];
      image[3 * pix + 1] = cg[k];
      image[3 * pix + 2] = cb[k];
      // (the internal copy keeps the sign: negative for a pixel that stopped)
      t_ws[pix] = T[k];
      if (t_user) t_user[pix] = fabsf(T[k]);
      ncontrib[pix] = last[k];
    }
  }
}

// Next tile for this workgroup: blockIdx.x on the first visit without a work
// queue, else the next index of the queue counter (lane 0 takes it, the
// wavefront shares it).
__device__ __forceinline__ uint32_t next_tile(uint32_t* work, bool first) {
  if (!work) return first ? blockIdx.x : 0xffffffffu;
  uint32_t t = 0;
  if (threadIdx.x == 0) t = atomicAdd(work, 1u);
  return uint32_t(__shfl(int(t), 0, 64));
}

template <int TW, int TH, int BATCH>
__global__ void __launch_bounds__(64) raster_fwd_kernel(
    const float* __restrict__ records, const uint32_t* __restrict__ values,
    const uint32_t* __restrict__ ranges, const DevView* __restrict__ views, int n_views,
    uint32_t n_tiles, const uint32_t* __restrict__ order, uint32_t* __restrict__ work,
    float* __restrict__ image, float* __restrict__ t_ws, float* __restrict__ t_user,
    uint32_t* __restrict__ ncontrib) {
  __shared__ float4 s0[BATCH], s1[BATCH], s2[BATCH];
  for (uint32_t q = next_tile(work, true); q < n_tiles; q = next_tile(work, false))
    raster_fwd_tile<TW, TH, BATCH>(order[q], s0, s1, s2, records, values, ranges, views, n_views,
                                   image, t_ws, t_user, ncontrib);
}

// Sums over each 16-lane row by DPP row rotations (by 1, 2, 4, 8), of N
// values at once: every lane of a row ends with the row's totals.  A rotation
// has no out-of-row source lane, so each step is one DPP add.
template <int CTRL>
__device__ __forceinline__ float dpp_row(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xf, 0xf, false));
}
template <int N>
__device__ __forceinline__ void row_sum_all(float* v) {
#pragma unroll
  for (int q = 0; q < N; ++q) v[q] += dpp_row<0x121>(v[q]);
#pragma unroll
  for (int q = 0; q < N; ++q) v[q] += dpp_row<0x122>(v[q]);
#pragma unroll
  for (int q = 0; q < N; ++q) v[q] += dpp_row<0x124>(v[q]);
#pragma unroll
  for (int q = 0; q < N; ++q) v[q] += dpp_row<0x128>(v[q]);
}
// Lane exchanges of gfx950: swap_halves(a, b) returns (a with its upper 32
// lanes replaced by b's lower 32, b with its lower 32 replaced by a's upper
// 32); swap_rows(a, b) does the same between a's odd rows and b's even rows
// (rows of 16 lanes).
struct FPair {
  float a, b;
};
__device__ __forceinline__ FPair swap_halves(float a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return FPair{__uint_as_float(r[0]), __uint_as_float(r[1])};
}
__device__ __forceinline__ FPair swap_rows(float a, float b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return FPair{__uint_as_float(r[0]), __uint_as_float(r[1])};
}
// Two zeros from one 64-bit move, which the compiler cannot rematerialise.
__device__ __forceinline__ void opaque_zero2(float& a, float& b) {
  uint64_t z;
  asm volatile("v_mov_b64 %0, 0" : "=v"(z));
  a = __uint_as_float(uint32_t(z));
  b = __uint_as_float(uint32_t(z >> 32));
}
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = min(x, uint32_t(__shfl_xor(int(x), o, 64)));
  return x;
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = max(x, uint32_t(__shfl_xor(int(x), o, 64)));
  return x;
}

// HAS_DT: a gradient of the final transmittance is given (d_tfinal).
template <int TW, int TH, int BATCH, bool HAS_DT>
__device__ __forceinline__ void raster_bwd_tile(
    uint32_t tile, float4* s0, float4* s1, float4* s2,
    const float* __restrict__ records,
    const uint32_t* __restrict__ values, const uint32_t* __restrict__ ranges,
    const DevView* __restrict__ views, int n_views, const float* __restrict__ t_ws,
    const uint32_t* __restrict__ ncontrib, const float* __restrict__ d_image,
    const float* __restrict__ d_tfinal, const float* __restrict__ l1_image,
    const float* __restrict__ l1_target, float l1_scale, float* __restrict__ grad2d) {
  constexpr int PPL = TileGeom<TW, TH>::PPL;
  constexpr int RSTEP = TileGeom<TW, TH>::RSTEP;
  constexpr int PER_LANE = BATCH / 64;
  const int lane = threadIdx.x;
  const DevView& V = views[view_of_tile(views, n_views, tile)];
  const uint32_t lt = tile - V.tile_base;
  const int ty = int(lt) / V.tiles_x, tx = int(lt) - ty * V.tiles_x;
  const int px = tx * TW + lane % TW;
  const int py0 = ty * TH + lane / TW;
  const float fx = float(px) + 0.5f;
  const uint32_t start = ranges[2 * size_t(tile)];
  // gTf: d loss / d T_final times T_final (the transmittance gradient enters
  // every record's d alpha as - gTf / (1 - alpha)); D: the pixel's colour
  // gradient dotted with the colour composited behind the current record
  float T[PPL], D[PPL], gR[PPL], gG[PPL], gB[PPL], gTf[PPL];
  uint32_t last[PPL];
  uint32_t lane_max = 0, lane_stop = 0xffffffffu;
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    const int py = py0 + k * RSTEP;
    float Tf = 1.0f;
    gR[k] = gG[k] = gB[k] = gTf[k] = 0.0f; last[k] = 0;
    if (px < V.W && py < V.H) {
      const size_t pix = size_t(V.pix_base) + size_t(py) * V.W + px;
      Tf = t_ws[pix];
      last[k] = ncontrib[pix];
      if (Tf < 0.0f) {   // the pixel stopped
        Tf = -Tf;
        lane_stop = min(lane_stop, last[k]);
      }
      if (d_image) {
        gR[k] = d_image[3 * pix];
        gG[k] = d_image[3 * pix + 1];
        gB[k] = d_image[3 * pix + 2];
        if (HAS_DT) gTf[k] = d_tfinal[pix] * Tf;
      } else {
        const float e0 = l1_image[3 * pix] - l1_target[3 * pix];
        const float e1 = l1_image[3 * pix + 1] - l1_target[3 * pix + 1];
        const float e2 = l1_image[3 * pix + 2] - l1_target[3 * pix + 2];
        gR[k] = e0 > 0.0f ? l1_scale : (e0 < 0.0f ? -l1_scale : 0.0f);
        gG[k] = e1 > 0.0f ? l1_scale : (e1 < 0.0f ? -l1_scale : 0.0f);
        gB[k] = e2 > 0.0f ? l1_scale : (e2 < 0.0f ? -l1_scale : 0.0f);
      }
    }
    T[k] = Tf;
    D[k] = 0.0f;
    lane_max = max(lane_max, last[k]);
  }
  // (wavefront-uniform: the batch loop runs on scalar counters)
  const uint32_t span = __builtin_amdgcn_readfirstlane(wave_max_u32(lane_max));
  // Records at or beyond a pixel's last contributor contribute nothing to it
  // unless the pixel stopped (its own alpha test fails there otherwise), so
  // only records at or beyond the smallest last contributor of a stopped
  // pixel need the position test.
  const uint32_t stop_min = __builtin_amdgcn_readfirstlane(wave_min_u32(lane_stop));
  for (uint32_t hi = span; hi > 0;) {
    const uint32_t lo = hi > uint32_t(BATCH) ? hi - uint32_t(BATCH) : 0u;
    const uint32_t cnt = hi - lo;
    __syncthreads();
#pragma unroll
    for (int m = 0; m < PER_LANE; ++m) {
      const uint32_t q = uint32_t(m * 64 + lane);
      if (q < cnt) {
        const Staged st = stage_record(records, values[start + lo + q]);
        s0[q] = st.g0;
        s1[q] = st.g1;
        s2[q] = st.g2;
      }
    }
    __syncthreads();
    // one record: the lane's pixel sums, then their wavefront totals added to
    // the record's gradient row (CHECK: test each pixel's last contributor)
    auto record = [&](auto check, int j) {
      constexpr bool CHECK = decltype(check)::value;
      const uint32_t pos = lo + uint32_t(j);
      const float4 g0 = s0[j], g1 = s1[j], g2 = s2[j];
      const float dx = fx - g0.x;
      const ColTerms ct = col_terms(g0, dx);
      // per-lane sums over the lane's pixels (the factors common to a record,
      // 1/o, ln 2 and -beta, are applied by the per-primitive adjoint):
      //   a_o = sum s,  a_be = sum s log2(1 - r),  a_dr = sum s / (1 - r)
      //   (a_dry, a_dryy: times dy, dy^2) with s = sigma d loss / d alpha
      // (zeros the compiler cannot rematerialise: otherwise it re-creates
      // them on every path that skips the first pixel's update)
      float a_r, a_g, a_b, a_o, a_be, a_dr, a_dry, a_dryy;
      opaque_zero2(a_r, a_g);
      opaque_zero2(a_b, a_o);
      opaque_zero2(a_be, a_dr);
      opaque_zero2(a_dry, a_dryy);
#pragma unroll
      for (int k = 0; k < PPL; ++k) {
        const float dy = float(py0 + k * RSTEP) + 0.5f - g0.y;
        const float r = eval_r(ct, g1.x, dy);
        // one branch per pixel: the rare cases inside it (alpha below
        // 1/255 at the support's rim, sigma at the 0.99 clamp) are taken
        // by zeroing alpha or sigma, which makes their updates no-ops
        if (!((!CHECK || pos < last[k]) && r <= g1.y)) continue;
        float l2;
        const float sigma0 = eval_sigma(r, g1.z, g1.w, &l2);
        const bool con = fminf(kAlphaMax, sigma0) >= kAlphaMin;
        const float alpha = con ? fminf(kAlphaMax, sigma0) : 0.0f;
        // sigma where alpha follows it (below the clamp), else 0
        const float sigma = alpha < kAlphaMax ? alpha : 0.0f;
        // (alpha = 0 gives ioma = 1 exactly: the hardware reciprocal is exact
        // on powers of two, so T passes unchanged)
        const float ioma = fast_rcp(1.0f - alpha);
        const float Ti = T[k] * ioma;
        const float w = alpha * Ti;
        a_r += gR[k] * w;
        a_g += gG[k] * w;
        a_b += gB[k] * w;
        // g . (c - S): the colour gradient g dotted with the record's colour
        // minus the colour S composited behind it; S updates as
        // S += alpha (c - S), so D = g . S as D += alpha dot
        const float dot = (gR[k] * g2.x + gG[k] * g2.y + gB[k] * g2.z) - D[k];
        const float dalpha = HAS_DT ? Ti * dot - gTf[k] * ioma : Ti * dot;
        const float sd = sigma * dalpha;
        a_o += sd;
        a_be += sd * l2;
        const float q = sd * fast_rcp(1.0f - r);
        a_dr += q;
        const float qy = q * dy;
        a_dry += qy;
        a_dryy += qy * dy;
        D[k] += alpha * dot;
        T[k] = Ti;
      }
      // the record's pixel sums (a record none of whose pixels contribute,
      // a few in a hundred thousand, adds zeros) (P, Q, U, V, E, A_o, A_b, colour): the
      // per-primitive adjoint turns them into record-field gradients
      float gv[kGradFloats];
      gv[0] = dx * a_dr;
      gv[1] = a_dry;
      gv[2] = dx * gv[0];
      gv[3] = dx * a_dry;
      gv[4] = a_dryy;
      gv[5] = a_o;
      gv[6] = a_be;
      gv[7] = a_r;
      gv[8] = a_g;
      gv[9] = a_b;
      // sums over the wavefront: halves folded onto each other (permlane32
      // swap: field 2p in lanes 0-31, 2p+1 in lanes 32-63), row pairs folded
      // (permlane16 swap: one field per row), then DPP sums within rows and
      // half-rows
      float h[5];
#pragma unroll
      for (int p = 0; p < 5; ++p) {
        const FPair sw = swap_halves(gv[2 * p], gv[2 * p + 1]);
        h[p] = sw.a + sw.b;
      }
      float t3[3];
      {
        const FPair s0 = swap_rows(h[0], h[1]);   // rows: fields 0, 2, 1, 3
        const FPair s1 = swap_rows(h[2], h[3]);   // rows: fields 4, 6, 5, 7
        t3[0] = s0.a + s0.b;
        t3[1] = s1.a + s1.b;
        t3[2] = h[4];   // rows: fields 8, 8, 9, 9, each row a partial sum
      }
      // t3[0] and t3[1] share one register from here: pairs of lanes 8
      // apart are summed in each, half-rows take t3[0]'s (lanes 0-7) or
      // t3[1]'s (8-15) sums, and a half-row mirror and two quad
      // permutations finish the 8-lane sums; t3[2] is summed over its rows
      float x0 = t3[0] + dpp_row<0x128>(t3[0]), x1 = t3[1] + dpp_row<0x128>(t3[1]);
      asm volatile("" : "+v"(x0), "+v"(x1));   // (both sums, then a select, not a branch)
      float u = (lane & 8) ? x1 : x0;
      u += dpp_row<0x141>(u);   // lane l of a half-row and lane 7 - l
      u += dpp_row<0x4E>(u);    // quad permutation [2, 3, 0, 1]
      u += dpp_row<0xB1>(u);    // quad permutation [1, 0, 3, 2]
      row_sum_all<1>(&t3[2]);
      // rows 1 and 3 add the totals of rows 0 and 2 (DPP row broadcast of
      // each row's lane 15 into the next row; rows 0 and 2 are not written):
      // fields 8 and 9 complete.  (One DPP add: the compiler would build it
      // from a move and an add.  The nop gives the two wait states a DPP
      // read needs after the VALU write of its source.)
      asm volatile("s_nop 1\n\tv_add_f32_dpp %0, %0, %0 row_bcast:15 row_mask:0xa bank_mask:0xf"
                   : "+v"(t3[2]));
      // keep the last DPP adds ahead of the branch (sunk into it, an add
      // could no longer take its operand through DPP)
      asm volatile("" : "+v"(u), "+v"(t3[2]));
      // one atomic instruction: lanes 7 + 8k add the eight totals of u, lanes
      // 22 and 54 (rows 1 and 3 of t3[2]) fields 8 and 9
      const bool lane_u = (lane & 7) == 7, lane_t = (lane & 31) == 22;
      if (lane_u || lane_t) {
        const int row = lane >> 4;
        const int sub = row == 1 ? 2 : (row == 2 ? 1 : row);
        const int field = lane_u ? ((lane & 8) ? 4 : 0) + sub : 8 + (row >> 1);
        atomicAdd(grad2d + size_t(__float_as_uint(g2.w)) * kGradFloats + field, lane_u ? u : t3[2]);
      }
    };
    if (hi <= stop_min) {
      for (int j = int(cnt) - 1; j >= 0; --j) record(std::false_type{}, j);
    } else {
      for (int j = int(cnt) - 1; j >= 0; --j) record(std::true_type{}, j);
    }
    hi = lo;
  }
}

// grad_dirty: set, so that a later backward pass over the same binning
// clears the record gradients first.
template <int TW, int TH, int BATCH>
__global__ void __launch_bounds__(64) raster_bwd_kernel(
    const float* __restrict__ records, const uint32_t* __restrict__ values,
    const uint32_t* __restrict__ ranges, const DevView* __restrict__ views, int n_views,
    uint32_t n_tiles, const uint32_t* __restrict__ order, uint32_t* __restrict__ work,
    uint32_t* __restrict__ grad_dirty,
    const float* __restrict__ t_ws,
    const uint32_t* __restrict__ ncontrib, const float* __restrict__ d_image,
    const float* __restrict__ d_tfinal, const float* __restrict__ l1_image,
    const float* __restrict__ l1_target, float l1_scale, float* __restrict__ grad2d) {
  __shared__ float4 s0[BATCH], s1[BATCH], s2[BATCH];
  if (blockIdx.x == 0 && threadIdx.x == 0) *grad_dirty = 1u;
  for (uint32_t q = next_tile(work, true); q < n_tiles; q = next_tile(work, false)) {
    const uint32_t tile = order[q];
    if (d_tfinal)
      raster_bwd_tile<TW, TH, BATCH, true>(tile, s0, s1, s2, records, values, ranges, views,
                                           n_views, t_ws, ncontrib, d_image, d_tfinal, l1_image,
                                           l1_target, l1_scale, grad2d);
    else
      raster_bwd_tile<TW, TH, BATCH, false>(tile, s0, s1, s2, records, values, ranges, views,
                                            n_views, t_ws, ncontrib, d_image, d_tfinal, l1_image,
                                            l1_target, l1_scale, grad2d);
  }
}

__global__ void reset_counter_kernel(uint32_t* __restrict__ c) {
  if (threadIdx.x == 0) *c = 0u;
}

// Launch geometry: one wavefront per tile (grid = tiles), or a persistent
// grid of `persistent_blocks` wavefronts taking tiles from a queue; either
// way the q-th tile handed out is order[q] (the binning's order, longest
// tiles first).
struct RasterLaunch {
  uint32_t n_tiles;
  uint32_t* work;            // queue counter, or nullptr
  uint32_t grid;
  const uint32_t* order;
};

static RasterLaunch raster_geometry(uint32_t n_tiles, uint32_t* work, uint32_t persistent_blocks,
                                    const uint32_t* order, hipStream_t st) {
  RasterLaunch g{n_tiles, nullptr, n_tiles, order};
  if (work && persistent_blocks > 0 && persistent_blocks < n_tiles) {
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, st, work);
    g.work = work;
    g.grid = persistent_blocks;
  }
  return g;
}

template <int TW, int TH, int BATCH>
static hipError_t raster_fwd_t(const RasterLaunch& g, const float* records, const uint32_t* values,
                               const uint32_t* ranges, const DevView* views, int n_views,
                               float* image, float* t_ws, float* t_user, uint32_t* ncontrib,
                               hipStream_t st) {
  hipLaunchKernelGGL((raster_fwd_kernel<TW, TH, BATCH>), dim3(g.grid), dim3(64), 0, st, records,
                     values, ranges, views, n_views, g.n_tiles, g.order, g.work, image, t_ws,
                     t_user, ncontrib);
  return hipGetLastError();
}

template <int TW, int TH, int BATCH>
static hipError_t raster_bwd_t(const RasterLaunch& g, uint32_t* grad_dirty, const float* records,
                               const uint32_t* values, const uint32_t* ranges,
                               const DevView* views, int n_views,
                               const float* t_ws, const uint32_t* ncontrib, const float* d_image,
                               const float* d_tfinal, const float* l1_image,
                               const float* l1_target, float l1_scale, float* grad2d,
                               hipStream_t st) {
  hipLaunchKernelGGL((raster_bwd_kernel<TW, TH, BATCH>), dim3(g.grid), dim3(64), 0, st, records,
                     values, ranges, views, n_views, g.n_tiles, g.order, g.work, grad_dirty, t_ws,
                     ncontrib, d_image, d_tfinal, l1_image, l1_target, l1_scale, grad2d);
  return hipGetLastError();
}

#define UBS_TILE_DISPATCH(FN, ...)                                                     \
  do {                                                                                 \
    const int bd = batch <= 64 ? 64 : (batch <= 128 ? 128 : 256);                      \
    if (tw == 16 && th == 16) {                                                        \
      if (bd == 64) return FN<16, 16, 64>(__VA_ARGS__);                                \
      if (bd == 128) return FN<16, 16, 128>(__VA_ARGS__);                              \
      return FN<16, 16, 256>(__VA_ARGS__);                                             \
    }                                                                                  \
    if (tw == 16 && th == 8) {                                                         \
      if (bd == 64) return FN<16, 8, 64>(__VA_ARGS__);                                 \
      if (bd == 128) return FN<16, 8, 128>(__VA_ARGS__);                               \
      return FN<16, 8, 256>(__VA_ARGS__);                                              \
    }                                                                                  \
    if (tw == 8 && th == 8) {                                                          \
      if (bd == 64) return FN<8, 8, 64>(__VA_ARGS__);                                  \
      if (bd == 128) return FN<8, 8, 128>(__VA_ARGS__);                                \
      return FN<8, 8, 256>(__VA_ARGS__);                                               \
    }                                                                                  \
    if (tw == 32 && th == 16) {                                                        \
      if (bd == 64) return FN<32, 16, 64>(__VA_ARGS__);                                \
      if (bd == 128) return FN<32, 16, 128>(__VA_ARGS__);                              \
      return FN<32, 16, 256>(__VA_ARGS__);                                             \
    }                                                                                  \
    return hipErrorInvalidValue;                                                       \
  } while (0)

hipError_t launch_raster_fwd(int tw, int th, int batch, uint32_t persistent_blocks,
                             uint32_t* work, const float* records, const uint32_t* values,
                             const uint32_t* ranges, const uint32_t* order,
                             const DevView* views, int n_views,
                             uint32_t n_tiles, float* image, float* t_ws, float* t_user,
                             uint32_t* ncontrib, hipStream_t st) {
  if (n_tiles == 0) return hipSuccess;
  const RasterLaunch g = raster_geometry(n_tiles, work, persistent_blocks, order, st);
  UBS_TILE_DISPATCH(raster_fwd_t, g, records, values, ranges, views, n_views, image, t_ws, t_user,
                    ncontrib, st);
}

hipError_t launch_raster_bwd(int tw, int th, int batch, uint32_t persistent_blocks,
                             uint32_t* work, uint32_t* grad_dirty, const float* records,
                             const uint32_t* values,
                             const uint32_t* ranges, const uint32_t* order,
                             const DevView* views, int n_views,
                             uint32_t n_tiles, const float* t_ws, const uint32_t* ncontrib,
                             const float* d_image, const float* d_tfinal, const float* l1_image,
                             const float* l1_target, float l1_scale, float* grad2d,
                             hipStream_t st) {
  if (n_tiles == 0) return hipSuccess;
  const RasterLaunch g = raster_geometry(n_tiles, work, persistent_blocks, order, st);
  UBS_TILE_DISPATCH(raster_bwd_t, g, grad_dirty, records, values, ranges, views, n_views, t_ws,
                    ncontrib, d_image, d_tfinal, l1_image, l1_target, l1_scale, grad2d, st);
}

}  // namespace ubs
