// Per-primitive math of Universal Beta Splatting, forward and adjoint.
//
// Forward (Section 4.2, 4.3 and the projection of Section 3):
//   Sigma = L L^T with L = [[R_x diag(s_x), 0], [L_qx, L_q]]
//     -> Sigma_x = M M^T, Sigma_xq = M L_qx^T, Sigma_q = L_qx L_qx^T + L_q L_q^T
//        (M = R_x diag(s_x))
//   q = d, [t, d] or [t, d, e] (e: the view's query values beyond 7-D),
//   d = unit(mu_x - camera centre); v = q - mu_q
//   Lhat = chol(Sigma_q); w = Lhat^-1 v;
//   o(q) = o prod_i (1 - tanh(w_i^2))^(4 exp(b_qi))
//   bt_i = min(exp(b_qi), 1); K = Sigma_xq Sigma_q^-1
//   mu_c = mu_x + K diag(bt) v; Sigma_c = Sigma_x - sym(K diag(bt) Sigma_qx)
//   p = W mu_c + t; Sigma' = J W Sigma_c W^T J^T + 0.3 I; conic = Sigma'^-1
//   rho = 1 - (255 o(q))^(-1/beta_x), beta_x = 4 exp(b_x)
// Adjoint: reverse of the above, written by hand.  The Cholesky adjoint is
//   Sigma_bar = sym(Lhat^-T Phi(Lhat^T Lhat_bar) Lhat^-1), Phi = lower
//   triangle with the diagonal halved (Murray 2016).
#pragma once

#include "ubs_internal.hpp"

namespace ubs {

template <typename T> __device__ __forceinline__ T m_exp(T x);
template <> __device__ __forceinline__ float m_exp<float>(float x) { return expf(x); }
template <> __device__ __forceinline__ double m_exp<double>(double x) { return exp(x); }
template <typename T> __device__ __forceinline__ T m_sqrt(T x);
template <> __device__ __forceinline__ float m_sqrt<float>(float x) { return sqrtf(x); }
template <> __device__ __forceinline__ double m_sqrt<double>(double x) { return sqrt(x); }
// 1 / sqrt(x): where both sqrt(x) and its reciprocal are needed, sqrt(x) is
// taken as x * rsqrt(x) (one library call instead of a root and a division)
template <typename T> __device__ __forceinline__ T m_rsqrt(T x);
template <> __device__ __forceinline__ float m_rsqrt<float>(float x) { return rsqrtf(x); }
template <> __device__ __forceinline__ double m_rsqrt<double>(double x) { return rsqrt(x); }

// Scalar factors of the opacity (the modulation terms, o(q), beta_x, rho)
// are well conditioned in their arguments, so they are evaluated in float32
// whatever T is; the linear algebra of the conditioning stays in T.
__device__ __forceinline__ float s_exp(float x) { return expf(x); }
__device__ __forceinline__ float s_log1p_exp_m2(float x) { return log1pf(expf(-2.0f * x)); }
// 1 - y^(-1/beta) for y >= 1, as -expm1(-log(y) / beta) (no cancellation for
// y near 1)
__device__ __forceinline__ float s_rho(float y, float beta) { return -expm1f(-logf(y) / beta); }

template <int C> struct Cdim { static constexpr int V = C > 0 ? C : 1; };

// Raw parameters of one primitive (float32, as stored).
template <int C, int ROT>
struct Raw {
  float mu[3];
  float muq[Cdim<C>::V];
  float rq[4];
  float logs[3];
  float lqx[Cdim<C>::V][3];
  float lq[Cdim<C>::V][Cdim<C>::V];  // full lower triangle, diagonal as log
  float bx;
  float bq[Cdim<C>::V];
  float o;
  float rgb[3];
  bool finite;  // every loaded parameter is finite
};

// A primitive's parameters from get(row), the value in parameter row `row`
// (finite: every value read is finite).
template <int C, int ROT, typename Get>
__device__ __forceinline__ void load_raw_rows(Get get, Raw<C, ROT>& r) {
  const ParamRows pr = param_rows(C, ROT);
  bool fin = true;
  auto ld = [&](int row) {
    const float x = get(row);
    fin = fin && isfinite(x);
    return x;
  };
#pragma unroll
  for (int k = 0; k < 3; ++k) r.mu[k] = ld(pr.mu_x + k);
#pragma unroll
  for (int k = 0; k < C; ++k) r.muq[k] = ld(pr.mu_q + k);
#pragma unroll
  for (int k = 0; k < 4; ++k) r.rq[k] = (k < (ROT == UBS_ROT_QUAT ? 4 : 3)) ? ld(pr.rot + k) : 0.0f;
#pragma unroll
  for (int k = 0; k < 3; ++k) r.logs[k] = ld(pr.log_s + k);
#pragma unroll
  for (int a = 0; a < C; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) r.lqx[a][b] = ld(pr.lqx + 3 * a + b);
  int k = 0;
#pragma unroll
  for (int a = 0; a < C; ++a)
#pragma unroll
    for (int b = 0; b <= a; ++b) { r.lq[a][b] = ld(pr.lq + k); ++k; }
  r.bx = ld(pr.b_x);
#pragma unroll
  for (int k2 = 0; k2 < C; ++k2) r.bq[k2] = ld(pr.b_q + k2);
  r.o = ld(pr.o);
#pragma unroll
  for (int k2 = 0; k2 < 3; ++k2) r.rgb[k2] = ld(pr.rgb + k2);
  r.finite = fin;
}

// Primitive i of the component-major array P (row stride n), with streaming
// loads: each parameter is read once per launch.
template <int C, int ROT>
__device__ __forceinline__ void load_raw(const float* __restrict__ P, int64_t n, int64_t i,
                                         Raw<C, ROT>& r) {
  load_raw_rows<C, ROT>(
      [&](int row) { return __builtin_nontemporal_load(&P[int64_t(row) * n + i]); }, r);
}

// View-independent quantities of a primitive.
template <typename T, int C, int ROT>
struct Geo {
  T s[3];
  T M[3][3];                         // R diag(s)
  T Sx[3][3];
  T Sxq[3][Cdim<C>::V];
  T Lh[Cdim<C>::V][Cdim<C>::V];      // chol(Sigma_q)
  T Li[Cdim<C>::V][Cdim<C>::V];      // Lh^-1 (lower)
  T bt[Cdim<C>::V];                  // min(exp(b_q), 1); 1 without the Beta condition
  T e[Cdim<C>::V];                   // 4 exp(b_q); 1 without the Beta opacity
  bool ok;
  bool beta_cond, beta_opacity;      // the Beta modulations in use (Sec. 5.3 ablations)
};

// Ablation variants (Sec. 5.3), bits of the frame's tuning flags.
constexpr uint32_t kVarNoBetaCond = UBS_TUNE_NO_BETA_COND;
constexpr uint32_t kVarNoBetaOpacity = UBS_TUNE_NO_BETA_OPACITY;

// Activated L_q (lower triangular, diagonal exp of the stored log scale).
template <typename T, int C, int ROT>
__device__ __forceinline__ T lq_entry(const Raw<C, ROT>& r, int a, int b) {
  return b < a ? T(r.lq[a][b]) : (b == a ? m_exp<T>(T(r.lq[a][a])) : T(0));
}

template <typename T, int C, int ROT>
__device__ __forceinline__ void geo_forward(const Raw<C, ROT>& r, Geo<T, C, ROT>& g,
                                            uint32_t variant) {
  g.ok = r.finite;
  g.beta_cond = (variant & kVarNoBetaCond) == 0;
  g.beta_opacity = (variant & kVarNoBetaOpacity) == 0;
  struct { T R[3][3]; } gr;
  auto& R = gr.R;
  if (ROT == UBS_ROT_QUAT) {
    T w = r.rq[0], x = r.rq[1], y = r.rq[2], z = r.rq[3];
    T nn = w * w + x * x + y * y + z * z;
    T inv = m_rsqrt<T>(nn);
    if (!(nn > T(0))) g.ok = false;
    w *= inv; x *= inv; y *= inv; z *= inv;
    R[0][0] = T(1) - T(2) * (y * y + z * z);
    R[0][1] = T(2) * (x * y - w * z);
    R[0][2] = T(2) * (x * z + w * y);
    R[1][0] = T(2) * (x * y + w * z);
    R[1][1] = T(1) - T(2) * (x * x + z * z);
    R[1][2] = T(2) * (y * z - w * x);
    R[2][0] = T(2) * (x * z - w * y);
    R[2][1] = T(2) * (y * z + w * x);
    R[2][2] = T(1) - T(2) * (x * x + y * y);
  } else {
    T w1 = r.rq[0], w2 = r.rq[1], w3 = r.rq[2];
    R[0][0] = T(1); R[0][1] = -w3;  R[0][2] = w2;
    R[1][0] = w3;   R[1][1] = T(1); R[1][2] = -w1;
    R[2][0] = -w2;  R[2][1] = w1;   R[2][2] = T(1);
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) g.s[k] = m_exp<T>(T(r.logs[k]));
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) g.M[a][b] = R[a][b] * g.s[b];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b <= a; ++b) {
      g.Sx[a][b] = g.M[a][0] * g.M[b][0] + g.M[a][1] * g.M[b][1] + g.M[a][2] * g.M[b][2];
      g.Sx[b][a] = g.Sx[a][b];
    }
  if constexpr (C > 0) {
    T Lq[Cdim<C>::V][Cdim<C>::V];
#pragma unroll
    for (int a = 0; a < C; ++a)
#pragma unroll
      for (int b = 0; b < C; ++b) Lq[a][b] = lq_entry<T, C, ROT>(r, a, b);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int k = 0; k < C; ++k)
        g.Sxq[a][k] = g.M[a][0] * T(r.lqx[k][0]) + g.M[a][1] * T(r.lqx[k][1]) + g.M[a][2] * T(r.lqx[k][2]);
    T Sq[Cdim<C>::V][Cdim<C>::V];
#pragma unroll
    for (int a = 0; a < C; ++a)
#pragma unroll
      for (int b = 0; b < C; ++b) {
        T acc = T(r.lqx[a][0]) * T(r.lqx[b][0]) + T(r.lqx[a][1]) * T(r.lqx[b][1]) +
                T(r.lqx[a][2]) * T(r.lqx[b][2]);
#pragma unroll
        for (int k = 0; k < C; ++k) acc += Lq[a][k] * Lq[b][k];
        Sq[a][b] = acc;
      }
    // Cholesky of Sigma_q (lower, positive diagonal)
#pragma unroll
    for (int j = 0; j < C; ++j) {
      T d = Sq[j][j];
#pragma unroll
      for (int k = 0; k < j; ++k) d -= g.Lh[j][k] * g.Lh[j][k];
      if (!(d > T(0))) { g.ok = false; d = T(1); }
      T inv = m_rsqrt<T>(d);
      g.Lh[j][j] = d * inv;
      g.Li[j][j] = inv;
#pragma unroll
      for (int i = j + 1; i < C; ++i) {
        T acc = Sq[i][j];
#pragma unroll
        for (int k = 0; k < j; ++k) acc -= g.Lh[i][k] * g.Lh[j][k];
        g.Lh[i][j] = acc * inv;
      }
#pragma unroll
      for (int i = 0; i < j; ++i) g.Lh[i][j] = T(0);
    }
    // inverse of the lower factor
#pragma unroll
    for (int j = 0; j < C; ++j) {
#pragma unroll
      for (int i = 0; i < C; ++i) {
        if (i < j) { g.Li[i][j] = T(0); continue; }
        if (i == j) continue;   // 1 / Lh[i][i], set by the factorisation
        T acc = T(0);
#pragma unroll
        for (int k = j; k < i; ++k) acc += g.Lh[i][k] * g.Li[k][j];
        g.Li[i][j] = -acc * g.Li[i][i];
      }
    }
#pragma unroll
    for (int k = 0; k < C; ++k) {
      T eb = m_exp<T>(T(r.bq[k]));
      g.bt[k] = (g.beta_cond && r.bq[k] < 0.0f) ? eb : T(1);
      g.e[k] = g.beta_opacity ? T(4) * eb : T(1);
    }
  }
}

// Per-view forward state kept for the adjoint.
template <typename T, int C>
struct ViewState {
  T dir[3];              // unit query direction
  T dist;                // |mu_x - camera centre|
  T v[Cdim<C>::V];       // q - mu_q
  T w[Cdim<C>::V];       // Lh^-1 v
  T ell[Cdim<C>::V];     // log(1 - tanh(w^2))
  T oq;                  // o(q)
  T mu_c[3];
  T Sc[3][3];
  T p[3];                // camera-frame mean
  T Tm[2][3];            // J W
  T Sp00, Sp01, Sp11;
  T ca, cb, cc;          // conic
  T mx, my;              // projected mean (pixels)
  T beta;
  T rho;
  bool live;
};

template <typename T, int C, int ROT>
__device__ __forceinline__ void view_forward(const Raw<C, ROT>& r, const Geo<T, C, ROT>& g,
                                             const DevView& V, ViewState<T, C>& s) {
  bool live = g.ok;
  T oq = T(r.o);
  T mu_c[3] = {T(r.mu[0]), T(r.mu[1]), T(r.mu[2])};
  T Sc[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) Sc[a][b] = g.Sx[a][b];
  if constexpr (C > 0) {
    T dv[3] = {T(r.mu[0]) - T(V.cam[0]), T(r.mu[1]) - T(V.cam[1]), T(r.mu[2]) - T(V.cam[2])};
    T dd = dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2];
    T inv = m_rsqrt<T>(dd);
    T dist = dd * inv;
    s.dist = dist;
#pragma unroll
    for (int k = 0; k < 3; ++k) s.dir[k] = dv[k] * inv;
    T q[Cdim<C>::V];
    if constexpr (C >= 4) {   // [t, d, query values of the view beyond 7-D]
      q[0] = T(V.time); q[1] = s.dir[0]; q[2] = s.dir[1]; q[3] = s.dir[2];
#pragma unroll
      for (int k = 4; k < C; ++k) q[k] = T(V.query[k - 4]);
    } else if constexpr (C == 3) {
      q[0] = s.dir[0]; q[1] = s.dir[1]; q[2] = s.dir[2];
    } else {
#pragma unroll
      for (int k = 0; k < C; ++k) q[k] = s.dir[k];   // C < 3: leading direction components
    }
#pragma unroll
    for (int k = 0; k < C; ++k) s.v[k] = q[k] - T(r.muq[k]);
    // whitening and opacity: log(1 - tanh x) = log 2 - 2x - log1p(exp(-2x))
    T lsum = T(0);
#pragma unroll
    for (int i = 0; i < C; ++i) {
      T acc = T(0);
#pragma unroll
      for (int k = 0; k <= i; ++k) acc += g.Li[i][k] * s.v[k];
      s.w[i] = acc;
      T x = acc * acc;
      // Gaussian opacity (ablation): e = 1 and ell = -w^2 / 2
      s.ell[i] = g.beta_opacity
                     ? T(0.69314718055994530942) - T(2) * x - T(s_log1p_exp_m2(float(x)))
                     : T(-0.5) * x;
      lsum += g.e[i] * s.ell[i];
    }
    oq = T(r.o) * T(s_exp(float(lsum)));
    // conditioning: K = Sigma_xq Sigma_q^-1 = (Sigma_xq Lh^-T) Lh^-1
    T K[3][Cdim<C>::V];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      T A[Cdim<C>::V];
#pragma unroll
      for (int k = 0; k < C; ++k) {
        T acc = T(0);
#pragma unroll
        for (int m = 0; m <= k; ++m) acc += g.Sxq[a][m] * g.Li[k][m];
        A[k] = acc;
      }
#pragma unroll
      for (int k = 0; k < C; ++k) {
        T acc = T(0);
#pragma unroll
        for (int m = k; m < C; ++m) acc += A[m] * g.Li[m][k];
        K[a][k] = acc;
      }
    }
    T Dv[Cdim<C>::V];
#pragma unroll
    for (int k = 0; k < C; ++k) Dv[k] = g.bt[k] * s.v[k];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      T acc = T(0);
#pragma unroll
      for (int k = 0; k < C; ++k) acc += K[a][k] * Dv[k];
      mu_c[a] += acc;
    }
    T X[3][3];   // K diag(bt) Sigma_qx
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        T acc = T(0);
#pragma unroll
        for (int k = 0; k < C; ++k) acc += K[a][k] * g.bt[k] * g.Sxq[b][k];
        X[a][b] = acc;
      }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) Sc[a][b] -= T(0.5) * (X[a][b] + X[b][a]);
  }
  s.oq = oq;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    s.mu_c[a] = mu_c[a];
#pragma unroll
    for (int b = 0; b < 3; ++b) s.Sc[a][b] = Sc[a][b];
  }
  // projection
  T p[3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
    p[a] = T(V.R[3 * a]) * mu_c[0] + T(V.R[3 * a + 1]) * mu_c[1] + T(V.R[3 * a + 2]) * mu_c[2] + T(V.t[a]);
#pragma unroll
  for (int a = 0; a < 3; ++a) s.p[a] = p[a];
  if (!(p[2] > T(kNear))) live = false;
  T z = p[2] > T(kNear) ? p[2] : T(1);
  T iz = T(1) / z;
  T fx = T(V.fx), fy = T(V.fy);
  T J00 = fx * iz, J02 = -fx * p[0] * iz * iz;
  T J11 = fy * iz, J12 = -fy * p[1] * iz * iz;
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    s.Tm[0][b] = J00 * T(V.R[b]) + J02 * T(V.R[6 + b]);
    s.Tm[1][b] = J11 * T(V.R[3 + b]) + J12 * T(V.R[6 + b]);
  }
  T U[2][3];   // Tm Sc
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      U[a][b] = s.Tm[a][0] * Sc[0][b] + s.Tm[a][1] * Sc[1][b] + s.Tm[a][2] * Sc[2][b];
  s.Sp00 = U[0][0] * s.Tm[0][0] + U[0][1] * s.Tm[0][1] + U[0][2] * s.Tm[0][2] + T(kDilation);
  s.Sp01 = U[0][0] * s.Tm[1][0] + U[0][1] * s.Tm[1][1] + U[0][2] * s.Tm[1][2];
  s.Sp11 = U[1][0] * s.Tm[1][0] + U[1][1] * s.Tm[1][1] + U[1][2] * s.Tm[1][2] + T(kDilation);
  T det = s.Sp00 * s.Sp11 - s.Sp01 * s.Sp01;
  if (!(det > T(0)) || !(s.Sp00 > T(0)) || !(s.Sp11 > T(0))) live = false;
  T idet = T(1) / (det > T(0) ? det : T(1));
  s.mx = fx * p[0] * iz + T(V.cx);
  s.my = fy * p[1] * iz + T(V.cy);
  s.ca = s.Sp11 * idet;
  s.cb = -s.Sp01 * idet;
  s.cc = s.Sp00 * idet;
  s.beta = T(4) * T(s_exp(r.bx));
  if (!(oq >= T(kAlphaMin))) live = false;
  T oqs = oq >= T(kAlphaMin) ? oq : T(1);
  s.rho = T(s_rho(float(T(255) * oqs), float(s.beta)));
  if (!(s.rho > T(0))) live = false;
  s.live = live;
}

// Gradients w.r.t. the view-independent quantities, summed over views
// (accumulated in float32: each view's contribution is evaluated in T).
template <typename T, int C>
struct GeoGrad {
  float Sx[3][3];
  float Sxq[3][Cdim<C>::V];
  float Z[Cdim<C>::V][Cdim<C>::V];   // w.r.t. Sigma_q^-1 (symmetric part used)
  float Lh[Cdim<C>::V][Cdim<C>::V];  // w.r.t. chol(Sigma_q) (lower)
  float mu[3], muq[Cdim<C>::V], bq[Cdim<C>::V], bt[Cdim<C>::V];
  float bx, o, rgb[3];
};

template <typename T, int C>
__device__ __forceinline__ void geograd_zero(GeoGrad<T, C>& G) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
#pragma unroll
    for (int b = 0; b < 3; ++b) G.Sx[a][b] = T(0);
#pragma unroll
    for (int k = 0; k < C; ++k) G.Sxq[a][k] = T(0);
    G.mu[a] = T(0);
    G.rgb[a] = T(0);
  }
#pragma unroll
  for (int a = 0; a < C; ++a) {
#pragma unroll
    for (int b = 0; b < C; ++b) { G.Z[a][b] = T(0); G.Lh[a][b] = T(0); }
    G.muq[a] = G.bq[a] = G.bt[a] = T(0);
  }
  G.bx = G.o = T(0);
}

// Adjoint of view_forward for one view.  gr: d loss / d record fields
// (mx, my, a, b, c, o(q), beta, r, g, b).
template <typename T, int C, int ROT>
__device__ __forceinline__ void view_backward(const Raw<C, ROT>& r, const Geo<T, C, ROT>& g,
                                              const DevView& V, const ViewState<T, C>& s,
                                              const float* gr, GeoGrad<T, C>& G) {
  G.rgb[0] += T(gr[7]);
  G.rgb[1] += T(gr[8]);
  G.rgb[2] += T(gr[9]);
  G.bx += T(gr[6]) * s.beta;
  // conic = Sigma'^-1:  G_Sigma' = -A G_A A with G_A = [[ga, gb/2], [gb/2, gc]]
  T a = s.ca, b = s.cb, c = s.cc;
  T ga = T(gr[2]), gb = T(0.5) * T(gr[3]), gc = T(gr[4]);
  T P00 = a * ga + b * gb, P01 = a * gb + b * gc;   // A G_A
  T P10 = b * ga + c * gb, P11 = b * gb + c * gc;
  T G00 = -(P00 * a + P01 * b);
  T G01 = -(P00 * b + P01 * c);
  T G11 = -(P10 * b + P11 * c);
  // Sigma' = Tm Sc Tm^T + 0.3 I
  T Gs[2][2] = {{G00, G01}, {G01, G11}};
  T GT[2][3];   // Gs Tm
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) GT[i][j] = Gs[i][0] * s.Tm[0][j] + Gs[i][1] * s.Tm[1][j];
  T Gc[3][3];   // Tm^T Gs Tm
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Gc[i][j] = s.Tm[0][i] * GT[0][j] + s.Tm[1][i] * GT[1][j];
  T GTm[2][3];  // 2 Gs Tm Sc
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      GTm[i][j] = T(2) * (GT[i][0] * s.Sc[0][j] + GT[i][1] * s.Sc[1][j] + GT[i][2] * s.Sc[2][j]);
  // Tm = J W  ->  G_J = GTm W^T  (W row-major in V.R)
  T GJ00 = GTm[0][0] * T(V.R[0]) + GTm[0][1] * T(V.R[1]) + GTm[0][2] * T(V.R[2]);
  T GJ02 = GTm[0][0] * T(V.R[6]) + GTm[0][1] * T(V.R[7]) + GTm[0][2] * T(V.R[8]);
  T GJ11 = GTm[1][0] * T(V.R[3]) + GTm[1][1] * T(V.R[4]) + GTm[1][2] * T(V.R[5]);
  T GJ12 = GTm[1][0] * T(V.R[6]) + GTm[1][1] * T(V.R[7]) + GTm[1][2] * T(V.R[8]);
  T z = s.p[2];
  T iz = T(1) / z, iz2 = iz * iz, iz3 = iz2 * iz;
  T fx = T(V.fx), fy = T(V.fy);
  T gmx = T(gr[0]), gmy = T(gr[1]);
  T gp[3];
  gp[0] = gmx * fx * iz + GJ02 * (-fx * iz2);
  gp[1] = gmy * fy * iz + GJ12 * (-fy * iz2);
  gp[2] = gmx * (-fx * s.p[0] * iz2) + gmy * (-fy * s.p[1] * iz2) + GJ00 * (-fx * iz2) +
          GJ02 * (T(2) * fx * s.p[0] * iz3) + GJ11 * (-fy * iz2) + GJ12 * (T(2) * fy * s.p[1] * iz3);
  T gmc[3];
#pragma unroll
  for (int j = 0; j < 3; ++j)
    gmc[j] = T(V.R[j]) * gp[0] + T(V.R[3 + j]) * gp[1] + T(V.R[6 + j]) * gp[2];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    G.mu[i] += gmc[i];
#pragma unroll
    for (int j = 0; j < 3; ++j) G.Sx[i][j] += Gc[i][j];
  }
  T goq = T(gr[5]);
  if constexpr (C == 0) {
    G.o += goq;
  } else {
    // ---- conditioning ----
    // Z = Sigma_q^-1 = Li^T Li
    T Z[Cdim<C>::V][Cdim<C>::V];
#pragma unroll
    for (int i = 0; i < C; ++i)
#pragma unroll
      for (int j = 0; j < C; ++j) {
        T acc = T(0);
#pragma unroll
        for (int k = 0; k < C; ++k) acc += g.Li[k][i] * g.Li[k][j];
        Z[i][j] = acc;
      }
    T Dv[Cdim<C>::V], ZDv[Cdim<C>::V], u[Cdim<C>::V], Zu[Cdim<C>::V];
#pragma unroll
    for (int k = 0; k < C; ++k) Dv[k] = g.bt[k] * s.v[k];
#pragma unroll
    for (int k = 0; k < C; ++k) {
      T acc = T(0), acc2 = T(0);
#pragma unroll
      for (int m = 0; m < C; ++m) acc += Z[k][m] * Dv[m];
      ZDv[k] = acc;
#pragma unroll
      for (int m = 0; m < 3; ++m) acc2 += g.Sxq[m][k] * gmc[m];
      u[k] = acc2;
    }
#pragma unroll
    for (int k = 0; k < C; ++k) {
      T acc = T(0);
#pragma unroll
      for (int m = 0; m < C; ++m) acc += Z[k][m] * u[m];
      Zu[k] = acc;
    }
    // Q = Sxq^T G Sxq ; GS = G Sxq
    T GS[3][Cdim<C>::V];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int k = 0; k < C; ++k)
        GS[i][k] = Gc[i][0] * g.Sxq[0][k] + Gc[i][1] * g.Sxq[1][k] + Gc[i][2] * g.Sxq[2][k];
    T Q[Cdim<C>::V][Cdim<C>::V];
#pragma unroll
    for (int k = 0; k < C; ++k)
#pragma unroll
      for (int l = 0; l < C; ++l)
        Q[k][l] = g.Sxq[0][k] * GS[0][l] + g.Sxq[1][k] * GS[1][l] + g.Sxq[2][k] * GS[2][l];
    // G_Sxq += gmc (Z Dv)^T - G Sxq (Z D + D Z)
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int l = 0; l < C; ++l) {
        T acc = gmc[i] * ZDv[l];
#pragma unroll
        for (int k = 0; k < C; ++k) acc -= GS[i][k] * (Z[k][l] * g.bt[l] + g.bt[k] * Z[k][l]);
        G.Sxq[i][l] += acc;
      }
    // G_Z += sym(u Dv^T) - (Q D + D Q)/2
#pragma unroll
    for (int k = 0; k < C; ++k)
#pragma unroll
      for (int l = 0; l < C; ++l)
        G.Z[k][l] += T(0.5) * (u[k] * Dv[l] + Dv[k] * u[l]) - T(0.5) * (Q[k][l] * g.bt[l] + g.bt[k] * Q[k][l]);
    // d bt_k += (Z u)_k v_k - (Z Q)_kk ;  g_v += bt (Z u)
    T gv[Cdim<C>::V];
#pragma unroll
    for (int k = 0; k < C; ++k) {
      T zq = T(0);
#pragma unroll
      for (int m = 0; m < C; ++m) zq += Z[k][m] * Q[m][k];
      G.bt[k] += Zu[k] * s.v[k] - zq;
      gv[k] = g.bt[k] * Zu[k];
    }
    // ---- opacity ----  o(q) = o exp(sum e_i ell_i),  ell = log(1 - tanh(w^2))
    T prod;
    {
      T lsum = T(0);
#pragma unroll
      for (int i = 0; i < C; ++i) lsum += g.e[i] * s.ell[i];
      prod = T(s_exp(float(lsum)));
    }
    G.o += goq * prod;
    T gw[Cdim<C>::V];
#pragma unroll
    for (int i = 0; i < C; ++i) {
      if (g.beta_opacity) {
        G.bq[i] += goq * s.oq * s.ell[i] * g.e[i];
        T x = s.w[i] * s.w[i];
        T th = T(tanhf(float(x)));
        gw[i] = goq * s.oq * g.e[i] * (-(T(1) + th)) * T(2) * s.w[i];
      } else {
        gw[i] = -goq * s.oq * s.w[i];   // d(-w^2/2)/dw; no b_q dependence
      }
    }
    // w = Li v:  g_v += Li^T gw ; G_Lh += -tril((Li^T gw) w^T)
    T ut[Cdim<C>::V];
#pragma unroll
    for (int k = 0; k < C; ++k) {
      T acc = T(0);
#pragma unroll
      for (int i = k; i < C; ++i) acc += g.Li[i][k] * gw[i];
      ut[k] = acc;
      gv[k] += acc;
    }
#pragma unroll
    for (int i = 0; i < C; ++i)
#pragma unroll
      for (int j = 0; j <= i; ++j) G.Lh[i][j] -= ut[i] * s.w[j];
    // v = q - mu_q ; q = [t, d] or d ; d = unit(mu_x - cam)
#pragma unroll
    for (int k = 0; k < C; ++k) G.muq[k] -= gv[k];
    T gd[3] = {T(0), T(0), T(0)};
    if constexpr (C >= 4) { gd[0] = gv[1]; gd[1] = gv[2]; gd[2] = gv[3]; }
    else if constexpr (C == 3) { gd[0] = gv[0]; gd[1] = gv[1]; gd[2] = gv[2]; }
    else {
#pragma unroll
      for (int k = 0; k < C; ++k) gd[k] = gv[k];
    }
    T dg = s.dir[0] * gd[0] + s.dir[1] * gd[1] + s.dir[2] * gd[2];
    T idist = T(1) / s.dist;
#pragma unroll
    for (int k = 0; k < 3; ++k) G.mu[k] += (gd[k] - s.dir[k] * dg) * idist;
  }
}

// Final chain from the view-independent gradients to the raw parameters.
// out[] is indexed by parameter row.
template <typename T, int C, int ROT>
__device__ __forceinline__ void geo_backward(const Raw<C, ROT>& r, const Geo<T, C, ROT>& g,
                                             const GeoGrad<T, C>& G, float* out) {
  const ParamRows pr = param_rows(C, ROT);
  T GM[3][3];
  // Sigma_x = M M^T (G_Sx symmetric): G_M = 2 G_Sx M
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      GM[i][j] = (G.Sx[i][0] + G.Sx[0][i]) * g.M[0][j] + (G.Sx[i][1] + G.Sx[1][i]) * g.M[1][j] +
                 (G.Sx[i][2] + G.Sx[2][i]) * g.M[2][j];
  if constexpr (C > 0) {
    T Z[Cdim<C>::V][Cdim<C>::V];
#pragma unroll
    for (int i = 0; i < C; ++i)
#pragma unroll
      for (int j = 0; j < C; ++j) {
        T acc = T(0);
#pragma unroll
        for (int k = 0; k < C; ++k) acc += g.Li[k][i] * g.Li[k][j];
        Z[i][j] = acc;
      }
    // G_Sq = -Z sym(G_Z) Z + sym(Li^T Phi(Lh^T G_Lh) Li)
    T GSq[Cdim<C>::V][Cdim<C>::V];
    {
      T A1[Cdim<C>::V][Cdim<C>::V];
#pragma unroll
      for (int i = 0; i < C; ++i)
#pragma unroll
        for (int j = 0; j < C; ++j) {
          T acc = T(0);
#pragma unroll
          for (int k = 0; k < C; ++k) acc += Z[i][k] * T(0.5) * (G.Z[k][j] + G.Z[j][k]);
          A1[i][j] = acc;
        }
#pragma unroll
      for (int i = 0; i < C; ++i)
#pragma unroll
        for (int j = 0; j < C; ++j) {
          T acc = T(0);
#pragma unroll
          for (int k = 0; k < C; ++k) acc += A1[i][k] * Z[k][j];
          GSq[i][j] = -acc;
        }
      T Pm[Cdim<C>::V][Cdim<C>::V];   // Phi(Lh^T G_Lh)
#pragma unroll
      for (int i = 0; i < C; ++i)
#pragma unroll
        for (int j = 0; j < C; ++j) {
          if (j > i) { Pm[i][j] = T(0); continue; }
          T acc = T(0);
#pragma unroll
          for (int k = 0; k < C; ++k) acc += g.Lh[k][i] * G.Lh[k][j];
          Pm[i][j] = (i == j) ? T(0.5) * acc : acc;
        }
      T B1[Cdim<C>::V][Cdim<C>::V];   // Li^T Pm
#pragma unroll
      for (int i = 0; i < C; ++i)
#pragma unroll
        for (int j = 0; j < C; ++j) {
          T acc = T(0);
#pragma unroll
          for (int k = 0; k < C; ++k) acc += g.Li[k][i] * Pm[k][j];
          B1[i][j] = acc;
        }
      T S1[Cdim<C>::V][Cdim<C>::V];   // B1 Li
#pragma unroll
      for (int i = 0; i < C; ++i)
#pragma unroll
        for (int j = 0; j < C; ++j) {
          T acc = T(0);
#pragma unroll
          for (int k = 0; k < C; ++k) acc += B1[i][k] * g.Li[k][j];
          S1[i][j] = acc;
        }
#pragma unroll
      for (int i = 0; i < C; ++i)
#pragma unroll
        for (int j = 0; j < C; ++j) GSq[i][j] += T(0.5) * (S1[i][j] + S1[j][i]);
    }
    // Sigma_q = Lqx Lqx^T + Lq Lq^T ; Sigma_xq = M Lqx^T
    T GSs[Cdim<C>::V][Cdim<C>::V];   // G_Sq + G_Sq^T
#pragma unroll
    for (int i = 0; i < C; ++i)
#pragma unroll
      for (int j = 0; j < C; ++j) GSs[i][j] = GSq[i][j] + GSq[j][i];
#pragma unroll
    for (int k = 0; k < C; ++k)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        T acc = T(0);
#pragma unroll
        for (int m = 0; m < C; ++m) acc += GSs[k][m] * T(r.lqx[m][j]);
#pragma unroll
        for (int m = 0; m < 3; ++m) acc += G.Sxq[m][k] * g.M[m][j];
        out[pr.lqx + 3 * k + j] = float(acc);
      }
    int idx = 0;
#pragma unroll
    for (int i = 0; i < C; ++i)
#pragma unroll
      for (int j = 0; j <= i; ++j) {
        T acc = T(0);
#pragma unroll
        for (int m = j; m < C; ++m) acc += GSs[i][m] * lq_entry<T, C, ROT>(r, m, j);
        out[pr.lq + idx] = float(i == j ? acc * lq_entry<T, C, ROT>(r, i, i) : acc);
        ++idx;
      }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        T acc = T(0);
#pragma unroll
        for (int k = 0; k < C; ++k) acc += G.Sxq[i][k] * T(r.lqx[k][j]);
        GM[i][j] += acc;
      }
#pragma unroll
    for (int k = 0; k < C; ++k) {
      out[pr.mu_q + k] = float(G.muq[k]);
      T gbq = G.bq[k];
      if (g.beta_cond && r.bq[k] < 0.0f) gbq += G.bt[k] * g.bt[k];
      out[pr.b_q + k] = float(gbq);
    }
  }
  // M = R diag(s)
  T GR[3][3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    T acc = T(0);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      GR[i][j] = GM[i][j] * g.s[j];
      acc += GM[i][j] * g.M[i][j];   // M = R diag(s): d/d log s_j = sum_i GM_ij R_ij s_j
    }
    out[pr.log_s + j] = float(acc);
  }
  if (ROT == UBS_ROT_QUAT) {
    T iq = m_rsqrt<T>(T(r.rq[0]) * T(r.rq[0]) + T(r.rq[1]) * T(r.rq[1]) +
                      T(r.rq[2]) * T(r.rq[2]) + T(r.rq[3]) * T(r.rq[3]));
    T w = T(r.rq[0]) * iq, x = T(r.rq[1]) * iq, y = T(r.rq[2]) * iq, z = T(r.rq[3]) * iq;
    T gw = T(2) * (-z * GR[0][1] + y * GR[0][2] + z * GR[1][0] - x * GR[1][2] - y * GR[2][0] + x * GR[2][1]);
    T gx = T(2) * (y * GR[0][1] + z * GR[0][2] + y * GR[1][0] - T(2) * x * GR[1][1] - w * GR[1][2] +
                   z * GR[2][0] + w * GR[2][1] - T(2) * x * GR[2][2]);
    T gy = T(2) * (-T(2) * y * GR[0][0] + x * GR[0][1] + w * GR[0][2] + x * GR[1][0] + z * GR[1][2] -
                   w * GR[2][0] + z * GR[2][1] - T(2) * y * GR[2][2]);
    T gz = T(2) * (-T(2) * z * GR[0][0] - w * GR[0][1] + x * GR[0][2] + w * GR[1][0] - T(2) * z * GR[1][1] +
                   y * GR[1][2] + x * GR[2][0] + y * GR[2][1]);
    T dotq = w * gw + x * gx + y * gy + z * gz;
    out[pr.rot + 0] = float((gw - w * dotq) * iq);
    out[pr.rot + 1] = float((gx - x * dotq) * iq);
    out[pr.rot + 2] = float((gy - y * dotq) * iq);
    out[pr.rot + 3] = float((gz - z * dotq) * iq);
  } else {
    out[pr.rot + 0] = float(GR[2][1] - GR[1][2]);
    out[pr.rot + 1] = float(GR[0][2] - GR[2][0]);
    out[pr.rot + 2] = float(GR[1][0] - GR[0][1]);
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    out[pr.mu_x + k] = float(G.mu[k]);
    out[pr.rgb + k] = float(G.rgb[k]);
  }
  out[pr.b_x] = float(G.bx);
  out[pr.o] = float(G.o);
}

}  // namespace ubs
