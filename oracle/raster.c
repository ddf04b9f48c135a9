/*
 * Oracle compositing, adjoint and binning reference -- plain C, float64.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline of the benchmark; never by the product path.  Shares no code
 * with the HIP kernels.
 *
 * Record format (one row of 12 doubles per primitive):
 *   mx my a b c rho o beta r g bl depth
 * mean (mx, my) in pixels, conic (a, b, c) = inverse 2-D covariance with the
 * quadratic form r = a dx^2 + 2 b dx dy + c dy^2 (the squared Mahalanobis
 * distance, Section 3 equation r), rho = support of the record (r <= rho),
 * o = conditioned opacity o(q), beta = spatial Beta exponent beta_x,
 * rgb colour, depth = camera-frame z.  A record with !(rho > 0) is culled.
 *
 * Per pixel (centre at x + 0.5, y + 0.5), with every live record taken in
 * ascending (depth, index) order and no tiles (Section 3 compositing):
 *   sigma = o (1 - r)^beta for r <= rho (Beta kernel, Section 3 / 4.3)
 *   alpha = min(0.99, sigma); skip if alpha < 1/255
 *   stop (excluding this record) once T (1 - alpha) < 1e-4
 *   C += c alpha T;  T *= (1 - alpha)
 * Readings: the 0.99 clamp, the 1/255 skip and the 1e-4 stop are the
 * standard-splatting conventions the paper defers to; background is black
 * (the caller adds bg * T_final).
 *
 * Ambiguity flags (bit mask per pixel) mark pixels whose result may
 * legitimately differ between this float64 evaluation and a float32 one:
 *   1  a record's r or alpha lies within a relative band of a threshold
 *   2  T (1 - alpha) lies within a relative band of 1e-4
 *   4  two consecutive contributors have depths within a relative band
 *   8  sigma lies within a relative band of the 0.99 clamp
 *   16 an "ambiguous" record (validity uncertain) may reach the pixel
 * amb[i] (when given) marks such records: 1 = its culling (near plane,
 * definiteness) is uncertain, so it may reach its whole support r < 1;
 * 2 = only o(q) >= 1/255 is uncertain (o(q) within band_opacity of it), so
 * it can add a contribution only where alpha may reach 1/255, i.e. at
 * r <= max(rho, 1 - (1 + band_opacity)^(-1/beta)).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ALPHA_MIN (1.0 / 255.0)
#define ALPHA_MAX 0.99
#define T_STOP 1e-4

typedef struct {
    double band_alpha, band_t, band_depth, band_clamp, band_opacity;
} bands_t;

static const double *g_depth;
static int cmp_depth(const void *pa, const void *pb)
{
    int ia = *(const int *)pa, ib = *(const int *)pb;
    double da = g_depth[ia], db = g_depth[ib];
    if (da < db) return -1;
    if (da > db) return 1;
    return (ia > ib) - (ia < ib);
}

/* Sort live record indices by (depth, index).  Returns the count. */
static int sorted_live(int n, const double *rec, const unsigned char *amb, int **out)
{
    int *idx = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    double *depth = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int m = 0;
    for (int i = 0; i < n; ++i) {
        depth[i] = rec[12 * (size_t)i + 11];
        if (rec[12 * (size_t)i + 5] > 0.0 || (amb && amb[i])) idx[m++] = i;
    }
    g_depth = depth;
    qsort(idx, (size_t)m, sizeof(int), cmp_depth);
    free(depth);
    *out = idx;
    return m;
}

/* Pixel rows touched by the r < 1 ellipse of a record (+1 px slack). */
static void row_span(const double *r, int H, int *y0, int *y1)
{
    double a = r[2], b = r[3], c = r[4];
    double det = a * c - b * b;
    if (!(det > 0.0) || !(a > 0.0)) { *y0 = 0; *y1 = H - 1; return; }
    double ey = sqrt(a / det);  /* sqrt of Sigma'_yy */
    double lo = floor(r[1] - ey - 1.5), hi = ceil(r[1] + ey + 0.5);
    *y0 = lo < 0 ? 0 : (lo > H ? H : (int)lo);
    *y1 = hi > H - 1 ? H - 1 : (hi < -1 ? -1 : (int)hi);
}

static void col_span(const double *r, int W, int *x0, int *x1)
{
    double a = r[2], b = r[3], c = r[4];
    double det = a * c - b * b;
    if (!(det > 0.0) || !(c > 0.0)) { *x0 = 0; *x1 = W - 1; return; }
    double ex = sqrt(c / det);  /* sqrt of Sigma'_xx */
    double lo = floor(r[0] - ex - 1.5), hi = ceil(r[0] + ex + 0.5);
    *x0 = lo < 0 ? 0 : (lo > W ? W : (int)lo);
    *x1 = hi > W - 1 ? W - 1 : (hi < -1 ? -1 : (int)hi);
}

typedef struct {
    int m;          /* live records */
    int *order;     /* [m] by (depth, index) */
    int *row_start; /* [H+1] CSR of per-row candidates (positions into order) */
    int *row_list;
} rows_t;

static void build_rows(int n, const double *rec, const unsigned char *amb, int H, rows_t *R)
{
    R->m = sorted_live(n, rec, amb, &R->order);
    R->row_start = (int *)calloc((size_t)H + 1, sizeof(int));
    for (int k = 0; k < R->m; ++k) {
        int y0, y1;
        row_span(rec + 12 * (size_t)R->order[k], H, &y0, &y1);
        for (int y = y0; y <= y1; ++y) R->row_start[y + 1]++;
    }
    for (int y = 0; y < H; ++y) R->row_start[y + 1] += R->row_start[y];
    R->row_list = (int *)malloc(sizeof(int) * (size_t)(R->row_start[H] > 0 ? R->row_start[H] : 1));
    int *fill = (int *)malloc(sizeof(int) * (size_t)(H > 0 ? H : 1));
    for (int y = 0; y < H; ++y) fill[y] = R->row_start[y];
    for (int k = 0; k < R->m; ++k) {  /* ascending k keeps each row list in depth order */
        int y0, y1;
        row_span(rec + 12 * (size_t)R->order[k], H, &y0, &y1);
        for (int y = y0; y <= y1; ++y) R->row_list[fill[y]++] = k;
    }
    free(fill);
}

static void free_rows(rows_t *R)
{
    free(R->order);
    free(R->row_start);
    free(R->row_list);
}

static int near_rel(double x, double ref, double band)
{
    return fabs(x - ref) <= band * fabs(ref);
}

typedef struct {
    int id;
    double alpha, sigma, T, r, dx, dy, base;
} contrib_t;

/*
 * Composite one pixel.  Fills list[] (if non-NULL, capacity cap) with the
 * contributors front to back; returns their count.  Writes colour, T_final
 * and the flag mask.
 */
static int shade_pixel(const double *rec, const unsigned char *amb, const rows_t *R, int x, int y,
                       int W, const bands_t *bd, double col[3], double *tfin, unsigned *flag,
                       contrib_t *list, int cap)
{
    double px = x + 0.5, py = y + 0.5;
    double T = 1.0;
    double prev_depth = -1.0;
    int cnt = 0;
    unsigned fl = 0;
    col[0] = col[1] = col[2] = 0.0;
    for (int p = R->row_start[y]; p < R->row_start[y + 1]; ++p) {
        int id = R->order[R->row_list[p]];
        const double *r = rec + 12 * (size_t)id;
        int x0, x1;
        col_span(r, W, &x0, &x1);
        if (x < x0 || x > x1) continue;
        double dx = px - r[0], dy = py - r[1];
        double q = r[2] * dx * dx + 2.0 * r[3] * dx * dy + r[4] * dy * dy;
        if (amb && amb[id]) {
            double reach = 1.0;
            if (amb[id] == 2) {
                reach = 1.0 - pow(1.0 + bd->band_opacity, -1.0 / r[7]);
                if (r[5] > reach) reach = r[5];
            }
            if (q < reach) fl |= 16;
            if (!(r[5] > 0.0)) continue;
        }
        double rho = r[5];
        if (!(q <= rho)) {
            if (near_rel(q, rho, bd->band_alpha)) fl |= 1;
            continue;
        }
        if (near_rel(q, rho, bd->band_alpha)) fl |= 1;
        double base = 1.0 - q;
        double sigma = r[6] * pow(base, r[7]);
        double alpha = sigma < ALPHA_MAX ? sigma : ALPHA_MAX;
        if (near_rel(sigma, ALPHA_MAX, bd->band_clamp)) fl |= 8;
        if (near_rel(alpha, ALPHA_MIN, bd->band_alpha)) fl |= 1;
        if (alpha < ALPHA_MIN) continue;
        double test = T * (1.0 - alpha);
        if (near_rel(test, T_STOP, bd->band_t)) fl |= 2;
        if (test < T_STOP) break;
        if (prev_depth >= 0.0 && near_rel(r[11], prev_depth, bd->band_depth)) fl |= 4;
        prev_depth = r[11];
        if (list && cnt < cap) {
            contrib_t *c = &list[cnt];
            c->id = id; c->alpha = alpha; c->sigma = sigma; c->T = T;
            c->r = q; c->dx = dx; c->dy = dy; c->base = base;
        }
        col[0] += r[8] * alpha * T;
        col[1] += r[9] * alpha * T;
        col[2] += r[10] * alpha * T;
        T = test;
        cnt++;
    }
    *tfin = T;
    *flag = fl;
    return cnt;
}

/*
 * Forward render of one view.  image [H][W][3], tfinal [H][W], ncontrib
 * [H][W] (number of contributors), flags [H][W].  amb may be NULL.
 * Pixels are restricted to rows [y_begin, y_end) (the rest is untouched).
 */
int oracle_render_fwd(int n, const double *rec, const unsigned char *amb, int W, int H,
                      int y_begin, int y_end, const double *bands5, double *image, double *tfinal,
                      int *ncontrib, unsigned *flags)
{
    bands_t bd = {bands5[0], bands5[1], bands5[2], bands5[3], bands5[4]};
    rows_t R;
    build_rows(n, rec, amb, H, &R);
    for (int y = y_begin; y < y_end; ++y)
        for (int x = 0; x < W; ++x) {
            size_t p = (size_t)y * W + x;
            double col[3], T;
            unsigned fl;
            int cnt = shade_pixel(rec, amb, &R, x, y, W, &bd, col, &T, &fl, NULL, 0);
            image[3 * p] = col[0];
            image[3 * p + 1] = col[1];
            image[3 * p + 2] = col[2];
            tfinal[p] = T;
            ncontrib[p] = cnt;
            flags[p] = fl;
        }
    free_rows(&R);
    return 0;
}

/* Forward values at an explicit list of pixels (xs, ys), for sampled checks. */
int oracle_render_pixels(int n, const double *rec, const unsigned char *amb, int W, int H,
                         int npix, const int *xs, const int *ys, const double *bands5,
                         double *color, double *tfinal, int *ncontrib, unsigned *flags)
{
    bands_t bd = {bands5[0], bands5[1], bands5[2], bands5[3], bands5[4]};
    rows_t R;
    build_rows(n, rec, amb, H, &R);
    for (int i = 0; i < npix; ++i) {
        double col[3], T;
        unsigned fl;
        int cnt = shade_pixel(rec, amb, &R, xs[i], ys[i], W, &bd, col, &T, &fl, NULL, 0);
        color[3 * i] = col[0];
        color[3 * i + 1] = col[1];
        color[3 * i + 2] = col[2];
        tfinal[i] = T;
        ncontrib[i] = cnt;
        flags[i] = fl;
    }
    free_rows(&R);
    return 0;
}

/*
 * Adjoint of the compositing for one view, written by hand from the
 * forward recurrence (reverse over each pixel's contributor list).
 * d_image [H][W][3], d_tfinal [H][W] (may be NULL); accumulates into
 * d_rec [n][10]: d mx, d my, d a, d b, d c, d o, d beta, d r, d g, d bl.
 * With T_i the transmittance in front of contributor i and
 * S_i = sum_{j>i} c_j alpha_j prod_{i<k<j} (1 - alpha_k):
 *   dC/dc_i = alpha_i T_i,  dC/dalpha_i = T_i (c_i - S_i),
 *   dT_final/dalpha_i = -T_final / (1 - alpha_i).
 * alpha = sigma below the clamp (else constant); sigma = o (1-r)^beta gives
 *   d/do = (1-r)^beta, d/dbeta = sigma ln(1-r), d/dr = -beta sigma/(1-r),
 * and r = a dx^2 + 2 b dx dy + c dy^2 with dx = px - mx, dy = py - my.
 * d_rec_abs (may be NULL) accumulates the absolute value of every per-pixel
 * term instead: the scale of the rounding error of a float32 summation.
 * Only rows [y_begin, y_end) are visited.
 */
int oracle_render_bwd(int n, const double *rec, int W, int H, int y_begin, int y_end,
                      const double *d_image, const double *d_tfinal, double *d_rec,
                      double *d_rec_abs)
{
    bands_t bd = {1e-300, 1e-300, 1e-300, 1e-300, 1e-300};
    rows_t R;
    build_rows(n, rec, NULL, H, &R);
    int cap = R.m > 0 ? R.m : 1;
    contrib_t *list = (contrib_t *)malloc(sizeof(contrib_t) * (size_t)cap);
    for (int y = y_begin; y < y_end; ++y)
        for (int x = 0; x < W; ++x) {
            size_t p = (size_t)y * W + x;
            double col[3], Tf;
            unsigned fl;
            int cnt = shade_pixel(rec, NULL, &R, x, y, W, &bd, col, &Tf, &fl, list, cap);
            const double *g = d_image + 3 * p;
            double gT = d_tfinal ? d_tfinal[p] : 0.0;
            double S[3] = {0.0, 0.0, 0.0};
            for (int k = cnt - 1; k >= 0; --k) {
                const contrib_t *c = &list[k];
                const double *r = rec + 12 * (size_t)c->id;
                double *dr = d_rec + 10 * (size_t)c->id;
                double a = c->alpha, Ti = c->T;
                double t[10] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                t[7] = g[0] * a * Ti;
                t[8] = g[1] * a * Ti;
                t[9] = g[2] * a * Ti;
                double dalpha = g[0] * Ti * (r[8] - S[0]) + g[1] * Ti * (r[9] - S[1])
                              + g[2] * Ti * (r[10] - S[2]) - gT * Tf / (1.0 - a);
                S[0] = a * r[8] + (1.0 - a) * S[0];
                S[1] = a * r[9] + (1.0 - a) * S[1];
                S[2] = a * r[10] + (1.0 - a) * S[2];
                if (c->sigma < ALPHA_MAX) {
                    double pw = pow(c->base, r[7]);
                    t[5] = dalpha * pw;
                    t[6] = dalpha * c->sigma * log(c->base);
                    double dq = dalpha * (-r[7] * c->sigma / c->base);
                    t[0] = dq * (-2.0) * (r[2] * c->dx + r[3] * c->dy);
                    t[1] = dq * (-2.0) * (r[3] * c->dx + r[4] * c->dy);
                    t[2] = dq * c->dx * c->dx;
                    t[3] = dq * 2.0 * c->dx * c->dy;
                    t[4] = dq * c->dy * c->dy;
                }
                for (int q = 0; q < 10; ++q) dr[q] += t[q];
                if (d_rec_abs)
                    for (int q = 0; q < 10; ++q) d_rec_abs[10 * (size_t)c->id + q] += fabs(t[q]);
            }
        }
    free(list);
    free_rows(&R);
    return 0;
}

/* ------------------------------------------------------------------------
 * Binning reference.
 *
 * A record overlaps a tile iff the minimum of its quadratic form over the
 * rectangle spanned by the tile's pixel centres (clipped to the image) is
 * at most rho * (1 + 2^-10).  Evaluated in float64 round-to-nearest with no
 * contraction and in exactly this operation order (the kernel takes the
 * same decision the same way), from float32 record fields:
 *   centre inside the rectangle -> overlap;
 *   otherwise, on each edge the 1-D minimiser of the quadratic is clamped to
 *   the edge, comparing with multiplications only.
 * Every tile of the view is tested (brute force).
 * --------------------------------------------------------------------- */
static int tile_hit(double mx, double my, double a, double b, double c, double rho,
                    double x0, double x1, double y0, double y1)
{
    double rb = rho * (1.0 + 0x1p-10);
    if (mx >= x0 && mx <= x1 && my >= y0 && my <= y1) return 1;
    double det = a * c - b * b;
    double dy0 = y0 - my, dy1 = y1 - my;
    double dx0 = x0 - mx, dx1 = x1 - mx;
    double dxs[2] = {dx0, dx1};
    for (int e = 0; e < 2; ++e) {
        double dx = dxs[e];
        double t = -(b * dx);
        double lo = c * dy0, hi = c * dy1;
        if (t >= lo && t <= hi) {
            if ((det * dx) * dx <= rb * c) return 1;
        } else {
            double dy = (t < lo) ? dy0 : dy1;
            double q = ((a * dx) * dx + ((2.0 * b) * dx) * dy) + (c * dy) * dy;
            if (q <= rb) return 1;
        }
    }
    double dys[2] = {dy0, dy1};
    for (int e = 0; e < 2; ++e) {
        double dy = dys[e];
        double t = -(b * dy);
        double lo = a * dx0, hi = a * dx1;
        if (t >= lo && t <= hi) {
            if ((det * dy) * dy <= rb * a) return 1;
        } else {
            double dx = (t < lo) ? dx0 : dx1;
            double q = ((a * dx) * dx + ((2.0 * b) * dx) * dy) + (c * dy) * dy;
            if (q <= rb) return 1;
        }
    }
    return 0;
}

/*
 * Emit (key, value) pairs for n float32 records of one view, records in
 * index order, tiles row-major.  key = ((tile_base + ty*tiles_x + tx) << 32)
 * | bits(depth as float32); value = rec_base + index.  Writes at most cap
 * pairs; returns the total number of pairs.
 */
/* Tiles worth testing for a record: those whose pixel-centre rectangle
 * meets the bounding box of the ellipse {r <= rho (1 + 2^-10)}, widened by
 * a millionth and a pixel (far more than the rounding of the tile test).
 * Pure speed: the products of the float32 conic entries are exact in
 * float64, so the determinant is accurate however elongated the ellipse;
 * a conic that is not positive definite, or any doubt, scans every tile.
 * g_bin_prefilter = 0 scans every tile of every record (the pins compare
 * the two). */
static int g_bin_prefilter = 1;
void oracle_set_bin_prefilter(int on) { g_bin_prefilter = on; }

static void tile_window(const float *r, int W, int H, int tw, int th, int tx_n, int ty_n,
                        int *tx_lo, int *tx_hi, int *ty_lo, int *ty_hi)
{
    *tx_lo = 0; *tx_hi = tx_n - 1; *ty_lo = 0; *ty_hi = ty_n - 1;
    if (!g_bin_prefilter) return;
    double a = (double)r[2], b = (double)r[3], c = (double)r[4];
    double det = a * c - b * b;
    if (!(det > 0.0) || !(a > 0.0) || !(c > 0.0)) return;
    double lim = (double)r[5] * (1.0 + 0x1p-10);
    double hx = sqrt(lim * c / det) * (1.0 + 1e-6) + 1.0;
    double hy = sqrt(lim * a / det) * (1.0 + 1e-6) + 1.0;
    double xmin = (double)r[0] - hx, xmax = (double)r[0] + hx;
    double ymin = (double)r[1] - hy, ymax = (double)r[1] + hy;
    if (!(xmax >= 0.0) || !(ymax >= 0.0) || !(xmin <= (double)W) || !(ymin <= (double)H)) {
        *tx_lo = 1; *tx_hi = 0;   /* no tile */
        return;
    }
    /* clip to the view (keeps the int conversions in range) */
    if (xmin < 0.0) xmin = 0.0;
    if (ymin < 0.0) ymin = 0.0;
    if (xmax > (double)W) xmax = (double)W;
    if (ymax > (double)H) ymax = (double)H;
    /* tile tx spans pixel centres [tx tw + 0.5, tx tw + tw - 0.5] */
    int lo = (int)floor((xmin - 0.5) / tw) - 1, hi = (int)floor((xmax - 0.5) / tw) + 1;
    if (lo > *tx_lo) *tx_lo = lo;
    if (hi < *tx_hi) *tx_hi = hi;
    lo = (int)floor((ymin - 0.5) / th) - 1;
    hi = (int)floor((ymax - 0.5) / th) + 1;
    if (lo > *ty_lo) *ty_lo = lo;
    if (hi < *ty_hi) *ty_hi = hi;
}

int64_t oracle_bin(int n, const float *rec32, int W, int H, int tw, int th, uint32_t tile_base,
                   uint32_t rec_base, int64_t cap, uint64_t *keys, uint32_t *vals)
{
    int tx_n = (W + tw - 1) / tw, ty_n = (H + th - 1) / th;
    int64_t k = 0;
    for (int i = 0; i < n; ++i) {
        const float *r = rec32 + 12 * (size_t)i;
        if (!(r[5] > 0.0f)) continue;
        uint32_t dbits;
        memcpy(&dbits, &r[11], 4);
        int tx_lo, tx_hi, ty_lo, ty_hi;
        tile_window(r, W, H, tw, th, tx_n, ty_n, &tx_lo, &tx_hi, &ty_lo, &ty_hi);
        for (int ty = ty_lo; ty <= ty_hi; ++ty)
            for (int tx = tx_lo; tx <= tx_hi; ++tx) {
                int px1 = tx * tw + tw - 1, py1 = ty * th + th - 1;
                if (px1 > W - 1) px1 = W - 1;
                if (py1 > H - 1) py1 = H - 1;
                double x0 = (double)(tx * tw) + 0.5, x1 = (double)px1 + 0.5;
                double y0 = (double)(ty * th) + 0.5, y1 = (double)py1 + 0.5;
                if (tile_hit((double)r[0], (double)r[1], (double)r[2], (double)r[3], (double)r[4],
                             (double)r[5], x0, x1, y0, y1)) {
                    if (k < cap) {
                        uint64_t tile = (uint64_t)tile_base + (uint64_t)ty * (uint64_t)tx_n + (uint64_t)tx;
                        keys[k] = (tile << 32) | (uint64_t)dbits;
                        vals[k] = rec_base + (uint32_t)i;
                    }
                    k++;
                }
            }
    }
    return k;
}

/* The single-tile test, exported for the pinning tests. */
int oracle_tile_hit(double mx, double my, double a, double b, double c, double rho,
                    double x0, double x1, double y0, double y1)
{
    return tile_hit(mx, my, a, b, c, rho, x0, x1, y0, y1);
}
