/*
 * degraf_oracle.c -- plain FP64 CPU oracle for the DeGraF + robust local optical flow path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file exists so that the tests, the smoke check and the
 * benchmark's CPU-baseline leg can compare the HIP library against a slow, obviously correct
 * implementation written straight from the method's definitions.  No product code may link,
 * load or call it, and it shares no code, header, table or helper with the HIP library.
 *
 * Sources of each computation (Stephenson, Breckon, Katramados, "DeGraF-Flow", 2019):
 *   - Key-point detection: Section 2, "Point detection": sliding window with step delta,
 *     Eq. (1) (positive centroid), Eq. (2) (negative centroid) and the rule after Eq. (2)
 *     that keeps the centroid with the larger weight sum.
 *   - Tracking: Section 2, "Sparse point tracking" (robust local optical flow, a Lucas-Kanade
 *     derivative, Section 1).  The paper leaves the tracker's internals to its citation, so the
 *     exact iteration below is the reading documented at each function: a coarse-to-fine
 *     image pyramid and, per level, iteratively re-weighted Gauss-Newton on a 2x2 system under
 *     a redescending robust norm.
 *   - Gradient of the converged flow w.r.t. both images: implicit differentiation of the
 *     level-0 fixed-point equation  F(u) = sum_k psi(r_k(u)) g_k = 0.
 *
 * Everything is double precision.  Loops follow the definitions one term at a time; the only
 * parallelism is an OpenMP loop over independent windows or points.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_ERR_ARG (-1)
#define OR_ERR_MEM (-2)

#define OR_ST_CONVERGED 0
#define OR_ST_NOT_CONVERGED 1
#define OR_ST_ILL_CONDITIONED 2
#define OR_ST_OUT_OF_BOUNDS 3

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* ------------------------------------------------------------------------------------------ */
/* DeGraF detection (Section 2 "Point detection", Eq. 1-2)                                     */
/* ------------------------------------------------------------------------------------------ */

/* Number of window positions.  Reading of "a sliding window is passed over the image with step
 * delta": windows lie fully inside the image, origins at (kx*delta, ky*delta) from (0, 0). */
int64_t or_detect_count(int W, int H, int win, int stride)
{
    if (win <= 0 || stride <= 0 || W < win || H < win) return 0;
    return (int64_t)((W - win) / stride + 1) * (int64_t)((H - win) / stride + 1);
}

/*
 * The two weighted sums of one w x h window at (x0, y0) (Eq. 1 and Eq. 2), as exact integers:
 *   out[0] = S_pos = sum I,          out[1] = sum i*I (row),          out[2] = sum j*I (column)
 *   out[3] = S_neg = sum (1+m-I),    out[4] = sum i*(1+m-I),          out[5] = sum j*(1+m-I)
 *   out[6] = m
 * m_mode 0: m is the window maximum (the subscript of max in Eq. 2);
 * m_mode 1: m = 255 (the alternative reading of "normalised 1 -> 256").
 */
void or_window_sums(const uint8_t *img, int64_t pitch, int x0, int y0, int w, int h, int m_mode,
                    int64_t out[7])
{
    int64_t m = 0;
    for (int i = 0; i < h; ++i)
        for (int j = 0; j < w; ++j) {
            int64_t v = img[(int64_t)(y0 + i) * pitch + (x0 + j)];
            if (v > m) m = v;
        }
    if (m_mode == 1) m = 255;
    int64_t s_pos = 0, i_pos = 0, j_pos = 0;
    int64_t s_neg = 0, i_neg = 0, j_neg = 0;
    for (int i = 0; i < h; ++i)
        for (int j = 0; j < w; ++j) {
            int64_t v = img[(int64_t)(y0 + i) * pitch + (x0 + j)];
            int64_t vn = 1 + m - v;
            s_pos += v;
            i_pos += (int64_t)i * v;
            j_pos += (int64_t)j * v;
            s_neg += vn;
            i_neg += (int64_t)i * vn;
            j_neg += (int64_t)j * vn;
        }
    out[0] = s_pos; out[1] = i_pos; out[2] = j_pos;
    out[3] = s_neg; out[4] = i_neg; out[5] = j_neg;
    out[6] = m;
}

/*
 * One key-point per window, in row-major window order (window n = ky*nx + kx).
 *   img      : uint8 grey image, row y at img + y*pitch
 *   m_mode   : see or_window_sums
 *   pts      : out [N][2] = (x, y), x = column, pixel centres at integer coordinates
 *   sel      : out [N] (nullable) 1 when the negative centroid was kept
 *   resp     : out [N] (nullable) |C_pos - C_neg|, with C_pos := window centre when S_pos = 0
 * Returns N, or a negative code.
 */
int64_t or_detect(const uint8_t *img, int W, int H, int64_t pitch, int win, int stride, int m_mode,
                  double *pts, uint8_t *sel, double *resp, int nthreads)
{
    if (!img || !pts || win <= 0 || stride <= 0 || W <= 0 || H <= 0 || pitch < W) return OR_ERR_ARG;
    int64_t N = or_detect_count(W, H, win, stride);
    if (N == 0) return 0;
    const int nx = (W - win) / stride + 1;
    const int w = win, h = win;
    if (nthreads < 1) nthreads = 1;

#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        const int kx = (int)(n % nx), ky = (int)(n / nx);
        const int x0 = kx * stride, y0 = ky * stride;
        int64_t S[7];
        or_window_sums(img, pitch, x0, y0, w, h, m_mode, S);
        const int64_t s_pos = S[0], s_neg = S[3];

        /* Centroids as (column, row) offsets inside the window: Eq. (1) gives the row
         * coordinate from sum i*I and the column coordinate from sum j*I. */
        double cpos_x, cpos_y;
        if (s_pos > 0) {
            cpos_x = (double)S[2] / (double)s_pos;
            cpos_y = (double)S[1] / (double)s_pos;
        } else { /* all-black window: C_pos undefined; use the window centre for the response */
            cpos_x = 0.5 * (w - 1);
            cpos_y = 0.5 * (h - 1);
        }
        /* s_neg >= w*h >= 1 because every weight 1 + m - I is at least 1 */
        double cneg_x = (double)S[5] / (double)s_neg;
        double cneg_y = (double)S[4] / (double)s_neg;

        /* Keep the centroid with the larger sum; a tie keeps the positive centroid. */
        int neg = s_neg > s_pos;
        pts[2 * n + 0] = (double)x0 + (neg ? cneg_x : cpos_x);
        pts[2 * n + 1] = (double)y0 + (neg ? cneg_y : cpos_y);
        if (sel) sel[n] = (uint8_t)neg;
        if (resp) resp[n] = hypot(cpos_x - cneg_x, cpos_y - cneg_y);
    }
    return N;
}

/*
 * The same detector on a real-valued image (double, row pitch in elements): Eq. (1) and Eq. (2)
 * with real sums and m the window maximum; the larger sum wins, a tie keeps the positive centroid.
 * Used to define, and check by finite differences, the gradient of the points w.r.t. the image.
 */
int64_t or_detect_f64(const double *img, int W, int H, int64_t pitch, int win, int stride, double *pts,
                      uint8_t *sel)
{
    if (!img || !pts || win <= 0 || stride <= 0 || W <= 0 || H <= 0 || pitch < W) return OR_ERR_ARG;
    int64_t N = or_detect_count(W, H, win, stride);
    const int nx = N ? (W - win) / stride + 1 : 1;
    for (int64_t n = 0; n < N; ++n) {
        const int x0 = (int)(n % nx) * stride, y0 = (int)(n / nx) * stride;
        double m = -INFINITY;
        for (int i = 0; i < win; ++i)
            for (int j = 0; j < win; ++j) m = fmax(m, img[(int64_t)(y0 + i) * pitch + x0 + j]);
        double sp = 0, ip = 0, jp = 0, sn = 0, in = 0, jn = 0;
        for (int i = 0; i < win; ++i)
            for (int j = 0; j < win; ++j) {
                double v = img[(int64_t)(y0 + i) * pitch + x0 + j], vn = 1.0 + m - v;
                sp += v;
                ip += i * v;
                jp += j * v;
                sn += vn;
                in += i * vn;
                jn += j * vn;
            }
        int neg = sn > sp;
        pts[2 * n + 0] = x0 + (neg ? jn / sn : jp / sp);
        pts[2 * n + 1] = y0 + (neg ? in / sn : ip / sp);
        if (sel) sel[n] = (uint8_t)neg;
    }
    return N;
}

/*
 * Gradient of the detected points w.r.t. the image (the centroid ratios of Eq. 1-2 are smooth in
 * the pixel values away from ties): for point n with upstream gradient dpoints[n] = dL/dp, ADDS
 *   dI[q] += dL/dp . dp/dI[q]
 * over its window.  Positive centroid C = sum c v / S: dC/dv(q) = (c(q) - C) / S.  Negative
 * centroid with weights 1 + m - v and m the window maximum (taken at the first maximal pixel q*
 * in row-major order): dC/dv(q) = (-(c(q) - C) + [q = q*] sum_q' (c(q') - C)) / S_neg.
 * sel gives the centroid each point took (as or_detect_f64 returns it).
 */
int or_detect_grad(const double *img, int W, int H, int64_t pitch, int win, int stride, const uint8_t *sel,
                   const double *dpoints, double *dI)
{
    if (!img || !sel || !dpoints || !dI || win <= 0 || stride <= 0 || W <= 0 || H <= 0 || pitch < W) return OR_ERR_ARG;
    int64_t N = or_detect_count(W, H, win, stride);
    const int nx = N ? (W - win) / stride + 1 : 1;
    for (int64_t n = 0; n < N; ++n) {
        const int x0 = (int)(n % nx) * stride, y0 = (int)(n / nx) * stride;
        const double lx = dpoints[2 * n], ly = dpoints[2 * n + 1];
        double m = -INFINITY;
        int qi = 0, qj = 0;
        for (int i = 0; i < win; ++i)
            for (int j = 0; j < win; ++j) {
                double v = img[(int64_t)(y0 + i) * pitch + x0 + j];
                if (v > m) {
                    m = v;
                    qi = i;
                    qj = j;
                }
            }
        double S = 0, Ci = 0, Cj = 0;
        for (int i = 0; i < win; ++i)
            for (int j = 0; j < win; ++j) {
                double v = img[(int64_t)(y0 + i) * pitch + x0 + j];
                double wv = sel[n] ? 1.0 + m - v : v;
                S += wv;
                Ci += i * wv;
                Cj += j * wv;
            }
        Ci /= S;
        Cj /= S;
        for (int i = 0; i < win; ++i)
            for (int j = 0; j < win; ++j) {
                double di, dj; /* d(Ci, Cj) / dv(i, j) */
                if (!sel[n]) {
                    di = (i - Ci) / S;
                    dj = (j - Cj) / S;
                } else {
                    di = -(i - Ci) / S;
                    dj = -(j - Cj) / S;
                    if (i == qi && j == qj) { /* the maximum raises every weight */
                        di += win * win * (0.5 * (win - 1) - Ci) / S;
                        dj += win * win * (0.5 * (win - 1) - Cj) / S;
                    }
                }
                dI[(int64_t)(y0 + i) * pitch + x0 + j] += lx * dj + ly * di;
            }
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------------------------ */
/* Image pyramid (the tracker is pyramidal; the paper gives no filter, this is the reading)   */
/* ------------------------------------------------------------------------------------------ */

/* Level l+1 has size ceil(W_l / 2) x ceil(H_l / 2); dims[2l] = W_l, dims[2l+1] = H_l. */
void or_pyr_dims(int W, int H, int levels, int *dims)
{
    for (int l = 0; l < levels; ++l) {
        dims[2 * l] = W;
        dims[2 * l + 1] = H;
        W = (W + 1) / 2;
        H = (H + 1) / 2;
    }
}

static const int k5[5] = {1, 4, 6, 4, 1};

/* One reduction step on a uint8 image: full 5x5 binomial sum with replicated borders, sampled at
 * even pixels, rounded half-up with integer arithmetic: (sum + 128) >> 8. */
int or_pyr_down_u8(const uint8_t *src, int W, int H, int64_t pitch, uint8_t *dst)
{
    if (!src || !dst || W <= 0 || H <= 0 || pitch < W) return OR_ERR_ARG;
    const int W2 = (W + 1) / 2, H2 = (H + 1) / 2;
    for (int y = 0; y < H2; ++y)
        for (int x = 0; x < W2; ++x) {
            int64_t sum = 0;
            for (int b = -2; b <= 2; ++b)
                for (int a = -2; a <= 2; ++a) {
                    int yy = clampi(2 * y + b, 0, H - 1), xx = clampi(2 * x + a, 0, W - 1);
                    sum += (int64_t)k5[a + 2] * k5[b + 2] * src[(int64_t)yy * pitch + xx];
                }
            dst[(int64_t)y * W2 + x] = (uint8_t)((sum + 128) >> 8);
        }
    return OR_OK;
}

/* The same reduction on a real-valued image, exact division by 256 (no rounding). */
int or_pyr_down_f64(const double *src, int W, int H, double *dst)
{
    if (!src || !dst || W <= 0 || H <= 0) return OR_ERR_ARG;
    const int W2 = (W + 1) / 2, H2 = (H + 1) / 2;
    for (int y = 0; y < H2; ++y)
        for (int x = 0; x < W2; ++x) {
            double sum = 0.0;
            for (int b = -2; b <= 2; ++b)
                for (int a = -2; a <= 2; ++a) {
                    int yy = clampi(2 * y + b, 0, H - 1), xx = clampi(2 * x + a, 0, W - 1);
                    sum += (double)(k5[a + 2] * k5[b + 2]) * src[(int64_t)yy * W + xx];
                }
            dst[(int64_t)y * W2 + x] = sum / 256.0;
        }
    return OR_OK;
}

/* ------------------------------------------------------------------------------------------ */
/* Sampling helpers                                                                           */
/* ------------------------------------------------------------------------------------------ */

/* Bilinear interpolation with each of the four taps clamped to the image (replicated border).
 * Pixel centres are at integer coordinates.  Non-finite coordinates give NaN.  Evaluated as two
 * linear interpolations along x and one along y (a + f (b - a)): the same interpolant as the
 * weighted four-tap sum, in a form that reproduces a constant neighbourhood exactly, so a
 * residual between flat regions of integer frames is an exact integer. */
double or_bilinear(const double *I, int W, int H, double x, double y)
{
    if (!isfinite(x) || !isfinite(y)) return NAN;
    double xf = floor(x), yf = floor(y);
    double fx = x - xf, fy = y - yf;
    /* Far outside the image every tap clamps to the border, so limiting the integer part first
     * changes nothing and keeps the conversion to int defined. */
    if (xf < -2.0) xf = -2.0;
    if (xf > (double)W) xf = (double)W;
    if (yf < -2.0) yf = -2.0;
    if (yf > (double)H) yf = (double)H;
    int x0 = (int)xf, y0 = (int)yf;
    int xa = clampi(x0, 0, W - 1), xb = clampi(x0 + 1, 0, W - 1);
    int ya = clampi(y0, 0, H - 1), yb = clampi(y0 + 1, 0, H - 1);
    double i00 = I[(int64_t)ya * W + xa], i10 = I[(int64_t)ya * W + xb];
    double i01 = I[(int64_t)yb * W + xa], i11 = I[(int64_t)yb * W + xb];
    double h0 = i00 + fx * (i10 - i00), h1 = i01 + fx * (i11 - i01);
    return h0 + fy * (h1 - h0);
}

/* ------------------------------------------------------------------------------------------ */
/* Robust norm                                                                                */
/* ------------------------------------------------------------------------------------------ */

/* Influence function of the robust norm: a continuous, piecewise-linear, redescending
 * (Hampel-type) function with thresholds s1 <= s2 in intensity units:
 *     psi(r) = r                                   |r| <= s1
 *            = sign(r) * s1 * (s2 - |r|) / (s2 - s1)  s1 < |r| < s2
 *            = 0                                   |r| >= s2
 * s1 = s2 = +inf is the least-squares (plain Lucas-Kanade) limit. */
double or_psi(double r, double s1, double s2)
{
    double a = fabs(r);
    if (a <= s1) return r;
    if (a >= s2) return 0.0;
    return copysign(s1 * (s2 - a) / (s2 - s1), r);
}

/* Derivative of psi, band by band (used by the implicit gradient). */
double or_dpsi(double r, double s1, double s2)
{
    double a = fabs(r);
    if (a <= s1) return 1.0;
    if (a >= s2) return 0.0;
    return -s1 / (s2 - s1);
}

/* IRLS weight psi(r)/r, with the limit 1 at r = 0. */
static double irls_weight(double r, double s1, double s2)
{
    if (r == 0.0) return 1.0;
    return or_psi(r, s1, s2) / r;
}

/* ------------------------------------------------------------------------------------------ */
/* Pyramids of both images as double arrays                                                   */
/* ------------------------------------------------------------------------------------------ */

typedef struct {
    int levels;
    int W[32], H[32];
    double *img[32]; /* level images */
} pyr_t;

static void pyr_free(pyr_t *p)
{
    for (int l = 0; l < p->levels; ++l) free(p->img[l]);
}

/* dtype 0: uint8 input, levels are uint8 images (integer rounding), converted to double;
 * dtype 1: double input, levels are exact double reductions. */
static int pyr_build(pyr_t *p, const void *src, int dtype, int W, int H, int64_t pitch, int levels)
{
    memset(p, 0, sizeof(*p));
    p->levels = levels;
    int dims[64];
    or_pyr_dims(W, H, levels, dims);
    uint8_t *u8prev = NULL, *u8cur = NULL;
    for (int l = 0; l < levels; ++l) {
        int Wl = dims[2 * l], Hl = dims[2 * l + 1];
        p->W[l] = Wl;
        p->H[l] = Hl;
        p->img[l] = (double *)malloc(sizeof(double) * (size_t)Wl * Hl);
        if (!p->img[l]) return OR_ERR_MEM;
        if (dtype == 0) {
            if (l == 0) {
                u8cur = (uint8_t *)malloc((size_t)Wl * Hl);
                if (!u8cur) return OR_ERR_MEM;
                for (int y = 0; y < Hl; ++y)
                    memcpy(u8cur + (size_t)y * Wl, (const uint8_t *)src + (int64_t)y * pitch, (size_t)Wl);
            } else {
                u8cur = (uint8_t *)malloc((size_t)Wl * Hl);
                if (!u8cur) return OR_ERR_MEM;
                or_pyr_down_u8(u8prev, dims[2 * l - 2], dims[2 * l - 1], dims[2 * l - 2], u8cur);
            }
            for (int64_t i = 0; i < (int64_t)Wl * Hl; ++i) p->img[l][i] = (double)u8cur[i];
            free(u8prev);
            u8prev = u8cur;
        } else {
            if (l == 0) {
                for (int y = 0; y < Hl; ++y)
                    for (int x = 0; x < Wl; ++x)
                        p->img[l][(int64_t)y * Wl + x] = ((const double *)src)[(int64_t)y * pitch + x];
            } else {
                or_pyr_down_f64(p->img[l - 1], dims[2 * l - 2], dims[2 * l - 1], p->img[l]);
            }
        }
    }
    free(u8prev);
    return OR_OK;
}

/* ------------------------------------------------------------------------------------------ */
/* Tracking                                                                                   */
/* ------------------------------------------------------------------------------------------ */

typedef struct {
    double sigma1, sigma2;   /* robust-norm thresholds, intensity units */
    double eps_coarse;       /* stop a level > 0 when |delta| < eps_coarse (px of that level) */
    double eps_fine;         /* stop level 0 when |delta| < eps_fine */
    double min_eig;          /* ill-conditioned when lambda_min(G0) / |support| < min_eig */
    int cross;               /* adaptive cross-based support (or_cross_mask) instead of the square */
    double tau;              /* its intensity threshold */
} or_opts;

/*
 * Adaptive cross-based support region of a template (the support RLOF(IM-GM) uses, Section 3
 * "Parameters"; defined in the tracker's citation).  Reading: the classic cross construction, on
 * a patch one pixel wider than the support on each side, Tx of size (s + 2) x (s + 2) (offsets
 * -r-1 .. r+1 from the point, index (ky + r + 1) (s + 2) + (kx + r + 1), s = 2r + 1; the tracker
 * fills it with cross_pixels):
 *   the vertical arm of the centre runs up and down from it while each next pixel of the centre
 *   column stays within tau of the centre value; every row the vertical arm covers gets a
 *   horizontal arm, anchored on that row's centre-column pixel, running left and right while
 *   each next pixel stays within tau of the anchor; the region is the union of the horizontal
 *   arms (the anchors and the centre are always in; |difference| <= tau, so a non-finite value
 *   ends an arm).
 * The support (mask, s x s, 1 = in) keeps a support pixel when it and its four neighbours -- the
 * stencil of its central-difference gradient -- all lie in the region, so no template gradient
 * in the support straddles the region's edge.  Returns the number of support pixels.
 */
int or_cross_mask(const double *Tx, int s, double tau, uint8_t *mask)
{
    const int r = s / 2, e = s + 2, re = r + 1;
    uint8_t *R = (uint8_t *)calloc((size_t)e * e, 1);
    if (!R) return 0;
    const double c = Tx[re * e + re];
    int up = 0, down = 0;
    while (up < re && fabs(Tx[(re - up - 1) * e + re] - c) <= tau) ++up;
    while (down < re && fabs(Tx[(re + down + 1) * e + re] - c) <= tau) ++down;
    for (int ky = -up; ky <= down; ++ky) {
        const double *row = Tx + (ky + re) * e;
        const double a = row[re];
        int left = 0, right = 0;
        while (left < re && fabs(row[re - left - 1] - a) <= tau) ++left;
        while (right < re && fabs(row[re + right + 1] - a) <= tau) ++right;
        for (int kx = -left; kx <= right; ++kx) R[(ky + re) * e + (kx + re)] = 1;
    }
    int count = 0;
    for (int ky = -r; ky <= r; ++ky)
        for (int kx = -r; kx <= r; ++kx) {
            const int q = (ky + re) * e + (kx + re);
            const uint8_t in = R[q] & R[q - 1] & R[q + 1] & R[q - e] & R[q + e];
            mask[(ky + r) * s + (kx + r)] = in;
            count += in;
        }
    free(R);
    return count;
}

/*
 * The (s + 2)^2 values the cross construction runs on: the level image's own pixels at
 * floor(p_l) + k, k in [-r-1, r+1]^2, border replicated (the pixel at the top-left of the cell each
 * template sample interpolates in).  Reading: the cross region is a segmentation of the image
 * around the point, so it is taken on the image's pixel grid; for integer frames every comparison
 * with tau is then exact, where differences of interpolated samples that share one set of bilinear
 * weights land exactly on an integer tau wherever the four underlying pixel differences agree, and
 * rounding would decide.
 */
static void cross_pixels(const double *I, int W, int H, double plx, double ply, int r, double *Tx)
{
    const int x0 = (int)floor(plx), y0 = (int)floor(ply), e = 2 * r + 3;
    for (int ky = -r - 1; ky <= r + 1; ++ky)
        for (int kx = -r - 1; kx <= r + 1; ++kx)
            Tx[(ky + r + 1) * e + (kx + r + 1)] =
                I[(int64_t)clampi(y0 + ky, 0, H - 1) * W + clampi(x0 + kx, 0, W - 1)];
}

/*
 * Track one point p (level-0 pixel coordinates) from I0 to I1.
 * Reading of the robust local flow iteration (the paper cites it without restating it):
 *   g = 0 at the coarsest level.  For l = L-1 .. 0, with p_l = p / 2^l and support offsets
 *   k in [-r, r]^2 (s = 2r + 1):
 *     T_k = B(I0_l, p_l + k), g_k = (B(I0_l, p_l + k + e_x) - B(I0_l, p_l + k - e_x)) / 2 and the
 *     same along y (central differences of the bilinear interpolant), G0 = sum g_k g_k^T.
 *     If lambda_min(G0)/s^2 < min_eig the level gives no update (for l > 0: g = 2 g, next
 *     level); at level 0 the point is ill-conditioned with u = g.
 *     d = 0; repeat up to iters times:
 *        r_k = B(I1_l, p_l + k + g + d) - T_k,  w_k = psi(r_k)/r_k,
 *        Gw = sum w_k g_k g_k^T,  b = -sum w_k r_k g_k,
 *        if det Gw <= 1e-6 det G0 (or is not a number), use w = 1 for this step,
 *        delta = Gw^-1 b,  d += delta,  stop the level when |delta|_2 < eps_l.
 *     A non-finite delta ends the point (not converged).  For l > 0: g = 2 (g + d).
 *   u = g + d.  Status: ill-conditioned, else not converged if level 0 did not stop on eps,
 *   else out of bounds if p + u leaves [0, W-1] x [0, H-1], else converged.
 * Points outside the image (or not finite) are out of bounds with u = 0.
 */
static void track_point(const pyr_t *P0, const pyr_t *P1, double px, double py, int L, int s,
                        int iters, const or_opts *o, double g0x, double g0y, int lstop, double *ux,
                        double *uy, uint8_t *st, int32_t *it_count)
{
    const int r = s / 2;
    const int W = P0->W[0], H = P0->H[0];
    if (!(isfinite(px) && isfinite(py)) || px < 0.0 || py < 0.0 || px > W - 1 || py > H - 1) {
        *ux = 0.0;
        *uy = 0.0;
        *st = OR_ST_OUT_OF_BOUNDS;
        return;
    }
    const int npix = s * s;
    double *T = (double *)malloc(sizeof(double) * npix);
    double *gxk = (double *)malloc(sizeof(double) * npix);
    double *gyk = (double *)malloc(sizeof(double) * npix);
    uint8_t *M = (uint8_t *)malloc((size_t)npix);
    double *Tx = (double *)malloc(sizeof(double) * (size_t)(s + 2) * (s + 2));

    double gX = g0x, gY = g0y; /* guess carried from the coarser level, in level-l pixels */
    double dX = 0.0, dY = 0.0;
    int conv = 0;
    int status = -1;
    for (int l = L - 1; l >= lstop; --l) {
        const double scale = ldexp(1.0, -l);
        const double plx = px * scale, ply = py * scale;
        const int Wl = P0->W[l], Hl = P0->H[l];

        /* template and its gradient: value of the bilinear interpolant of the border-replicated
         * level image, and central differences of that interpolant at +-1 px */
        double a = 0.0, b = 0.0, c = 0.0; /* G0 = [[a, b], [b, c]] over the support */
        const double *I0l = P0->img[l];
        for (int ky = -r; ky <= r; ++ky)
            for (int kx = -r; kx <= r; ++kx) {
                int k = (ky + r) * s + (kx + r);
                double x = plx + kx, y = ply + ky;
                T[k] = or_bilinear(I0l, Wl, Hl, x, y);
                gxk[k] = 0.5 * (or_bilinear(I0l, Wl, Hl, x + 1.0, y) - or_bilinear(I0l, Wl, Hl, x - 1.0, y));
                gyk[k] = 0.5 * (or_bilinear(I0l, Wl, Hl, x, y + 1.0) - or_bilinear(I0l, Wl, Hl, x, y - 1.0));
            }
        /* support of this level: the square window, or its adaptive cross-based part */
        int nsup = npix;
        if (o->cross) {
            cross_pixels(I0l, Wl, Hl, plx, ply, r, Tx);
            nsup = or_cross_mask(Tx, s, o->tau, M);
        } else {
            memset(M, 1, (size_t)npix);
        }
        for (int k = 0; k < npix; ++k)
            if (M[k]) {
                a += gxk[k] * gxk[k];
                b += gxk[k] * gyk[k];
                c += gyk[k] * gyk[k];
            }
        const double lam_min = 0.5 * (a + c) - sqrt(0.25 * (a - c) * (a - c) + b * b);
        if (!(lam_min / (double)nsup >= o->min_eig)) {
            if (l == lstop) { /* the last level's support cannot be tracked */
                *ux = gX;
                *uy = gY;
                status = OR_ST_ILL_CONDITIONED;
                break;
            }
            /* a flat coarse level gives no update: the guess goes on to the next level as is */
            if (it_count) it_count[L - 1 - l] = 0;
            gX = 2.0 * gX;
            gY = 2.0 * gY;
            continue;
        }
        const double det0 = a * c - b * b;
        const double eps = (l > 0) ? o->eps_coarse : o->eps_fine;

        dX = 0.0;
        dY = 0.0;
        conv = 0;
        int bad = 0;
        int it = 0;
        for (it = 1; it <= iters; ++it) {
            double A = 0.0, B = 0.0, C = 0.0, bx = 0.0, by = 0.0;
            for (int ky = -r; ky <= r; ++ky)
                for (int kx = -r; kx <= r; ++kx) {
                    int k = (ky + r) * s + (kx + r);
                    if (!M[k]) continue;
                    double J = or_bilinear(P1->img[l], Wl, Hl, plx + kx + gX + dX, ply + ky + gY + dY);
                    double res = J - T[k];
                    double w = irls_weight(res, o->sigma1, o->sigma2);
                    A += w * gxk[k] * gxk[k];
                    B += w * gxk[k] * gyk[k];
                    C += w * gyk[k] * gyk[k];
                    bx -= w * res * gxk[k];
                    by -= w * res * gyk[k];
                }
            double det = A * C - B * B;
            if (!(det > 1e-6 * det0)) { /* too many down-weighted pixels: least-squares step */
                A = a;
                B = b;
                C = c;
                bx = 0.0;
                by = 0.0;
                for (int ky = -r; ky <= r; ++ky)
                    for (int kx = -r; kx <= r; ++kx) {
                        int k = (ky + r) * s + (kx + r);
                        if (!M[k]) continue;
                        double J = or_bilinear(P1->img[l], Wl, Hl, plx + kx + gX + dX, ply + ky + gY + dY);
                        double res = J - T[k];
                        bx -= res * gxk[k];
                        by -= res * gyk[k];
                    }
                det = det0;
            }
            double stepX = (C * bx - B * by) / det;
            double stepY = (A * by - B * bx) / det;
            if (!(isfinite(stepX) && isfinite(stepY))) {
                bad = 1;
                break;
            }
            dX += stepX;
            dY += stepY;
            if (sqrt(stepX * stepX + stepY * stepY) < eps) {
                conv = 1;
                break;
            }
        }
        if (it_count) it_count[L - 1 - l] = (it > iters) ? iters : it;
        if (bad) {
            *ux = NAN;
            *uy = NAN;
            status = OR_ST_NOT_CONVERGED;
            break;
        }
        if (l > lstop) {
            gX = 2.0 * (gX + dX);
            gY = 2.0 * (gY + dY);
        }
    }
    if (status < 0) {
        *ux = gX + dX;
        *uy = gY + dY;
        if (!conv)
            status = OR_ST_NOT_CONVERGED;
        else if (lstop > 0) /* a pass that stops above level 0 reports the step test only */
            status = OR_ST_CONVERGED;
        else {
            double qx = px + *ux, qy = py + *uy;
            status = (qx >= 0.0 && qy >= 0.0 && qx <= W - 1 && qy <= H - 1) ? OR_ST_CONVERGED
                                                                            : OR_ST_OUT_OF_BOUNDS;
        }
    }
    *st = (uint8_t)status;
    free(T);
    free(gxk);
    free(gyk);
    free(M);
    free(Tx);
}

/* Solves the n x n system A x = b (A row-major, both overwritten) by Gaussian elimination with
 * partial pivoting.  Returns 0, or -1 when a pivot is zero or not a number (x is then NaN). */
static int solve_dense(double *A, double *b, int n, double *x)
{
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(A[r * n + c]) > fabs(A[piv * n + c])) piv = r;
        if (!(fabs(A[piv * n + c]) > 0.0)) {
            for (int i = 0; i < n; ++i) x[i] = NAN;
            return -1;
        }
        if (piv != c) {
            for (int k = 0; k < n; ++k) {
                double t = A[c * n + k];
                A[c * n + k] = A[piv * n + k];
                A[piv * n + k] = t;
            }
            double t = b[c];
            b[c] = b[piv];
            b[piv] = t;
        }
        for (int r = c + 1; r < n; ++r) {
            double f = A[r * n + c] / A[c * n + c];
            for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
            b[r] -= f * b[c];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double acc = b[r];
        for (int k = r + 1; k < n; ++k) acc -= A[r * n + k] * x[k];
        x[r] = acc / A[r * n + r];
    }
    return 0;
}

/* Determinant of a 4 x 4 matrix by elimination on a copy (0 when singular). */
static double det4(const double *M)
{
    double A[16], b[4] = {0, 0, 0, 0}, x[4];
    memcpy(A, M, sizeof(A));
    /* the elimination in solve_dense leaves U in A; its diagonal product times the sign of the
     * row swaps is the determinant */
    double det = 1.0;
    for (int c = 0; c < 4; ++c) {
        int piv = c;
        for (int r = c + 1; r < 4; ++r)
            if (fabs(A[r * 4 + c]) > fabs(A[piv * 4 + c])) piv = r;
        if (!(fabs(A[piv * 4 + c]) > 0.0)) return 0.0;
        if (piv != c) {
            for (int k = 0; k < 4; ++k) {
                double t = A[c * 4 + k];
                A[c * 4 + k] = A[piv * 4 + k];
                A[piv * 4 + k] = t;
            }
            det = -det;
        }
        det *= A[c * 4 + c];
        for (int r = c + 1; r < 4; ++r) {
            double f = A[r * 4 + c] / A[c * 4 + c];
            for (int k = c; k < 4; ++k) A[r * 4 + k] -= f * A[c * 4 + k];
        }
    }
    (void)b;
    (void)x;
    return det;
}

/*
 * Illumination-model variant of track_point.  The paper's tracker configuration, RLOF(IM-GM)
 * (Section 3, "Parameters"), matches the support under a linear illumination change whose
 * definition is in the tracker's citation; the reading used here is a per-point gain and offset,
 *   I1(p + k + u) ~ (1 + m) I0(p + k) + c,
 * estimated jointly with u.  Per level, with theta = (d, m, c) and
 * phi_k = ((1 + m) g_x, (1 + m) g_y, -T_k, -1) -- the derivatives of the residual below, taking
 * the gradient of I1 at the match as the model predicts it, (1 + m) g_k:
 *   r_k = B(I1_l, p_l + k + g + d) - (1 + m) T_k - c,   w_k = psi(r_k) / r_k,
 *   (sum w_k phi_k phi_k^T) delta = - sum w_k r_k phi_k,   theta += delta,
 *   least-squares step (w = 1) when the weighted determinant is <= 1e-6 of the unweighted one
 *   (both with the current m), stop the level when |delta_d|_2 < eps_l.
 * m and c start at 0 on the coarsest level and carry over unchanged between levels (pyramid levels
 * are weighted averages, under which a gain and an offset stay the same).  Template, gradient,
 * level propagation of g and the statuses are those of track_point, except that
 *   - a support of fewer than four pixels (fewer than the unknowns) is flat as well;
 *   - a point whose gain 1 + m has left [1/4, 4] at the end of a coarse level (one it iterated
 *     on) ends NOT_CONVERGED with a NaN flow, as after a non-finite step: carried on, such
 *     iterates drift towards gain 0, where the motion drops out of the model and the steps in d
 *     grow without bound;
 *   - a point whose final gain lies outside [1/2, 2] is NOT_CONVERGED: such a match explains the
 *     support by a contrast change (or inversion) instead of a motion.  (m, c) of the last level are
 * returned in illum.
 */
static void track_point_illum(const pyr_t *P0, const pyr_t *P1, double px, double py, int L, int s,
                              int iters, const or_opts *o, double g0x, double g0y, int lstop, double *ux,
                              double *uy, uint8_t *st, int32_t *it_count, double *illum)
{
    const int r = s / 2;
    const int W = P0->W[0], H = P0->H[0];
    illum[0] = 0.0;
    illum[1] = 0.0;
    if (!(isfinite(px) && isfinite(py)) || px < 0.0 || py < 0.0 || px > W - 1 || py > H - 1) {
        *ux = 0.0;
        *uy = 0.0;
        *st = OR_ST_OUT_OF_BOUNDS;
        return;
    }
    const int npix = s * s;
    double *T = (double *)malloc(sizeof(double) * npix);
    double *gxk = (double *)malloc(sizeof(double) * npix);
    double *gyk = (double *)malloc(sizeof(double) * npix);
    uint8_t *M = (uint8_t *)malloc((size_t)npix);
    double *Tx = (double *)malloc(sizeof(double) * (size_t)(s + 2) * (s + 2));

    double gX = g0x, gY = g0y, dX = 0.0, dY = 0.0;
    double m = 0.0, c = 0.0; /* gain change and offset, carried across levels */
    int conv = 0;
    int status = -1;
    for (int l = L - 1; l >= lstop; --l) {
        const double scale = ldexp(1.0, -l);
        const double plx = px * scale, ply = py * scale;
        const int Wl = P0->W[l], Hl = P0->H[l];
        const double *I0l = P0->img[l];

        /* template, its gradient, and the 2 x 2 gradient matrix for the trackability test */
        double a2 = 0.0, b2 = 0.0, c2 = 0.0;
        for (int ky = -r; ky <= r; ++ky)
            for (int kx = -r; kx <= r; ++kx) {
                int k = (ky + r) * s + (kx + r);
                double x = plx + kx, y = ply + ky;
                T[k] = or_bilinear(I0l, Wl, Hl, x, y);
                gxk[k] = 0.5 * (or_bilinear(I0l, Wl, Hl, x + 1.0, y) - or_bilinear(I0l, Wl, Hl, x - 1.0, y));
                gyk[k] = 0.5 * (or_bilinear(I0l, Wl, Hl, x, y + 1.0) - or_bilinear(I0l, Wl, Hl, x, y - 1.0));
            }
        int nsup = npix;
        if (o->cross) {
            cross_pixels(I0l, Wl, Hl, plx, ply, r, Tx);
            nsup = or_cross_mask(Tx, s, o->tau, M);
        } else {
            memset(M, 1, (size_t)npix);
        }
        for (int k = 0; k < npix; ++k)
            if (M[k]) {
                a2 += gxk[k] * gxk[k];
                b2 += gxk[k] * gyk[k];
                c2 += gyk[k] * gyk[k];
            }
        const double lam_min = 0.5 * (a2 + c2) - sqrt(0.25 * (a2 - c2) * (a2 - c2) + b2 * b2);
        /* four unknowns need at least four support pixels (fewer make the 4 x 4 system singular) */
        if (!(lam_min / (double)nsup >= o->min_eig) || nsup < 4) {
            if (l == lstop) {
                *ux = gX;
                *uy = gY;
                status = OR_ST_ILL_CONDITIONED;
                break;
            }
            if (it_count) it_count[L - 1 - l] = 0;
            gX = 2.0 * gX;
            gY = 2.0 * gY;
            continue;
        }
        const double eps = (l > 0) ? o->eps_coarse : o->eps_fine;

        dX = 0.0;
        dY = 0.0;
        conv = 0;
        int bad = 0;
        int it = 0;
        for (it = 1; it <= iters; ++it) {
            double G[16] = {0}, G0[16] = {0}, rhs[4] = {0, 0, 0, 0}, rhs0[4] = {0, 0, 0, 0};
            for (int ky = -r; ky <= r; ++ky)
                for (int kx = -r; kx <= r; ++kx) {
                    int k = (ky + r) * s + (kx + r);
                    if (!M[k]) continue;
                    double J = or_bilinear(P1->img[l], Wl, Hl, plx + kx + gX + dX, ply + ky + gY + dY);
                    double res = J - (1.0 + m) * T[k] - c;
                    double w = irls_weight(res, o->sigma1, o->sigma2);
                    double phi[4] = {(1.0 + m) * gxk[k], (1.0 + m) * gyk[k], -T[k], -1.0};
                    for (int a = 0; a < 4; ++a) {
                        for (int b = 0; b < 4; ++b) {
                            G[a * 4 + b] += w * phi[a] * phi[b];
                            G0[a * 4 + b] += phi[a] * phi[b];
                        }
                        rhs[a] -= w * res * phi[a];
                        rhs0[a] -= res * phi[a];
                    }
                }
            if (!(det4(G) > 1e-6 * det4(G0))) { /* too many down-weighted pixels: least-squares step */
                memcpy(G, G0, sizeof(G));
                memcpy(rhs, rhs0, sizeof(rhs));
            }
            double delta[4];
            solve_dense(G, rhs, 4, delta);
            if (!(isfinite(delta[0]) && isfinite(delta[1]) && isfinite(delta[2]) && isfinite(delta[3]))) {
                bad = 1;
                break;
            }
            dX += delta[0];
            dY += delta[1];
            m += delta[2];
            c += delta[3];
            if (sqrt(delta[0] * delta[0] + delta[1] * delta[1]) < eps) {
                conv = 1;
                break;
            }
        }
        if (it_count) it_count[L - 1 - l] = (it > iters) ? iters : it;
        if (!bad && l > lstop && !(1.0 + m >= 0.25 && 1.0 + m <= 4.0)) bad = 1; /* runaway gain */
        if (bad) {
            *ux = NAN;
            *uy = NAN;
            status = OR_ST_NOT_CONVERGED;
            break;
        }
        if (l > lstop) {
            gX = 2.0 * (gX + dX);
            gY = 2.0 * (gY + dY);
        }
    }
    if (status < 0) {
        *ux = gX + dX;
        *uy = gY + dY;
        if (!conv || !(1.0 + m >= 0.5 && 1.0 + m <= 2.0))
            status = OR_ST_NOT_CONVERGED;
        else if (lstop > 0)
            status = OR_ST_CONVERGED;
        else {
            double qx = px + *ux, qy = py + *uy;
            status = (qx >= 0.0 && qy >= 0.0 && qx <= W - 1 && qy <= H - 1) ? OR_ST_CONVERGED
                                                                            : OR_ST_OUT_OF_BOUNDS;
        }
    }
    illum[0] = m;
    illum[1] = c;
    *st = (uint8_t)status;
    free(T);
    free(gxk);
    free(gyk);
    free(M);
    free(Tx);
}

/*
 * Global motion prior (the "GM" of RLOF(IM-GM), Section 3 "Parameters"; defined in the tracker's
 * citation).  Reading: one global affine motion of the frame, fitted robustly to sample motions
 * v_i at positions p_i (level-0 pixels), v ~ A (x - cx, y - cy, 1)^T with A 2 x 3:
 *   weighted least squares with weights w_i (1 for every sample to start), then `iters` times:
 *   residual e_i = |v_i - A p~_i|_2, Tukey biweight w_i = (1 - (e_i / c)^2)^2 for e_i < c, else 0,
 *   c = 4.685 scale, and the weighted least squares again.
 *   When fewer than 3 samples carry weight, or the weighted position covariance C has
 *   det C <= 1e-4 (tr C)^2, the model is the weighted mean motion (a translation); with no
 *   sample of positive weight the previous model stays (none at the start: A = 0).
 * pts, mot: [n][2]; use: [n], nonzero for a sample.  A: out [2][3] row-major.
 * Returns 2 (affine), 1 (translation) or 0 (no model, A = 0).
 */
int or_gm_fit(const double *pts, const double *mot, const uint8_t *use, int64_t n, double cx, double cy,
              double scale, int iters, double *A)
{
    for (int k = 0; k < 6; ++k) A[k] = 0.0;
    double *w = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!w) return 0;
    for (int64_t i = 0; i < n; ++i) w[i] = use[i] ? 1.0 : 0.0;
    const double c = 4.685 * scale;
    int kind = 0;
    for (int pass = 0; pass <= iters; ++pass) {
        if (pass > 0)
            for (int64_t i = 0; i < n; ++i) {
                if (!use[i]) continue;
                const double x = pts[2 * i] - cx, y = pts[2 * i + 1] - cy;
                const double ex = mot[2 * i] - (A[0] * x + A[1] * y + A[2]);
                const double ey = mot[2 * i + 1] - (A[3] * x + A[4] * y + A[5]);
                const double e = sqrt(ex * ex + ey * ey);
                const double t = e / c;
                w[i] = (e < c) ? (1.0 - t * t) * (1.0 - t * t) : 0.0;
            }
        double S = 0, Sx = 0, Sy = 0, Sxx = 0, Sxy = 0, Syy = 0;
        double Su = 0, Sxu = 0, Syu = 0, Sv = 0, Sxv = 0, Syv = 0;
        int64_t nz = 0;
        for (int64_t i = 0; i < n; ++i) {
            if (!(w[i] > 0.0)) continue;
            const double x = pts[2 * i] - cx, y = pts[2 * i + 1] - cy, u = mot[2 * i], v = mot[2 * i + 1];
            ++nz;
            S += w[i];
            Sx += w[i] * x;
            Sy += w[i] * y;
            Sxx += w[i] * x * x;
            Sxy += w[i] * x * y;
            Syy += w[i] * y * y;
            Su += w[i] * u;
            Sxu += w[i] * x * u;
            Syu += w[i] * y * u;
            Sv += w[i] * v;
            Sxv += w[i] * x * v;
            Syv += w[i] * y * v;
        }
        if (nz == 0) break; /* keep the previous model */
        const double mx = Sx / S, my = Sy / S;
        const double Cxx = Sxx / S - mx * mx, Cxy = Sxy / S - mx * my, Cyy = Syy / S - my * my;
        const double trC = Cxx + Cyy, detC = Cxx * Cyy - Cxy * Cxy;
        if (nz < 3 || !(detC > 1e-4 * trC * trC)) {
            A[0] = A[1] = A[3] = A[4] = 0.0;
            A[2] = Su / S;
            A[5] = Sv / S;
            kind = 1;
            continue;
        }
        double N[9] = {Sxx, Sxy, Sx, Sxy, Syy, Sy, Sx, Sy, S}, N2[9];
        double bu[3] = {Sxu, Syu, Su}, bv[3] = {Sxv, Syv, Sv}, au[3], av[3];
        memcpy(N2, N, sizeof(N));
        const int e1 = solve_dense(N, bu, 3, au), e2 = solve_dense(N2, bv, 3, av);
        if (e1 != 0 || e2 != 0) break;
        for (int k = 0; k < 3; ++k) {
            A[k] = au[k];
            A[3 + k] = av[k];
        }
        kind = 2;
    }
    free(w);
    return kind;
}

/*
 * Track n points.  I0/I1: dtype 0 = uint8 (row pitch in bytes), 1 = double (pitch in elements).
 * flow: out [n][2];  status: out [n];  iters_out: nullable [n][L], iterations run per level,
 * coarsest level first (0 where the point stopped before reaching that level).
 * illum: 0 = plain tracker (track_point); 1 = illumination model (track_point_illum), whose
 * final (m, c) go to illum_out (nullable, [n][2]).
 * cross: adaptive cross-based supports with threshold tau (or_cross_mask) at every level.
 * gm: global motion prior.  A first pass tracks every point on the coarsest level alone from zero
 * motion (same tracker, options and iteration limit); the points it reports converged there give
 * the samples (motion times 2^(L-1), at their level-0 positions) of or_gm_fit about the image
 * centre ((W-1)/2, (H-1)/2), scale 2^(L-1) px (one coarsest-level pixel), 10 reweightings; the
 * tracking proper then starts every point on the coarsest level from the model's motion at its
 * position (divided by 2^(L-1)) instead of zero.  gm_out (nullable, [6]) receives the model.
 */
int or_track(const void *I0, const void *I1, int dtype, int W, int H, int64_t pitch, const double *pts,
             int64_t n, int levels, int support, int iters, double sigma1, double sigma2,
             double eps_coarse, double eps_fine, double min_eig, int illum, int cross, double tau, int gm,
             double *flow, uint8_t *status, int32_t *iters_out, double *illum_out, double *gm_out, int nthreads)
{
    if (!I0 || !I1 || (n > 0 && (!pts || !flow || !status))) return OR_ERR_ARG;
    if (W <= 0 || H <= 0 || levels < 1 || levels > 16 || support < 1 || (support % 2) == 0 || iters < 1)
        return OR_ERR_ARG;
    if (dtype != 0 && dtype != 1) return OR_ERR_ARG;
    if (nthreads < 1) nthreads = 1;
    or_opts o = {sigma1, sigma2, eps_coarse, eps_fine, min_eig, cross, tau};
    pyr_t P0, P1;
    int rc0 = pyr_build(&P0, I0, dtype, W, H, pitch, levels);
    int rc1 = pyr_build(&P1, I1, dtype, W, H, pitch, levels);
    if (rc0 != OR_OK || rc1 != OR_OK) {
        pyr_free(&P0);
        pyr_free(&P1);
        return OR_ERR_MEM;
    }
    if (iters_out) memset(iters_out, 0, sizeof(int32_t) * (size_t)n * levels);
    const double top = ldexp(1.0, levels - 1); /* level-0 pixels per coarsest-level pixel */
    double *init = (double *)calloc((size_t)(n > 0 ? 2 * n : 2), sizeof(double));
    double A[6] = {0, 0, 0, 0, 0, 0};
    if (gm && n > 0) {
        double *mot = (double *)malloc(sizeof(double) * 2 * (size_t)n);
        uint8_t *st1 = (uint8_t *)malloc((size_t)n);
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 16)
        for (int64_t i = 0; i < n; ++i) {
            double mc[2];
            if (illum)
                track_point_illum(&P0, &P1, pts[2 * i], pts[2 * i + 1], levels, support, iters, &o, 0.0, 0.0,
                                  levels - 1, &mot[2 * i], &mot[2 * i + 1], &st1[i], NULL, mc);
            else
                track_point(&P0, &P1, pts[2 * i], pts[2 * i + 1], levels, support, iters, &o, 0.0, 0.0,
                            levels - 1, &mot[2 * i], &mot[2 * i + 1], &st1[i], NULL);
        }
        for (int64_t i = 0; i < n; ++i) {
            st1[i] = (st1[i] == OR_ST_CONVERGED && isfinite(mot[2 * i]) && isfinite(mot[2 * i + 1])) ? 1 : 0;
            mot[2 * i] *= top;
            mot[2 * i + 1] *= top;
        }
        or_gm_fit(pts, mot, st1, n, 0.5 * (W - 1), 0.5 * (H - 1), top, 10, A);
        for (int64_t i = 0; i < n; ++i) {
            const double x = pts[2 * i] - 0.5 * (W - 1), y = pts[2 * i + 1] - 0.5 * (H - 1);
            init[2 * i] = (A[0] * x + A[1] * y + A[2]) / top;
            init[2 * i + 1] = (A[3] * x + A[4] * y + A[5]) / top;
        }
        free(mot);
        free(st1);
    }
    if (gm_out)
        for (int k = 0; k < 6; ++k) gm_out[k] = A[k];
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        if (illum) {
            double mc[2];
            track_point_illum(&P0, &P1, pts[2 * i], pts[2 * i + 1], levels, support, iters, &o, init[2 * i],
                              init[2 * i + 1], 0, &flow[2 * i], &flow[2 * i + 1], &status[i],
                              iters_out ? &iters_out[i * levels] : NULL, mc);
            if (illum_out) {
                illum_out[2 * i] = mc[0];
                illum_out[2 * i + 1] = mc[1];
            }
        } else {
            track_point(&P0, &P1, pts[2 * i], pts[2 * i + 1], levels, support, iters, &o, init[2 * i],
                        init[2 * i + 1], 0, &flow[2 * i], &flow[2 * i + 1], &status[i],
                        iters_out ? &iters_out[i * levels] : NULL);
        }
    }
    free(init);
    pyr_free(&P0);
    pyr_free(&P1);
    return OR_OK;
}

/* ------------------------------------------------------------------------------------------ */
/* Gradient of the converged flow w.r.t. both images (implicit differentiation)               */
/* ------------------------------------------------------------------------------------------ */

/* Bilinear taps: indices and weights of the four (clamped) samples, and the analytic derivative
 * of the interpolant w.r.t. x and y inside the cell. */
static void bilinear_taps(int W, int H, double x, double y, int64_t idx[4], double wt[4], int cx[4],
                          int cy[4], double *fx_out, double *fy_out)
{
    double xf = floor(x), yf = floor(y);
    double fx = x - xf, fy = y - yf;
    if (xf < -2.0) xf = -2.0;
    if (xf > (double)W) xf = (double)W;
    if (yf < -2.0) yf = -2.0;
    if (yf > (double)H) yf = (double)H;
    int x0 = (int)xf, y0 = (int)yf;
    int xa = clampi(x0, 0, W - 1), xb = clampi(x0 + 1, 0, W - 1);
    int ya = clampi(y0, 0, H - 1), yb = clampi(y0 + 1, 0, H - 1);
    cx[0] = xa; cy[0] = ya; wt[0] = (1.0 - fx) * (1.0 - fy);
    cx[1] = xb; cy[1] = ya; wt[1] = fx * (1.0 - fy);
    cx[2] = xa; cy[2] = yb; wt[2] = (1.0 - fx) * fy;
    cx[3] = xb; cy[3] = yb; wt[3] = fx * fy;
    for (int t = 0; t < 4; ++t) idx[t] = (int64_t)cy[t] * W + cx[t];
    *fx_out = fx;
    *fy_out = fy;
}

/* Gradient of the bilinear interpolant (inside the cell that holds (x, y); clamped taps, so it
 * vanishes across the replicated border). */
static void bilinear_grad(const double *I, int W, int H, double x, double y, double g[2])
{
    int64_t idx[4]; double wt[4]; int cx[4], cy[4]; double fx, fy;
    bilinear_taps(W, H, x, y, idx, wt, cx, cy, &fx, &fy);
    g[0] = (1.0 - fy) * (I[idx[1]] - I[idx[0]]) + fy * (I[idx[3]] - I[idx[2]]);
    g[1] = (1.0 - fx) * (I[idx[2]] - I[idx[0]]) + fx * (I[idx[3]] - I[idx[1]]);
}

/*
 * Whether the step the tracker takes at the converged flow u is its least-squares one: the
 * fallback rule of track_point (weighted 2 x 2 matrix sum w g g^T, w = psi(r)/r, with a
 * determinant at most 1e-6 of the unweighted one's, or not a number) evaluated at u.  The forward
 * pass stopped on a step of that system there, so its fixed point solves the least-squares
 * equation sum r g = 0, and that is the equation the gradient differentiates (psi(r) = r).
 */
static int ls_regime(const double *I0, const double *I1, int W, int H, double px, double py, int r, double ux,
                     double uy, double sigma1, double sigma2)
{
    double a = 0.0, b = 0.0, c = 0.0, a0 = 0.0, b0 = 0.0, c0 = 0.0;
    for (int ky = -r; ky <= r; ++ky)
        for (int kx = -r; kx <= r; ++kx) {
            const double x = px + kx, y = py + ky;
            const double T = or_bilinear(I0, W, H, x, y);
            const double g0 = 0.5 * (or_bilinear(I0, W, H, x + 1.0, y) - or_bilinear(I0, W, H, x - 1.0, y));
            const double g1 = 0.5 * (or_bilinear(I0, W, H, x, y + 1.0) - or_bilinear(I0, W, H, x, y - 1.0));
            const double w = irls_weight(or_bilinear(I1, W, H, x + ux, y + uy) - T, sigma1, sigma2);
            a += w * g0 * g0;
            b += w * g0 * g1;
            c += w * g1 * g1;
            a0 += g0 * g0;
            b0 += g0 * g1;
            c0 += g1 * g1;
        }
    return !(a * c - b * b > 1e-6 * (a0 * c0 - b0 * b0));
}

/* The same for the illumination model (track_point_illum's rule: the weighted and unweighted
 * 4 x 4 systems with phi = ((1 + m) g, -T, -1) at the converged (u, m, c)). */
static int ls_regime_illum(const double *I0, const double *I1, int W, int H, double px, double py, int r,
                           double ux, double uy, double m, double c, double sigma1, double sigma2)
{
    double G[16] = {0}, G0[16] = {0};
    for (int ky = -r; ky <= r; ++ky)
        for (int kx = -r; kx <= r; ++kx) {
            const double x = px + kx, y = py + ky;
            const double T = or_bilinear(I0, W, H, x, y);
            const double g0 = 0.5 * (or_bilinear(I0, W, H, x + 1.0, y) - or_bilinear(I0, W, H, x - 1.0, y));
            const double g1 = 0.5 * (or_bilinear(I0, W, H, x, y + 1.0) - or_bilinear(I0, W, H, x, y - 1.0));
            const double res = or_bilinear(I1, W, H, x + ux, y + uy) - (1.0 + m) * T - c;
            const double w = irls_weight(res, sigma1, sigma2);
            const double phi[4] = {(1.0 + m) * g0, (1.0 + m) * g1, -T, -1.0};
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b) {
                    G[a * 4 + b] += w * phi[a] * phi[b];
                    G0[a * 4 + b] += phi[a] * phi[b];
                }
        }
    return !(det4(G) > 1e-6 * det4(G0));
}

/*
 * For every point with status CONVERGED, with upstream gradient lambda = dflow[i] (= dL/du):
 *   J = dF/du = sum_k psi'(r_k) g_k (grad B(I1, p + k + u))^T        (2x2, not symmetric)
 *   solve J^T mu = lambda
 *   dL/dI1[q] = - sum_k psi'(r_k) (mu . g_k) beta_k(q)
 *   dL/dI0[q] = + sum_k psi'(r_k) (mu . g_k) alpha_k(q) - sum_k psi(r_k) mu . dg_k/dI0[q]
 * where alpha_k, beta_k are the bilinear tap weights of the template sample and of the I1
 * sample, and g_k = (B(I0, x_k + e_x) - B(I0, x_k - e_x)) / 2 (and along y), so dg_k/dI0 is the
 * difference of the tap weights of the two shifted samples, halved.  Only the level-0 images
 * enter: coarser levels decide which fixed point is reached but not its local dependence.
 * Results are ADDED to dI0 and dI1 ([H][W] doubles).  I0, I1 are double images, pitch W.
 * dpoints (nullable, [n][2]) receives dL/dp, the gradient w.r.t. the point positions (zero for
 * points that contribute nothing).
 */
int or_track_grad(const double *I0, const double *I1, int W, int H, const double *pts, int64_t n, int support,
                  double sigma1, double sigma2, const double *flow, const uint8_t *status,
                  const double *dflow, double *dI0, double *dI1, double *dpoints)
{
    if (!I0 || !I1 || W <= 0 || H <= 0 || support < 1 || (support % 2) == 0) return OR_ERR_ARG;
    if (n > 0 && (!pts || !flow || !status || !dflow || !dI0 || !dI1)) return OR_ERR_ARG;
    const int r = support / 2;

    for (int64_t i = 0; i < n; ++i) {
        if (dpoints) {
            dpoints[2 * i] = 0.0;
            dpoints[2 * i + 1] = 0.0;
        }
        if (status[i] != OR_ST_CONVERGED) continue;
        const double px = pts[2 * i], py = pts[2 * i + 1];
        const double ux = flow[2 * i], uy = flow[2 * i + 1];
        /* the norm of the equation the forward pass stopped on (least squares in its fallback regime) */
        const int ls = ls_regime(I0, I1, W, H, px, py, r, ux, uy, sigma1, sigma2);
        const double s1 = ls ? INFINITY : sigma1, s2 = ls ? INFINITY : sigma2;

        /* J = sum psi' g (grad J)^T */
        double J00 = 0.0, J01 = 0.0, J10 = 0.0, J11 = 0.0;
        for (int ky = -r; ky <= r; ++ky)
            for (int kx = -r; kx <= r; ++kx) {
                double x = px + kx, y = py + ky;
                double T = or_bilinear(I0, W, H, x, y);
                double g0 = 0.5 * (or_bilinear(I0, W, H, x + 1.0, y) - or_bilinear(I0, W, H, x - 1.0, y));
                double g1 = 0.5 * (or_bilinear(I0, W, H, x, y + 1.0) - or_bilinear(I0, W, H, x, y - 1.0));
                int64_t idx[4]; double wt[4]; int cx[4], cy[4]; double fx, fy;
                bilinear_taps(W, H, x + ux, y + uy, idx, wt, cx, cy, &fx, &fy);
                double Jv = or_bilinear(I1, W, H, x + ux, y + uy);
                double djx = (1.0 - fy) * (I1[idx[1]] - I1[idx[0]]) + fy * (I1[idx[3]] - I1[idx[2]]);
                double djy = (1.0 - fx) * (I1[idx[2]] - I1[idx[0]]) + fx * (I1[idx[3]] - I1[idx[1]]);
                double dp = or_dpsi(Jv - T, s1, s2);
                J00 += dp * g0 * djx;
                J01 += dp * g0 * djy;
                J10 += dp * g1 * djx;
                J11 += dp * g1 * djy;
            }
        /* J^T mu = lambda, with J^T = [[J00, J10], [J01, J11]] */
        const double lx = dflow[2 * i], ly = dflow[2 * i + 1];
        const double det = J00 * J11 - J01 * J10;
        if (!(det != 0.0) || !isfinite(det)) continue;
        const double mux = (J11 * lx - J10 * ly) / det;
        const double muy = (J00 * ly - J01 * lx) / det;

        if (dpoints) {
            /* The flow also depends on the point: dF/dp = J + K with
             *   K = sum_k [ -psi'(r_k) g_k (grad B(I0, p + k))^T + psi(r_k) dG/dx(p + k) ],
             * G(x) = central differences of B(I0, .) at x, so dG/dx has rows
             * (grad B(I0, x + e_x) - grad B(I0, x - e_x)) / 2 and the same along y; then
             * du/dp = -J^-1 (J + K) and dL/dp = -lambda - K^T mu. */
            double K00 = 0.0, K01 = 0.0, K10 = 0.0, K11 = 0.0;
            for (int ky = -r; ky <= r; ++ky)
                for (int kx = -r; kx <= r; ++kx) {
                    double x = px + kx, y = py + ky;
                    double T = or_bilinear(I0, W, H, x, y);
                    double g0 = 0.5 * (or_bilinear(I0, W, H, x + 1.0, y) - or_bilinear(I0, W, H, x - 1.0, y));
                    double g1 = 0.5 * (or_bilinear(I0, W, H, x, y + 1.0) - or_bilinear(I0, W, H, x, y - 1.0));
                    double Jv = or_bilinear(I1, W, H, x + ux, y + uy);
                    double ps = or_psi(Jv - T, s1, s2), dp = or_dpsi(Jv - T, s1, s2);
                    double gT[2], gxp[2], gxm[2], gyp[2], gym[2];
                    bilinear_grad(I0, W, H, x, y, gT);
                    bilinear_grad(I0, W, H, x + 1.0, y, gxp);
                    bilinear_grad(I0, W, H, x - 1.0, y, gxm);
                    bilinear_grad(I0, W, H, x, y + 1.0, gyp);
                    bilinear_grad(I0, W, H, x, y - 1.0, gym);
                    K00 += -dp * g0 * gT[0] + ps * 0.5 * (gxp[0] - gxm[0]);
                    K01 += -dp * g0 * gT[1] + ps * 0.5 * (gxp[1] - gxm[1]);
                    K10 += -dp * g1 * gT[0] + ps * 0.5 * (gyp[0] - gym[0]);
                    K11 += -dp * g1 * gT[1] + ps * 0.5 * (gyp[1] - gym[1]);
                }
            dpoints[2 * i + 0] = -lx - (K00 * mux + K10 * muy);
            dpoints[2 * i + 1] = -ly - (K01 * mux + K11 * muy);
        }

        for (int ky = -r; ky <= r; ++ky)
            for (int kx = -r; kx <= r; ++kx) {
                double x = px + kx, y = py + ky;
                int64_t ia[4]; double wa[4]; int ax[4], ay[4]; double fxa, fya;
                bilinear_taps(W, H, x, y, ia, wa, ax, ay, &fxa, &fya);
                /* taps of the four shifted samples that form the template gradient */
                int64_t ixp[4], ixm[4], iyp[4], iym[4];
                double wxp[4], wxm[4], wyp[4], wym[4];
                int dcx[4], dcy[4]; double dfx, dfy;
                bilinear_taps(W, H, x + 1.0, y, ixp, wxp, dcx, dcy, &dfx, &dfy);
                bilinear_taps(W, H, x - 1.0, y, ixm, wxm, dcx, dcy, &dfx, &dfy);
                bilinear_taps(W, H, x, y + 1.0, iyp, wyp, dcx, dcy, &dfx, &dfy);
                bilinear_taps(W, H, x, y - 1.0, iym, wym, dcx, dcy, &dfx, &dfy);
                /* values as in the first pass (the taps only distribute the gradient) */
                double T = or_bilinear(I0, W, H, x, y);
                double g0 = 0.5 * (or_bilinear(I0, W, H, x + 1.0, y) - or_bilinear(I0, W, H, x - 1.0, y));
                double g1 = 0.5 * (or_bilinear(I0, W, H, x, y + 1.0) - or_bilinear(I0, W, H, x, y - 1.0));
                int64_t ib[4]; double wb[4]; int bxx[4], byy[4]; double fxb, fyb;
                bilinear_taps(W, H, x + ux, y + uy, ib, wb, bxx, byy, &fxb, &fyb);
                double Jv = or_bilinear(I1, W, H, x + ux, y + uy);
                double res = Jv - T;
                double ps = or_psi(res, s1, s2);
                double dp = or_dpsi(res, s1, s2);
                double mg = mux * g0 + muy * g1;
                const double cx = -ps * mux * 0.5, cy = -ps * muy * 0.5;
                for (int t = 0; t < 4; ++t) {
                    dI1[ib[t]] -= dp * mg * wb[t];
                    dI0[ia[t]] += dp * mg * wa[t];
                    dI0[ixp[t]] += cx * wxp[t];
                    dI0[ixm[t]] -= cx * wxm[t];
                    dI0[iyp[t]] += cy * wyp[t];
                    dI0[iym[t]] -= cy * wym[t];
                }
            }
    }
    return OR_OK;
}

/*
 * Implicit gradient of the illumination-model tracker (track_point_illum).  At a converged point
 * theta = (u, m, c) solves F(theta) = sum_k psi(r_k) phi_k = 0 with
 * r_k = B(I1, p + k + u) - (1 + m) T_k - c and phi_k = ((1 + m) g_k, -T_k, -1).  For the upstream
 * gradient lambda = (dL/du, 0, 0) (the loss depends on the flow only):
 *   A = dF/dtheta = sum_k psi'(r_k) phi_k (grad B(I1, p + k + u), -T_k, -1)^T
 *                   + sum_k psi(r_k) (g_k, 0, 0) in the column of m      (phi depends on m;
 *                     this term is (1 + m)^-1 times the d rows of F, so it vanishes at the fixed point)
 *   solve A^T mu = lambda,
 *   dL/dI1[q] = - sum_k psi'(r_k) (mu . phi_k) beta_k(q)
 *   dL/dI0[q] = sum_k [((1 + m) psi'(r_k) (mu . phi_k) + psi(r_k) mu_m) alpha_k(q)
 *                      - (1 + m) psi(r_k) mu_d . dg_k/dI0[q]]
 * illum holds (m, c) per point as the forward pass returned them.  Results are ADDED.
 */
int or_track_grad_illum(const double *I0, const double *I1, int W, int H, const double *pts, int64_t n, int support,
                        double sigma1, double sigma2, const double *flow, const double *illum, const uint8_t *status,
                        const double *dflow, double *dI0, double *dI1, double *dpoints)
{
    if (!I0 || !I1 || W <= 0 || H <= 0 || support < 1 || (support % 2) == 0) return OR_ERR_ARG;
    if (n > 0 && (!pts || !flow || !illum || !status || !dflow || !dI0 || !dI1)) return OR_ERR_ARG;
    const int r = support / 2;
    for (int64_t i = 0; i < n; ++i) {
        if (dpoints) {
            dpoints[2 * i] = 0.0;
            dpoints[2 * i + 1] = 0.0;
        }
        if (status[i] != OR_ST_CONVERGED) continue;
        const double px = pts[2 * i], py = pts[2 * i + 1];
        const double ux = flow[2 * i], uy = flow[2 * i + 1];
        const double m = illum[2 * i], c = illum[2 * i + 1];
        /* the norm of the equation the forward pass stopped on (least squares in its fallback regime) */
        const int ls = ls_regime_illum(I0, I1, W, H, px, py, r, ux, uy, m, c, sigma1, sigma2);
        const double s1 = ls ? INFINITY : sigma1, s2 = ls ? INFINITY : sigma2;
        double A[16] = {0};
        /* dependence of F on the point (the template moves with it, the images do not):
         * dF/dp = A[:, u] + K, K = sum -(1 + m) psi' phi (grad T)^T + psi dphi/dp with
         * dphi/dp = ((1 + m) dg/dp, -(grad T)^T, 0) */
        double K[4][2] = {{0}};
        for (int ky = -r; ky <= r; ++ky)
            for (int kx = -r; kx <= r; ++kx) {
                double x = px + kx, y = py + ky;
                double T = or_bilinear(I0, W, H, x, y);
                double g0 = 0.5 * (or_bilinear(I0, W, H, x + 1.0, y) - or_bilinear(I0, W, H, x - 1.0, y));
                double g1 = 0.5 * (or_bilinear(I0, W, H, x, y + 1.0) - or_bilinear(I0, W, H, x, y - 1.0));
                double gJ[2];
                bilinear_grad(I1, W, H, x + ux, y + uy, gJ);
                double res = or_bilinear(I1, W, H, x + ux, y + uy) - (1.0 + m) * T - c;
                double ps = or_psi(res, s1, s2), dp = or_dpsi(res, s1, s2);
                double phi[4] = {(1.0 + m) * g0, (1.0 + m) * g1, -T, -1.0};
                double dr[4] = {gJ[0], gJ[1], -T, -1.0};
                for (int a = 0; a < 4; ++a)
                    for (int b = 0; b < 4; ++b) A[a * 4 + b] += dp * phi[a] * dr[b];
                A[0 * 4 + 2] += ps * g0;
                A[1 * 4 + 2] += ps * g1;
                if (dpoints) {
                    double gT[2], gxp[2], gxm[2], gyp[2], gym[2];
                    bilinear_grad(I0, W, H, x, y, gT);
                    bilinear_grad(I0, W, H, x + 1.0, y, gxp);
                    bilinear_grad(I0, W, H, x - 1.0, y, gxm);
                    bilinear_grad(I0, W, H, x, y + 1.0, gyp);
                    bilinear_grad(I0, W, H, x, y - 1.0, gym);
                    for (int b = 0; b < 2; ++b) {
                        for (int a = 0; a < 4; ++a) K[a][b] += -(1.0 + m) * dp * phi[a] * gT[b];
                        K[0][b] += ps * (1.0 + m) * 0.5 * (gxp[b] - gxm[b]);
                        K[1][b] += ps * (1.0 + m) * 0.5 * (gyp[b] - gym[b]);
                        K[2][b] += -ps * gT[b];
                    }
                }
            }
        double At[16], lam[4] = {dflow[2 * i], dflow[2 * i + 1], 0.0, 0.0}, mu[4];
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) At[a * 4 + b] = A[b * 4 + a];
        if (solve_dense(At, lam, 4, mu) != 0 || !(isfinite(mu[0]) && isfinite(mu[1]) && isfinite(mu[2]) && isfinite(mu[3])))
            continue;
        if (dpoints) /* du/dp = -I - (A^-1 K)[u rows], so dL/dp = -lambda - K^T mu */
            for (int b = 0; b < 2; ++b)
                dpoints[2 * i + b] = -dflow[2 * i + b] - (K[0][b] * mu[0] + K[1][b] * mu[1] + K[2][b] * mu[2] +
                                                          K[3][b] * mu[3]);
        for (int ky = -r; ky <= r; ++ky)
            for (int kx = -r; kx <= r; ++kx) {
                double x = px + kx, y = py + ky;
                int64_t ia[4], ixp[4], ixm[4], iyp[4], iym[4], ib[4];
                double wa[4], wxp[4], wxm[4], wyp[4], wym[4], wb[4];
                int ccx[4], ccy[4]; double ffx, ffy;
                bilinear_taps(W, H, x, y, ia, wa, ccx, ccy, &ffx, &ffy);
                bilinear_taps(W, H, x + 1.0, y, ixp, wxp, ccx, ccy, &ffx, &ffy);
                bilinear_taps(W, H, x - 1.0, y, ixm, wxm, ccx, ccy, &ffx, &ffy);
                bilinear_taps(W, H, x, y + 1.0, iyp, wyp, ccx, ccy, &ffx, &ffy);
                bilinear_taps(W, H, x, y - 1.0, iym, wym, ccx, ccy, &ffx, &ffy);
                bilinear_taps(W, H, x + ux, y + uy, ib, wb, ccx, ccy, &ffx, &ffy);
                /* values as in the first pass (the taps only distribute the gradient) */
                double T = or_bilinear(I0, W, H, x, y);
                double g0 = 0.5 * (or_bilinear(I0, W, H, x + 1.0, y) - or_bilinear(I0, W, H, x - 1.0, y));
                double g1 = 0.5 * (or_bilinear(I0, W, H, x, y + 1.0) - or_bilinear(I0, W, H, x, y - 1.0));
                double Jv = or_bilinear(I1, W, H, x + ux, y + uy);
                double res = Jv - (1.0 + m) * T - c;
                double ps = or_psi(res, s1, s2), dp = or_dpsi(res, s1, s2);
                double mphi = mu[0] * (1.0 + m) * g0 + mu[1] * (1.0 + m) * g1 - mu[2] * T - mu[3];
                double a0 = (1.0 + m) * dp * mphi + ps * mu[2];
                double cx = -0.5 * (1.0 + m) * ps * mu[0], cy = -0.5 * (1.0 + m) * ps * mu[1];
                for (int t = 0; t < 4; ++t) {
                    dI1[ib[t]] -= dp * mphi * wb[t];
                    dI0[ia[t]] += a0 * wa[t];
                    dI0[ixp[t]] += cx * wxp[t];
                    dI0[ixm[t]] -= cx * wxm[t];
                    dI0[iyp[t]] += cy * wyp[t];
                    dI0[iym[t]] -= cy * wym[t];
                }
            }
    }
    return OR_OK;
}
