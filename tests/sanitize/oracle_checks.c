/* Runs every oracle entry point on small seeded inputs, for the AddressSanitizer and
 * UndefinedBehaviorSanitizer build of tests/test_sanitizers.py: a clean run (exit 0, no report)
 * shows the oracle's indexing stays inside its buffers on these shapes, borders included. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int64_t or_detect_count(int W, int H, int win, int stride);
int64_t or_detect(const uint8_t *img, int W, int H, int64_t pitch, int win, int stride, int m_mode, double *pts,
                  uint8_t *sel, double *resp, int nthreads);
int64_t or_detect_f64(const double *img, int W, int H, int64_t pitch, int win, int stride, double *pts, uint8_t *sel);
int or_detect_grad(const double *img, int W, int H, int64_t pitch, int win, int stride, const uint8_t *sel,
                   const double *dpoints, double *dI);
int or_pyr_down_u8(const uint8_t *src, int W, int H, int64_t pitch, uint8_t *dst);
int or_pyr_down_f64(const double *src, int W, int H, double *dst);
int or_track(const void *I0, const void *I1, int dtype, int W, int H, int64_t pitch, const double *pts, int64_t n,
             int levels, int support, int iters, double sigma1, double sigma2, double eps_coarse, double eps_fine,
             double min_eig, int illum, int cross, double tau, int gm, double *flow, uint8_t *status,
             int32_t *iters_out, double *illum_out, double *gm_out, int nthreads);
int or_track_grad(const double *I0, const double *I1, int W, int H, const double *pts, int64_t n, int support,
                  double sigma1, double sigma2, const double *flow, const uint8_t *status, const double *dflow,
                  double *dI0, double *dI1, double *dpoints);
int or_track_grad_illum(const double *I0, const double *I1, int W, int H, const double *pts, int64_t n, int support,
                        double sigma1, double sigma2, const double *flow, const double *illum, const uint8_t *status,
                        const double *dflow, double *dI0, double *dI1, double *dpoints);
int or_gm_fit(const double *pts, const double *mot, const uint8_t *use, int64_t n, double cx, double cy,
              double scale, int iters, double *A);
int or_epic(const uint8_t *I, int W, int H, int64_t pitch, const double *pts, const double *flow,
            const uint8_t *status, int64_t n, int k, int kappa, int h, double *dense, int64_t *D_out,
            int32_t *L_out, int32_t *nb_out, int64_t *nd_out, double *model_out, uint8_t *alive_out);

static uint32_t rng = 12345u;
static double urand(void) { rng = rng * 1664525u + 1013904223u; return (rng >> 8) * (1.0 / 16777216.0); }

#define CHECK(c)                                                                                                   \
    do {                                                                                                           \
        if (!(c)) {                                                                                                \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__);                                         \
            return 1;                                                                                              \
        }                                                                                                          \
    } while (0)

int main(void)
{
    const int W = 61, H = 47; /* odd sizes: every pyramid level has a ragged border */
    uint8_t *u0 = malloc(W * H), *u1 = malloc(W * H);
    double *f0 = malloc(sizeof(double) * W * H), *f1 = malloc(sizeof(double) * W * H);
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            /* smooth texture plus noise, shifted by (1.3, -0.6) in the second frame */
            const double a = 120.0 + 60.0 * sin(0.31 * x) * cos(0.23 * y) + 20.0 * urand();
            const double b = 120.0 + 60.0 * sin(0.31 * (x - 1.3)) * cos(0.23 * (y + 0.6)) + 20.0 * urand();
            f0[y * W + x] = a;
            f1[y * W + x] = b;
            u0[y * W + x] = (uint8_t)a;
            u1[y * W + x] = (uint8_t)b;
        }
    const int64_t n = or_detect_count(W, H, 9, 4);
    CHECK(n > 0);
    double *pts = malloc(sizeof(double) * 2 * (n + 2)), *resp = malloc(sizeof(double) * n);
    uint8_t *sel = malloc(n);
    CHECK(or_detect(u0, W, H, W, 9, 4, 0, pts, sel, resp, 2) == n);
    CHECK(or_detect_f64(f0, W, H, W, 9, 4, pts, sel) == n);
    /* two extra points: on the border and outside the image */
    pts[2 * n] = 0.0;
    pts[2 * n + 1] = H - 1;
    pts[2 * n + 2] = W + 3.5;
    pts[2 * n + 3] = -2.0;
    const int64_t m = n + 2;
    uint8_t *pyr8 = malloc(W * H);
    double *pyrf = malloc(sizeof(double) * W * H);
    CHECK(or_pyr_down_u8(u0, W, H, W, pyr8) == 0);
    CHECK(or_pyr_down_f64(f0, W, H, pyrf) == 0);
    double *flow = malloc(sizeof(double) * 2 * m), *ill = malloc(sizeof(double) * 2 * m), A[6];
    uint8_t *st = malloc(m);
    int32_t *its = malloc(sizeof(int32_t) * m * 4);
    /* every tracker form, uint8 and real frames */
    for (int form = 0; form < 8; ++form) {
        const int illum = form & 1, cross = (form >> 1) & 1, gm = (form >> 2) & 1;
        CHECK(or_track(u0, u1, 0, W, H, W, pts, m, 3, 9, 10, 8.0, 32.0, 1e-2, 1e-4, 6.5, illum, cross, 25.0, gm, flow,
                       st, its, ill, A, 2) == 0);
        CHECK(or_track(f0, f1, 1, W, H, W, pts, m, 4, 7, 10, 8.0, 32.0, 1e-2, 1e-4, 6.5, illum, cross, 25.0, gm, flow,
                       st, its, ill, A, 2) == 0);
    }
    /* the implicit gradients at the last forward result (plain, then illumination model) */
    double *df = malloc(sizeof(double) * 2 * m), *d0 = calloc(W * H, sizeof(double)), *d1 = calloc(W * H, sizeof(double));
    double *dp = malloc(sizeof(double) * 2 * m);
    for (int64_t i = 0; i < 2 * m; ++i) df[i] = urand() - 0.5;
    CHECK(or_track(f0, f1, 1, W, H, W, pts, m, 1, 7, 30, 8.0, 32.0, 1e-2, 1e-6, 6.5, 0, 0, 25.0, 0, flow, st, NULL,
                   NULL, NULL, 2) == 0);
    CHECK(or_track_grad(f0, f1, W, H, pts, m, 7, 8.0, 32.0, flow, st, df, d0, d1, dp) == 0);
    CHECK(or_track(f0, f1, 1, W, H, W, pts, m, 1, 7, 30, 8.0, 32.0, 1e-2, 1e-6, 6.5, 1, 0, 25.0, 0, flow, st, NULL,
                   ill, NULL, 2) == 0);
    CHECK(or_track_grad_illum(f0, f1, W, H, pts, m, 7, 8.0, 32.0, flow, ill, st, df, d0, d1, dp) == 0);
    CHECK(or_detect_grad(f0, W, H, W, 9, 4, sel, dp, d0) == 0);
    /* the global fit on the tracked samples */
    uint8_t *use = malloc(m);
    for (int64_t i = 0; i < m; ++i) use[i] = st[i] == 0;
    or_gm_fit(pts, flow, use, m, 0.5 * (W - 1), 0.5 * (H - 1), 4.0, 10, A);
    /* dense interpolation of the tracked points */
    double *dense = malloc(sizeof(double) * 2 * W * H);
    CHECK(or_epic(u0, W, H, W, pts, flow, st, m, 8, 8, 64, dense, NULL, NULL, NULL, NULL, NULL, NULL) == 0);
    printf("oracle checks passed (%lld points)\n", (long long)m);
    free(u0); free(u1); free(f0); free(f1); free(pts); free(resp); free(sel); free(pyr8); free(pyrf); free(flow);
    free(ill); free(st); free(its); free(df); free(d0); free(d1); free(dp); free(use); free(dense);
    return 0;
}
