/*
 * epic_oracle.c -- plain FP64 CPU oracle for the edge-preserving interpolation of the tracked
 * points into a dense flow field.
 *
 * TEST INFRASTRUCTURE ONLY (same rules as degraf_oracle.c: only the tests, the smoke check and
 * the benchmark's CPU-baseline leg use it; it shares nothing with the HIP library).
 *
 * Source: DeGraF-Flow, Section 2 "Interpolation" and Section 3 "Parameters": the dense field is
 * obtained by fitting, for every pixel, an affine motion to the k nearest tracked points, nearness
 * being a geodesic distance that penalises crossing image edges, the edges taken from image
 * gradients; k = 128.  The construction of the geodesic neighbours follows the cited
 * interpolator (EpicFlow): a geodesic Voronoi partition of the pixels among the points, a graph
 * on the points whose edges join adjacent cells, and neighbours and distances taken on that graph,
 * so that all pixels of one cell share their point's model.  The readings that make each step
 * exact (integer edge map and step costs, tie rules, weights, degenerate fits) are stated at each
 * function; distances are exact integers, so the partition, the graph and the neighbour lists
 * are unique.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_ERR_ARG (-1)
#define OR_ERR_MEM (-2)

static int clampi_e(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* Edge map from image gradients: E(x, y) = |I(x+1, y) - I(x-1, y)| + |I(x, y+1) - I(x, y-1)|
 * (central differences, replicated border), an integer in [0, 510]. */
void or_epic_edges(const uint8_t *I, int W, int H, int64_t pitch, int32_t *E)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            const int xl = clampi_e(x - 1, 0, W - 1), xr = clampi_e(x + 1, 0, W - 1);
            const int yu = clampi_e(y - 1, 0, H - 1), yd = clampi_e(y + 1, 0, H - 1);
            const int gx = (int)I[(int64_t)y * pitch + xr] - (int)I[(int64_t)y * pitch + xl];
            const int gy = (int)I[(int64_t)yd * pitch + x] - (int)I[(int64_t)yu * pitch + x];
            E[(int64_t)y * W + x] = abs(gx) + abs(gy);
        }
}

/* ---- binary min-heap of (key, payload), keys compared lexicographically ------------------ */
typedef struct {
    int64_t k0, k1; /* primary: distance; secondary: label or node index */
    int64_t v;      /* payload: pixel or node */
} hitem;
typedef struct {
    hitem *a;
    int64_t n, cap;
} heap_t;

static int hless(const hitem *x, const hitem *y) { return x->k0 < y->k0 || (x->k0 == y->k0 && x->k1 < y->k1); }

static int hpush(heap_t *h, int64_t k0, int64_t k1, int64_t v)
{
    if (h->n == h->cap) {
        int64_t nc = h->cap ? 2 * h->cap : 1024;
        hitem *na = (hitem *)realloc(h->a, (size_t)nc * sizeof(hitem));
        if (!na) return -1;
        h->a = na;
        h->cap = nc;
    }
    int64_t i = h->n++;
    hitem it = {k0, k1, v};
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (!hless(&it, &h->a[p])) break;
        h->a[i] = h->a[p];
        i = p;
    }
    h->a[i] = it;
    return 0;
}

static hitem hpop(heap_t *h)
{
    hitem top = h->a[0], last = h->a[--h->n];
    int64_t i = 0;
    for (;;) {
        int64_t c = 2 * i + 1;
        if (c >= h->n) break;
        if (c + 1 < h->n && hless(&h->a[c + 1], &h->a[c])) ++c;
        if (!hless(&h->a[c], &last)) break;
        h->a[i] = h->a[c];
        i = c;
    }
    if (h->n > 0) h->a[i] = last;
    return top;
}

/* Seed pixel of a point: (floor(x + 1/2), floor(y + 1/2)) clamped into the image. */
static int64_t seed_pixel(double x, double y, int W, int H)
{
    const int px = clampi_e((int)floor(x + 0.5), 0, W - 1), py = clampi_e((int)floor(y + 0.5), 0, H - 1);
    return (int64_t)py * W + px;
}

/*
 * Geodesic Voronoi partition.  Step cost between 4-neighbours p, q: kappa + E(p) + E(q) (an
 * integer, so path costs are exact).  Seeds: the points with status 0 (converged) whose position
 * and flow (nullable) are finite, at their seed pixels; a point whose seed pixel is that of a
 * lower-index seed is dropped.  For every pixel q:
 * D(q) = the least path cost from any seed, L(q) = the lowest seed index among the seeds that
 * reach q at cost D(q) (-1 and D = -1 when there is no seed).  Dijkstra on keys (cost, label)
 * ordered lexicographically: cost and label both carry along a path, so the least key of q is
 * (D(q), L(q)) exactly.
 */
int or_epic_voronoi(const uint8_t *I, int W, int H, int64_t pitch, const double *pts, const double *flow,
                    const uint8_t *status, int64_t n, int kappa, int64_t *D, int32_t *L, uint8_t *alive)
{
    if (W <= 0 || H <= 0 || kappa < 1) return OR_ERR_ARG;
    const int64_t N = (int64_t)W * H;
    int32_t *E = (int32_t *)malloc((size_t)N * sizeof(int32_t));
    if (!E) return OR_ERR_MEM;
    or_epic_edges(I, W, H, pitch, E);
    for (int64_t q = 0; q < N; ++q) {
        D[q] = -1;
        L[q] = -1;
    }
    heap_t h = {0, 0, 0};
    for (int64_t i = 0; i < n; ++i) {
        alive[i] = 0;
        if (status[i] != 0) continue;
        if (!isfinite(pts[2 * i]) || !isfinite(pts[2 * i + 1])) continue; /* cannot be placed */
        if (flow && (!isfinite(flow[2 * i]) || !isfinite(flow[2 * i + 1]))) continue;
        const int64_t q = seed_pixel(pts[2 * i], pts[2 * i + 1], W, H);
        if (L[q] >= 0) continue; /* pixel already seeded by a lower index */
        D[q] = 0;
        L[q] = (int32_t)i;
        alive[i] = 1;
        if (hpush(&h, 0, i, q)) {
            free(E);
            free(h.a);
            return OR_ERR_MEM;
        }
    }
    uint8_t *done = (uint8_t *)calloc((size_t)N, 1);
    if (!done) {
        free(E);
        free(h.a);
        return OR_ERR_MEM;
    }
    static const int dx[4] = {1, -1, 0, 0}, dy[4] = {0, 0, 1, -1};
    while (h.n > 0) {
        const hitem it = hpop(&h);
        const int64_t p = it.v;
        if (done[p]) continue;
        if (it.k0 != D[p] || it.k1 != L[p]) continue; /* stale entry */
        done[p] = 1;
        const int x = (int)(p % W), y = (int)(p / W);
        for (int k = 0; k < 4; ++k) {
            const int xn = x + dx[k], yn = y + dy[k];
            if (xn < 0 || yn < 0 || xn >= W || yn >= H) continue;
            const int64_t q = (int64_t)yn * W + xn;
            if (done[q]) continue;
            const int64_t c = it.k0 + kappa + E[p] + E[q];
            if (D[q] < 0 || c < D[q] || (c == D[q] && it.k1 < L[q])) {
                D[q] = c;
                L[q] = (int32_t)it.k1;
                if (hpush(&h, c, it.k1, q)) {
                    free(E);
                    free(done);
                    free(h.a);
                    return OR_ERR_MEM;
                }
            }
        }
    }
    free(E);
    free(done);
    free(h.a);
    return OR_OK;
}

typedef struct {
    int64_t s, t, w;
} edge_t;

static int edge_cmp(const void *a, const void *b)
{
    const edge_t *x = (const edge_t *)a, *y = (const edge_t *)b;
    if (x->s != y->s) return x->s < y->s ? -1 : 1;
    if (x->t != y->t) return x->t < y->t ? -1 : 1;
    return x->w < y->w ? -1 : (x->w > y->w);
}

/*
 * Graph on the seeds: s and t (s != t) are joined when some 4-adjacent pixel pair (p, q) has
 * L(p) = s and L(q) = t; the edge length is the least D(p) + (kappa + E(p) + E(q)) + D(q) over
 * such pairs (the cost of the cheapest pixel path from s to t through that pair).  Written as a
 * CSR: adj_off[n + 1], adj_t[], adj_w[] (allocated here, freed by the caller).
 */
static int seed_graph(const int32_t *E, int W, int H, const int64_t *D, const int32_t *L, int64_t n, int kappa,
                      int64_t **adj_off, int64_t **adj_t, int64_t **adj_w)
{
    const int64_t N = (int64_t)W * H;
    edge_t *e = (edge_t *)malloc((size_t)(4 * N + 1) * sizeof(edge_t));
    if (!e) return OR_ERR_MEM;
    int64_t m = 0;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            const int64_t p = (int64_t)y * W + x;
            const int64_t nb[2] = {x + 1 < W ? p + 1 : -1, y + 1 < H ? p + W : -1};
            for (int k = 0; k < 2; ++k) {
                const int64_t q = nb[k];
                if (q < 0 || L[p] == L[q] || L[p] < 0 || L[q] < 0) continue;
                const int64_t w = D[p] + kappa + E[p] + E[q] + D[q];
                e[m++] = (edge_t){L[p], L[q], w};
                e[m++] = (edge_t){L[q], L[p], w};
            }
        }
    qsort(e, (size_t)m, sizeof(edge_t), edge_cmp);
    int64_t *off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *tt = (int64_t *)malloc((size_t)(m + 1) * sizeof(int64_t));
    int64_t *ww = (int64_t *)malloc((size_t)(m + 1) * sizeof(int64_t));
    if (!off || !tt || !ww) {
        free(e);
        free(off);
        free(tt);
        free(ww);
        return OR_ERR_MEM;
    }
    int64_t u = 0;
    for (int64_t i = 0; i < m; ++i) {
        if (i > 0 && e[i].s == e[i - 1].s && e[i].t == e[i - 1].t) continue; /* sorted: first is least */
        tt[u] = e[i].t;
        ww[u] = e[i].w;
        off[e[i].s + 1]++;
        ++u;
    }
    for (int64_t s = 0; s < n; ++s) off[s + 1] += off[s];
    free(e);
    *adj_off = off;
    *adj_t = tt;
    *adj_w = ww;
    return OR_OK;
}

/* Weighted least-squares affine model of the flow around one seed, centred at the seed's own
 * position (sx, sy):  u(x, y) = A (x - sx, y - sy, 1)^T with A 2x3 (row-major model[6]).
 * Weights w_j = 2^(-delta_j / h).  Degenerate (fewer than 3 neighbours, or a weighted position
 * covariance C with det C <= 1e-4 (tr C)^2): the weighted mean flow, model = (0, 0, mx, 0, 0, my).
 * Otherwise the minimiser of sum_j w_j |A (x_j, y_j, 1) - u_j|^2, computed by Householder QR of
 * the rows sqrt(w_j) (1, x_j, y_j) (the weights can span 64 binades, far beyond what the normal
 * equations resolve). */
static void fit_affine(const double *pts, const double *flow, const int32_t *nb, const int64_t *nd, int cnt,
                       int64_t s, int h, double model[6])
{
    const double sx = pts[2 * s], sy = pts[2 * s + 1];
    double sw = 0, sx1 = 0, sy1 = 0, sxx = 0, sxy = 0, syy = 0, mx = 0, my = 0;
    for (int j = 0; j < cnt; ++j) {
        const int64_t t = nb[j];
        const double w = exp2(-(double)nd[j] / (double)h);
        const double x = pts[2 * t] - sx, y = pts[2 * t + 1] - sy;
        sw += w;
        sx1 += w * x;
        sy1 += w * y;
        sxx += w * x * x;
        sxy += w * x * y;
        syy += w * y * y;
        mx += w * flow[2 * t];
        my += w * flow[2 * t + 1];
    }
    /* weighted covariance of the positions about their weighted mean */
    const double ex = sx1 / sw, ey = sy1 / sw;
    const double cxx = sxx / sw - ex * ex, cyy = syy / sw - ey * ey, cxy = sxy / sw - ex * ey;
    const double tr = cxx + cyy, det = cxx * cyy - cxy * cxy;
    if (cnt < 3 || !(det > 1e-4 * tr * tr)) {
        model[0] = model[1] = model[3] = model[4] = 0.0;
        model[2] = mx / sw;
        model[5] = my / sw;
        return;
    }
    /* rows sqrt(w) (1, x, y | u, v); Householder reflections zero each column below the diagonal */
    double *R = (double *)malloc((size_t)cnt * 5 * sizeof(double));
    if (!R) {
        for (int e = 0; e < 6; ++e) model[e] = NAN;
        return;
    }
    for (int j = 0; j < cnt; ++j) {
        const int64_t t = nb[j];
        const double r = sqrt(exp2(-(double)nd[j] / (double)h));
        R[5 * j + 0] = r;
        R[5 * j + 1] = r * (pts[2 * t] - sx);
        R[5 * j + 2] = r * (pts[2 * t + 1] - sy);
        R[5 * j + 3] = r * flow[2 * t];
        R[5 * j + 4] = r * flow[2 * t + 1];
    }
    for (int c = 0; c < 3; ++c) {
        double norm = 0;
        for (int j = c; j < cnt; ++j) norm += R[5 * j + c] * R[5 * j + c];
        norm = sqrt(norm);
        const double alpha = R[5 * c + c] > 0 ? -norm : norm; /* reflect onto -sign(x0) |x| e0 */
        /* v = x - alpha e0, applied as H = I - 2 v v^T / (v^T v) to the remaining columns */
        const double v0 = R[5 * c + c] - alpha;
        double vv = v0 * v0;
        for (int j = c + 1; j < cnt; ++j) vv += R[5 * j + c] * R[5 * j + c];
        if (vv > 0)
            for (int e = c + 1; e < 5; ++e) {
                double dot = v0 * R[5 * c + e];
                for (int j = c + 1; j < cnt; ++j) dot += R[5 * j + c] * R[5 * j + e];
                const double f = 2.0 * dot / vv;
                R[5 * c + e] -= f * v0;
                for (int j = c + 1; j < cnt; ++j) R[5 * j + e] -= f * R[5 * j + c];
            }
        R[5 * c + c] = alpha;
        for (int j = c + 1; j < cnt; ++j) R[5 * j + c] = 0.0;
    }
    /* back substitution R c = (Q^T b)[0:3] for each right-hand side; c = (offset, d/dx, d/dy) */
    for (int rhs = 0; rhs < 2; ++rhs) {
        double c3[3];
        for (int r = 2; r >= 0; --r) {
            double acc = R[5 * r + 3 + rhs];
            for (int e = r + 1; e < 3; ++e) acc -= R[5 * r + e] * c3[e];
            c3[r] = acc / R[5 * r + r];
        }
        model[3 * rhs + 0] = c3[1];
        model[3 * rhs + 1] = c3[2];
        model[3 * rhs + 2] = c3[0];
    }
    free(R);
}

/*
 * The whole interpolation.  Inputs: the uint8 frame I (W x H, row pitch in bytes), n points
 * (x, y) with their flows and tracker statuses.  Parameters: k (neighbours per seed), kappa (flat
 * step cost), h (weight half-distance, in the same cost units).
 *   1. Voronoi partition and distances (or_epic_voronoi).
 *   2. Seed graph (seed_graph).
 *   3. For each live seed s: the seeds nearest to s on the graph, in increasing (distance, index)
 *      order, s itself first at 0, at most k of them and only those at graph distance <= 64 h
 *      (weight >= 2^-64): Dijkstra from s stopped after k settles.  nb[s][j], nd[s][j]; unused
 *      slots -1.
 *   4. The affine model of each live seed (fit_affine); dead seeds get NaN.
 *   5. Every pixel q takes the model of its cell's seed s = L(q), evaluated at q = (x, y): the
 *      geodesic distance from q to a seed t is read as D(q) + delta(s, t), whose common term
 *      D(q) scales all of q's weights alike and so drops out of the fit.
 * Outputs (all nullable except dense): dense[H][W][2], D[H][W], L[H][W], nb[n][k], nd[n][k],
 * model[n][6], alive[n].  No seed at all: dense is NaN everywhere.
 */
int or_epic(const uint8_t *I, int W, int H, int64_t pitch, const double *pts, const double *flow,
            const uint8_t *status, int64_t n, int k, int kappa, int h, double *dense, int64_t *D_out,
            int32_t *L_out, int32_t *nb_out, int64_t *nd_out, double *model_out, uint8_t *alive_out)
{
    if (W <= 0 || H <= 0 || k < 1 || kappa < 1 || h < 1 || n < 0 || !dense) return OR_ERR_ARG;
    const int64_t N = (int64_t)W * H;
    int rc = OR_ERR_MEM;
    int64_t *D = (int64_t *)malloc((size_t)N * sizeof(int64_t));
    int32_t *L = (int32_t *)malloc((size_t)N * sizeof(int32_t));
    int32_t *E = (int32_t *)malloc((size_t)N * sizeof(int32_t));
    uint8_t *alive = (uint8_t *)malloc((size_t)n + 1);
    int32_t *nb = (int32_t *)malloc((size_t)(n * k + 1) * sizeof(int32_t));
    int64_t *nd = (int64_t *)malloc((size_t)(n * k + 1) * sizeof(int64_t));
    double *model = (double *)malloc((size_t)(6 * n + 1) * sizeof(double));
    int64_t *adj_off = NULL, *adj_t = NULL, *adj_w = NULL;
    if (!D || !L || !E || !alive || !nb || !nd || !model) goto out;
    if ((rc = or_epic_voronoi(I, W, H, pitch, pts, flow, status, n, kappa, D, L, alive)) != OR_OK) goto out;
    or_epic_edges(I, W, H, pitch, E);
    if ((rc = seed_graph(E, W, H, D, L, n, kappa, &adj_off, &adj_t, &adj_w)) != OR_OK) goto out;
    const int64_t dmax = 64 * (int64_t)h;

    int fail = 0;
#pragma omp parallel
    {
        int64_t *dist = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
        uint8_t *settled = (uint8_t *)calloc((size_t)n + 1, 1);
        int64_t *touched = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
        heap_t hp = {0, 0, 0};
        if (!dist || !settled || !touched) {
#pragma omp atomic write
            fail = 1;
        } else {
            for (int64_t i = 0; i < n; ++i) dist[i] = -1;
#pragma omp for schedule(dynamic, 64)
            for (int64_t s = 0; s < n; ++s) {
                int32_t *nbs = nb + s * k;
                int64_t *nds = nd + s * k;
                for (int j = 0; j < k; ++j) {
                    nbs[j] = -1;
                    nds[j] = -1;
                }
                if (!alive[s]) {
                    for (int j = 0; j < 6; ++j) model[6 * s + j] = NAN;
                    continue;
                }
                int64_t nt = 0;
                int cnt = 0;
                hp.n = 0;
                dist[s] = 0;
                touched[nt++] = s;
                if (hpush(&hp, 0, s, s)) {
#pragma omp atomic write
                    fail = 1;
                }
                while (hp.n > 0 && cnt < k) {
                    const hitem it = hpop(&hp);
                    const int64_t v = it.v;
                    if (settled[v] || it.k0 != dist[v]) continue;
                    settled[v] = 1;
                    nbs[cnt] = (int32_t)v;
                    nds[cnt] = it.k0;
                    ++cnt;
                    for (int64_t e = adj_off[v]; e < adj_off[v + 1]; ++e) {
                        const int64_t t = adj_t[e], c = it.k0 + adj_w[e];
                        if (settled[t] || c > dmax) continue;
                        if (dist[t] < 0 || c < dist[t]) {
                            if (dist[t] < 0) touched[nt++] = t;
                            dist[t] = c;
                            if (hpush(&hp, c, t, t)) {
#pragma omp atomic write
                                fail = 1;
                            }
                        }
                    }
                }
                for (int64_t j = 0; j < nt; ++j) {
                    dist[touched[j]] = -1;
                    settled[touched[j]] = 0;
                }
                fit_affine(pts, flow, nbs, nds, cnt, s, h, model + 6 * s);
            }
        }
        free(dist);
        free(settled);
        free(touched);
        free(hp.a);
    }
    if (fail) {
        rc = OR_ERR_MEM;
        goto out;
    }
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            const int64_t q = (int64_t)y * W + x;
            const int32_t s = L[q];
            if (s < 0) {
                dense[2 * q] = dense[2 * q + 1] = NAN;
                continue;
            }
            const double *m = model + 6 * (int64_t)s;
            const double rx = x - pts[2 * s], ry = y - pts[2 * s + 1];
            dense[2 * q] = m[0] * rx + m[1] * ry + m[2];
            dense[2 * q + 1] = m[3] * rx + m[4] * ry + m[5];
        }
    if (D_out) memcpy(D_out, D, (size_t)N * sizeof(int64_t));
    if (L_out) memcpy(L_out, L, (size_t)N * sizeof(int32_t));
    if (nb_out) memcpy(nb_out, nb, (size_t)(n * k) * sizeof(int32_t));
    if (nd_out) memcpy(nd_out, nd, (size_t)(n * k) * sizeof(int64_t));
    if (model_out) memcpy(model_out, model, (size_t)(6 * n) * sizeof(double));
    if (alive_out) memcpy(alive_out, alive, (size_t)n);
    rc = OR_OK;
out:
    free(D);
    free(L);
    free(E);
    free(alive);
    free(nb);
    free(nd);
    free(model);
    free(adj_off);
    free(adj_t);
    free(adj_w);
    return rc;
}

/* Endpoint error of a dense field against a reference (the norm of the difference; Eq. 3 is read
 * as the plain norm) over the pixels with valid[q] != 0: sum of errors, count of errors above
 * `thresh` px, and the count of pixels.  out[0] = sum EPE, out[1] = outliers, out[2] = count. */
void or_flow_error(const double *flow, const double *ref, const uint8_t *valid, int64_t npix, double thresh,
                   double out[3])
{
    double se = 0, no = 0, nc = 0;
    for (int64_t q = 0; q < npix; ++q) {
        if (valid && !valid[q]) continue;
        const double ex = flow[2 * q] - ref[2 * q], ey = flow[2 * q + 1] - ref[2 * q + 1];
        const double e = sqrt(ex * ex + ey * ey);
        se += e;
        no += e > thresh;
        nc += 1;
    }
    out[0] = se;
    out[1] = no;
    out[2] = nc;
}
