// epic.hip -- dense flow from the tracked points by edge-preserving interpolation (DeGraF-Flow,
// Section 2 "Interpolation"; k from Section 3 "Parameters").  Every pixel takes an affine motion
// fitted to the k tracked points nearest to it in a geodesic distance that penalises crossing
// edges of an image-gradient map.  Geodesic neighbours are built as in the cited interpolator:
// a geodesic Voronoi partition of the pixels among the points, a graph on the points joining
// adjacent cells, and neighbour searches on that graph, so every pixel of a cell shares its
// point's model.
//
// GPU structure (one pass each unless noted):
//   k_epic_prep     edge map (uint16) and cleared tables, HBM bound
//   k_epic_seed     one 64-bit atomicMin per converged point: key = (0 << 32) | index
//   k_epic_relax    32x32 tiles relaxed in LDS to a local fixed point, written back with 64-bit
//                   atomics; launched until a launch changes nothing (host checks a counter
//                   every few launches: the one synchronisation of the call)
//   k_epic_graph    adjacent-cell pairs inserted into fixed-size per-seed adjacency rows
//   k_epic_knn_fit  one wavefront per seed: Dijkstra on the seed graph with the frontier and a
//                   hash index in LDS, stopped after k settles; FP64 weighted affine fit by
//                   modified Gram-Schmidt across the wavefront
//   k_epic_dense    every pixel evaluates its cell's model, HBM bound
// Keys pack (distance << 32 | seed index), so one unsigned 64-bit minimum orders by distance and
// breaks ties by the lower index; all distances are exact integers.
#include <math.h>
#include <string.h>

#include "dgf_internal.hpp"

namespace dgf {
namespace {

constexpr int kMaxDeg = 32;          // graph neighbours a seed can hold
constexpr int kCand = 512;           // candidates one neighbour search can hold
constexpr int kHash = 1024;          // LDS hash slots of one search (power of two, > kCand + kMaxDeg)
constexpr int kMaxK = 256;           // largest k
constexpr int kTile = 32;            // relaxation tile side
constexpr int kTileThreads = 256;    // 8 rows of 32 lanes; each lane owns 4 pixels of its column
constexpr int kLocalIters = 4 * kTile;
constexpr int kChunk = 4;            // relaxation launches between two convergence checks
constexpr int kMaxRelaxLaunches = 1 << 14;
constexpr uint64_t kNoKey = ~0ull;
constexpr uint64_t kDistCap = 0xFFFFFFFEull;
constexpr int kMaxEdge = 510;        // largest edge-map value

enum : uint32_t { kErrDegree = 1u, kErrCand = 2u };

struct EpicWs {
    uint64_t *keys;  // [H*W]
    uint16_t *E;     // [H*W]
    int32_t *adj_id; // [n][kMaxDeg], -1 = empty
    uint32_t *adj_w; // [n][kMaxDeg]
    float *model;    // [n][8]: affine coefficients (6), seed position (2)
    uint32_t *ctr;   // [kChunk] tiles changed per relaxation launch, then [1] error bits
};

int64_t align256(int64_t v) { return (v + 255) / 256 * 256; }

int64_t ws_layout(int W, int H, int64_t n, EpicWs *ws, char *base)
{
    const int64_t N = (int64_t)W * H;
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
        const int64_t o = off;
        off += align256(bytes);
        return base ? base + o : nullptr;
    };
    char *keys = take(8 * N), *E = take(2 * N), *aid = take(4 * n * kMaxDeg), *aw = take(4 * n * kMaxDeg);
    char *model = take(32 * n), *ctr = take(4 * (kChunk + 1));
    if (ws) {
        ws->keys = (uint64_t *)keys;
        ws->E = (uint16_t *)E;
        ws->adj_id = (int32_t *)aid;
        ws->adj_w = (uint32_t *)aw;
        ws->model = (float *)model;
        ws->ctr = (uint32_t *)ctr;
    }
    return off;
}

__device__ __forceinline__ uint64_t load_key(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Edge map and cleared key / adjacency tables / counters.
__global__ void k_epic_prep(const uint8_t *I, int64_t pitch, int W, int H, int64_t n, EpicWs ws)
{
    const uint32_t N = (uint32_t)W * (uint32_t)H;
    const int64_t S = n * kMaxDeg;
    const int64_t tot = S > (int64_t)N ? S : (int64_t)N;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
        if (i < (int64_t)N) {
            const uint32_t q = (uint32_t)i, y = q / (uint32_t)W, x = q - y * (uint32_t)W;
            const int xl = x > 0 ? (int)x - 1 : 0, xr = (int)x + 1 < W ? (int)x + 1 : W - 1;
            const int yu = y > 0 ? (int)y - 1 : 0, yd = (int)y + 1 < H ? (int)y + 1 : H - 1;
            const uint8_t *row = I + (int64_t)y * pitch;
            const int gx = (int)row[xr] - (int)row[xl];
            const int gy = (int)I[(int64_t)yd * pitch + x] - (int)I[(int64_t)yu * pitch + x];
            ws.E[i] = (uint16_t)(abs(gx) + abs(gy));
            ws.keys[i] = kNoKey;
        }
        if (i < S) {
            ws.adj_id[i] = -1;
            ws.adj_w[i] = 0xFFFFFFFFu;
        }
        if (i < kChunk + 1) ws.ctr[i] = 0u;
    }
}

// Seed pixel of a point, (floor(x + 1/2), floor(y + 1/2)) clamped into the image; false for a
// point that takes no part (not converged, or a non-finite position or flow).
__device__ __forceinline__ bool seed_pixel(const float *pts, const float *flow, const uint8_t *status, int64_t i,
                                           int W, int H, uint32_t &q)
{
    if (status[i] != DGF_ST_CONVERGED) return false;
    const float x = pts[2 * i], y = pts[2 * i + 1];
    if (!isfinite(x) || !isfinite(y) || !isfinite(flow[2 * i]) || !isfinite(flow[2 * i + 1])) return false;
    const int px = (int)fminf(fmaxf(floorf(x + 0.5f), 0.f), (float)(W - 1));
    const int py = (int)fminf(fmaxf(floorf(y + 0.5f), 0.f), (float)(H - 1));
    q = (uint32_t)py * (uint32_t)W + (uint32_t)px;
    return true;
}

__global__ void k_epic_seed(const float *pts, const float *flow, const uint8_t *status, int64_t n, int W, int H,
                            uint64_t *keys)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t q;
    if (seed_pixel(pts, flow, status, i, W, H, q)) atomicMin((unsigned long long *)(keys + q), (unsigned long long)i);
}

// One relaxation round: each 32x32 tile (plus a one-pixel halo read from the current global
// state) iterates key(p) = min(key(p), min over 4-neighbours q of key(q) + step(q, p)) in LDS until
// nothing changes (or kLocalIters rounds), then writes its improved pixels back.  Keys only ever
// decrease and always belong to a real path, so any interleaving of tiles converges to the exact
// least keys; a launch in which no tile changes anything is at that fixed point.
__global__ __launch_bounds__(kTileThreads) void k_epic_relax(int W, int H, int kappa, uint64_t *keys,
                                                             const uint16_t *E, uint32_t *changed)
{
    constexpr int T2 = kTile + 2;
    __shared__ uint64_t K[T2 * T2];
    __shared__ uint16_t Es[T2 * T2];
    const int x0 = (int)blockIdx.x * kTile - 1, y0 = (int)blockIdx.y * kTile - 1;
    for (int c = threadIdx.x; c < T2 * T2; c += kTileThreads) {
        const int ly = c / T2, lx = c - ly * T2;
        const int gx = x0 + lx, gy = y0 + ly;
        uint64_t k = kNoKey;
        uint16_t e = 0;
        if (gx >= 0 && gy >= 0 && gx < W && gy < H) {
            const uint32_t q = (uint32_t)gy * (uint32_t)W + (uint32_t)gx;
            k = load_key(keys + q);
            e = E[q];
        }
        K[c] = k;
        Es[c] = e;
    }
    __syncthreads();
    const int tx = threadIdx.x % kTile, ty = threadIdx.x / kTile;
    int cell[4];
    bool inside[4];
    uint64_t orig[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int lx = tx + 1, ly = ty + 8 * j + 1;
        cell[j] = ly * T2 + lx;
        inside[j] = x0 + lx < W && y0 + ly < H;
        orig[j] = K[cell[j]];
    }
    for (int it = 0; it < kLocalIters; ++it) {
        uint64_t nv[4];
        bool imp = false;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int c = cell[j];
            const uint64_t cur = K[c];
            uint64_t best = cur;
            if (inside[j]) {
                const uint32_t ec = (uint32_t)kappa + Es[c];
                const int nbc[4] = {c - 1, c + 1, c - T2, c + T2};
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    const uint64_t kn = K[nbc[d]];
                    if (kn == kNoKey) continue;
                    uint64_t dist = (kn >> 32) + ec + Es[nbc[d]];
                    dist = dist < kDistCap ? dist : kDistCap;
                    const uint64_t cand = (dist << 32) | (kn & 0xFFFFFFFFull);
                    best = cand < best ? cand : best;
                }
            }
            nv[j] = best;
            imp |= best < cur;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 4; ++j) K[cell[j]] = nv[j];
        if (!__syncthreads_or(imp)) break;
    }
    bool wrote = false;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint64_t k = K[cell[j]];
        if (inside[j] && k < orig[j]) {
            const uint32_t q = (uint32_t)(y0 + ty + 8 * j + 1) * (uint32_t)W + (uint32_t)(x0 + tx + 1);
            atomicMin((unsigned long long *)(keys + q), (unsigned long long)k);
            wrote = true;
        }
    }
    if (__syncthreads_or(wrote) && threadIdx.x == 0) atomicAdd(changed, 1u);
}

__global__ void k_epic_clear(uint32_t *c, int m)
{
    if ((int)threadIdx.x < m) c[threadIdx.x] = 0u;
}

// Insert (or lower) the edge s -> t of length w into s's adjacency row.
__device__ void adj_insert(const EpicWs &ws, uint32_t s, int32_t t, uint32_t w, uint32_t *err)
{
    int32_t *ids = ws.adj_id + (int64_t)s * kMaxDeg;
    for (int j = 0; j < kMaxDeg; ++j) {
        int32_t v = __hip_atomic_load(ids + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (v == -1) {
            const int32_t old = atomicCAS(ids + j, -1, t);
            v = old == -1 ? t : old;
        }
        if (v == t) {
            atomicMin(ws.adj_w + (int64_t)s * kMaxDeg + j, w);
            return;
        }
    }
    atomicOr(err, kErrDegree);
}

// Seed graph: every right / down pixel pair whose cells differ gives both cells an edge of
// length D(p) + step(p, q) + D(q); each row keeps the least length per neighbour.
__global__ void k_epic_graph(int W, int H, int kappa, const uint64_t *keys, const uint16_t *E, EpicWs ws,
                             uint32_t *err)
{
    const uint32_t N = (uint32_t)W * (uint32_t)H;
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < N; p += gridDim.x * blockDim.x) {
        const uint32_t y = p / (uint32_t)W, x = p - y * (uint32_t)W;
        const uint64_t kp = keys[p];
        const uint32_t nbq[2] = {x + 1 < (uint32_t)W ? p + 1 : N, y + 1 < (uint32_t)H ? p + (uint32_t)W : N};
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            const uint32_t q = nbq[d];
            if (q >= N) continue;
            const uint64_t kq = keys[q];
            const uint32_t ls = (uint32_t)kp, lt = (uint32_t)kq;
            if (ls == lt) continue;
            const uint64_t w64 = (kp >> 32) + (uint64_t)kappa + E[p] + E[q] + (kq >> 32);
            const uint32_t w = w64 < 0xFFFFFFFFull ? (uint32_t)w64 : 0xFFFFFFFFu;
            adj_insert(ws, ls, (int32_t)lt, w, err);
            adj_insert(ws, lt, (int32_t)ls, w, err);
        }
    }
}

struct EpicFit {
    const float *pts, *flow;
    const uint8_t *status;
    const uint64_t *keys;
    EpicWs ws;
    int64_t n;
    int W, H, k, h;
    uint32_t dmax;
    int32_t *nbr;
    uint32_t *nbr_dist;
    float *model_out;
    uint32_t *err;
};

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint64_t w = __shfl_xor(v, o, 64);
        v = w < v ? w : v;
    }
    return v;
}

__device__ __forceinline__ double wave_sum_f64(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ int hash_slot(int32_t t) { return (int)(((uint32_t)t * 2654435761u) >> 22); }

// One wavefront per seed s: its k nearest seeds on the seed graph in increasing (distance, index)
// order (Dijkstra from s, at graph distance <= 64 h, stopped after k settles), then the
// weighted least-squares affine model of the flow around s, in FP64.
__global__ __launch_bounds__(64) void k_epic_knn_fit(EpicFit F)
{
    static_assert(kHash == 1 << 10, "hash_slot returns 10 bits");
    __shared__ int32_t hkey[kHash];
    __shared__ int16_t hval[kHash];
    __shared__ int32_t cid[kCand];
    __shared__ uint32_t cdist[kCand];
    __shared__ uint8_t cdone[kCand];
    __shared__ int32_t sid[kMaxK];
    __shared__ uint32_t sdist[kMaxK];
    const int li = threadIdx.x;
    const int64_t s = blockIdx.x;
    if (s >= F.n) return; // whole wave

    uint32_t q = 0;
    bool alive = seed_pixel(F.pts, F.flow, F.status, s, F.W, F.H, q);
    if (alive) alive = F.keys[q] == (uint64_t)s; // s owns its pixel at distance 0
    int cnt = 0;
    bool overflow = false;
    if (alive) {
        for (int j = li; j < kHash; j += 64) hkey[j] = -1;
        __syncthreads();
        if (li == 0) {
            hkey[hash_slot((int32_t)s)] = (int32_t)s;
            hval[hash_slot((int32_t)s)] = 0;
            cid[0] = (int32_t)s;
            cdist[0] = 0u;
            cdone[0] = 0;
        }
        int m = 1;
        __syncthreads();
        while (cnt < F.k) {
            uint64_t best = kNoKey;
            int bslot = -1;
            for (int j = li; j < m; j += 64) {
                if (cdone[j]) continue;
                const uint64_t key = ((uint64_t)cdist[j] << 32) | (uint32_t)cid[j];
                if (key < best) {
                    best = key;
                    bslot = j;
                }
            }
            const uint64_t wbest = wave_min_u64(best);
            if (wbest == kNoKey) break;
            if (bslot >= 0 && best == wbest) cdone[bslot] = 1;
            const int32_t v = (int32_t)(uint32_t)wbest;
            const uint32_t dv = (uint32_t)(wbest >> 32);
            if (li == 0) {
                sid[cnt] = v;
                sdist[cnt] = dv;
            }
            ++cnt;
            // relax v's edges, one lane per adjacency slot
            int32_t t = -1;
            uint32_t c = 0;
            int hpos = -1;
            bool is_new = false;
            if (li < kMaxDeg) {
                t = F.ws.adj_id[(int64_t)v * kMaxDeg + li];
                if (t >= 0) {
                    const uint64_t c64 = (uint64_t)dv + F.ws.adj_w[(int64_t)v * kMaxDeg + li];
                    if (c64 <= F.dmax) {
                        c = (uint32_t)c64;
                        int hs = hash_slot(t);
                        for (int probe = 0; probe < kHash; ++probe) {
                            const int32_t old = atomicCAS(&hkey[hs], -1, t);
                            if (old == -1 || old == t) {
                                hpos = hs;
                                is_new = old == -1;
                                break;
                            }
                            hs = (hs + 1) & (kHash - 1);
                        }
                    } else {
                        t = -1;
                    }
                }
            }
            __syncthreads();
            const uint64_t nb = __ballot(is_new);
            const int total = __popcll(nb);
            if (m + total > kCand) {
                overflow = true;
                break;
            }
            if (is_new) {
                const int slot = m + __popcll(nb & ((1ull << li) - 1ull));
                hval[hpos] = (int16_t)slot;
                cid[slot] = t;
                cdist[slot] = c;
                cdone[slot] = 0;
            } else if (hpos >= 0) {
                const int slot = hval[hpos];
                if (!cdone[slot] && c < cdist[slot]) cdist[slot] = c;
            }
            m += total;
            __syncthreads();
        }
        __syncthreads();
    }
    if (overflow && li == 0) atomicOr(F.err, kErrCand);
    if (!alive || overflow) cnt = 0;
    if (F.nbr)
        for (int j = li; j < F.k; j += 64) {
            F.nbr[s * F.k + j] = j < cnt ? sid[j] : -1;
            F.nbr_dist[s * F.k + j] = j < cnt ? sdist[j] : 0xFFFFFFFFu;
        }
    float *mo = F.ws.model + 8 * s;
    if (!alive || overflow) {
        if (li < 6) {
            mo[li] = __builtin_nanf("");
            if (F.model_out) F.model_out[6 * s + li] = __builtin_nanf("");
        }
        return;
    }
    // weighted position moments about the seed's own position (for the degeneracy test)
    constexpr int RPL = kMaxK / 64; // rows per lane
    const double sx = F.pts[2 * s], sy = F.pts[2 * s + 1];
    double c1[RPL], cx[RPL], cy[RPL], bu[RPL], bv[RPL]; // sqrt(w) (1, x, y | u, v)
    double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};              // w, x, y, xx, xy, yy, u, v
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int j = li + 64 * r;
        c1[r] = cx[r] = cy[r] = bu[r] = bv[r] = 0.0;
        if (j < cnt) {
            const int32_t t = sid[j];
            const double w = exp2(-(double)sdist[j] / (double)F.h);
            const double x = (double)F.pts[2 * t] - sx, y = (double)F.pts[2 * t + 1] - sy;
            const double u = F.flow[2 * t], v = F.flow[2 * t + 1];
            a[0] += w;
            a[1] += w * x;
            a[2] += w * y;
            a[3] += w * x * x;
            a[4] += w * x * y;
            a[5] += w * y * y;
            a[6] += w * u;
            a[7] += w * v;
            const double rw = sqrt(w);
            c1[r] = rw;
            cx[r] = rw * x;
            cy[r] = rw * y;
            bu[r] = rw * u;
            bv[r] = rw * v;
        }
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) a[e] = wave_sum_f64(a[e]);
    double mdl[6];
    const double sw = a[0], ex = a[1] / sw, ey = a[2] / sw;
    const double cxx = a[3] / sw - ex * ex, cyy = a[5] / sw - ey * ey, cxy = a[4] / sw - ex * ey;
    const double tr = cxx + cyy, det = cxx * cyy - cxy * cxy;
    if (cnt < 3 || !(det > 1e-4 * tr * tr)) {
        mdl[0] = mdl[1] = mdl[3] = mdl[4] = 0.0;
        mdl[2] = a[6] / sw;
        mdl[5] = a[7] / sw;
    } else {
        // weighted least squares by modified Gram-Schmidt on the columns sqrt(w) (1, x, y), the
        // right-hand sides carried along as further columns (backward stable for least squares;
        // the weights can span 64 binades, beyond what the normal equations resolve)
        auto dot = [&](const double *p, const double *q) {
            double acc = 0.0;
#pragma unroll
            for (int r = 0; r < RPL; ++r) acc += p[r] * q[r];
            return wave_sum_f64(acc);
        };
        auto axpy = [&](double f, const double *q, double *p) {
#pragma unroll
            for (int r = 0; r < RPL; ++r) p[r] -= f * q[r];
        };
        auto scale = [&](double f, double *p) {
#pragma unroll
            for (int r = 0; r < RPL; ++r) p[r] *= f;
        };
        const double r11 = sqrt(dot(c1, c1));
        scale(1.0 / r11, c1);
        const double r12 = dot(c1, cx), r13 = dot(c1, cy), z1u = dot(c1, bu), z1v = dot(c1, bv);
        axpy(r12, c1, cx);
        axpy(r13, c1, cy);
        axpy(z1u, c1, bu);
        axpy(z1v, c1, bv);
        const double r22 = sqrt(dot(cx, cx));
        scale(1.0 / r22, cx);
        const double r23 = dot(cx, cy), z2u = dot(cx, bu), z2v = dot(cx, bv);
        axpy(r23, cx, cy);
        axpy(z2u, cx, bu);
        axpy(z2v, cx, bv);
        const double r33 = sqrt(dot(cy, cy));
        scale(1.0 / r33, cy);
        const double z3u = dot(cy, bu), z3v = dot(cy, bv);
        // R (offset, d/dx, d/dy)^T = z
        const double gyu = z3u / r33, gyv = z3v / r33;
        const double gxu = (z2u - r23 * gyu) / r22, gxv = (z2v - r23 * gyv) / r22;
        mdl[0] = gxu;
        mdl[1] = gyu;
        mdl[2] = (z1u - r12 * gxu - r13 * gyu) / r11;
        mdl[3] = gxv;
        mdl[4] = gyv;
        mdl[5] = (z1v - r12 * gxv - r13 * gyv) / r11;
    }
    if (li != 0) return;
    for (int e = 0; e < 6; ++e) {
        mo[e] = (float)mdl[e];
        if (F.model_out) F.model_out[6 * s + e] = (float)mdl[e];
    }
    mo[6] = (float)sx;
    mo[7] = (float)sy;
}

// Every pixel evaluates the model of its cell's seed at its own coordinates.
__global__ void k_epic_dense(int W, int H, const uint64_t *keys, const float *model, float *dense, int64_t dpitch,
                             int32_t *labels, uint32_t *dist)
{
    const uint32_t N = (uint32_t)W * (uint32_t)H;
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < N; p += gridDim.x * blockDim.x) {
        const uint32_t y = p / (uint32_t)W, x = p - y * (uint32_t)W;
        const uint64_t k = keys[p];
        float2 f;
        if (k == kNoKey) {
            f = make_float2(__builtin_nanf(""), __builtin_nanf(""));
        } else {
            const float4 *m = reinterpret_cast<const float4 *>(model + 8 * (int64_t)(uint32_t)k);
            const float4 m0 = m[0], m1 = m[1];
            const float rx = (float)x - m1.z, ry = (float)y - m1.w;
            f = make_float2(fmaf(m0.x, rx, fmaf(m0.y, ry, m0.z)), fmaf(m0.w, rx, fmaf(m1.x, ry, m1.y)));
        }
        *reinterpret_cast<float2 *>(dense + (int64_t)y * dpitch + 2 * x) = f;
        if (labels) labels[p] = k == kNoKey ? -1 : (int32_t)(uint32_t)k;
        if (dist) dist[p] = k == kNoKey ? 0xFFFFFFFFu : (uint32_t)(k >> 32);
    }
}

unsigned grid_for(int64_t items, int threads)
{
    const int64_t b = (items + threads - 1) / threads;
    return (unsigned)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

bool epic_image_ok(const dgf_image *im)
{
    if (!im || !im->data || im->dtype != DGF_U8 || im->width < 1 || im->height < 1) return false;
    if (im->pitch_bytes < im->width) return false;
    if ((int64_t)im->width * im->height > (int64_t)INT32_MAX) return false;
    return true;
}

} // namespace
} // namespace dgf

using namespace dgf;

extern "C" {

int dgf_epic_opts_default(dgf_epic_opts *o)
{
    if (!o) return DGF_ERR_INVALID_ARG;
    o->k = 128;
    o->kappa = 8;
    o->half_dist = 64;
    return DGF_OK;
}

size_t dgf_epic_workspace_bytes(int32_t width, int32_t height, int64_t n)
{
    if (width < 1 || height < 1 || n < 0) return 0;
    return (size_t)ws_layout(width, height, n, nullptr, nullptr);
}

int dgf_epic(const dgf_image *I0, const float *points, const float *flow, const uint8_t *status, int64_t n,
             const dgf_epic_opts *opts, void *workspace, size_t ws_bytes, float *dense, int64_t dense_pitch,
             int32_t *labels, uint32_t *dist, int32_t *nbr, uint32_t *nbr_dist, float *model, void *stream)
{
    if (!epic_image_ok(I0)) return DGF_ERR_INVALID_ARG;
    const int W = I0->width, H = I0->height;
    dgf_epic_opts o;
    if (opts)
        o = *opts;
    else
        dgf_epic_opts_default(&o);
    if (o.k < 1 || o.k > kMaxK || o.kappa < 1 || o.kappa > (1 << 20) || o.half_dist < 1 || o.half_dist > (1 << 24))
        return DGF_ERR_INVALID_ARG;
    // every least distance is at most that of a straight row-then-column path
    if ((uint64_t)(W - 1 + H - 1) * (uint64_t)(o.kappa + 2 * kMaxEdge) > kDistCap) return DGF_ERR_UNSUPPORTED;
    if (n < 0 || n >= (int64_t)INT32_MAX) return DGF_ERR_INVALID_ARG;
    if (n > 0 && (!points || !flow || !status)) return DGF_ERR_INVALID_ARG;
    if (!dense || dense_pitch < 2 * (int64_t)W || dense_pitch % 2 != 0 || (uintptr_t)dense % 8 != 0)
        return DGF_ERR_INVALID_ARG;
    if ((nbr == nullptr) != (nbr_dist == nullptr)) return DGF_ERR_INVALID_ARG;
    const size_t need = (size_t)ws_layout(W, H, n, nullptr, nullptr);
    if (!workspace || ws_bytes < need) return DGF_ERR_WORKSPACE;
    EpicWs ws;
    ws_layout(W, H, n, &ws, (char *)workspace);
    hipStream_t st = (hipStream_t)stream;
    const int64_t N = (int64_t)W * H;

    const int64_t prep_items = N > n * kMaxDeg ? N : n * kMaxDeg;
    hipLaunchKernelGGL(k_epic_prep, dim3(grid_for(prep_items, 256)), dim3(256), 0, st, (const uint8_t *)I0->data,
                       I0->pitch_bytes, W, H, n, ws);
    if (hipGetLastError() != hipSuccess) return DGF_ERR_HIP;
    uint32_t *err = ws.ctr + kChunk;
    if (n > 0) {
        hipLaunchKernelGGL(k_epic_seed, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, points, flow, status, n, W,
                           H, ws.keys);
        if (hipGetLastError() != hipSuccess) return DGF_ERR_HIP;
        const dim3 tiles((unsigned)((W + kTile - 1) / kTile), (unsigned)((H + kTile - 1) / kTile));
        bool converged = false;
        for (int base = 0; base < kMaxRelaxLaunches && !converged; base += kChunk) {
            hipLaunchKernelGGL(k_epic_clear, dim3(1), dim3(64), 0, st, ws.ctr, kChunk);
            for (int j = 0; j < kChunk; ++j)
                hipLaunchKernelGGL(k_epic_relax, tiles, dim3(kTileThreads), 0, st, W, H, o.kappa, ws.keys,
                                   (const uint16_t *)ws.E, ws.ctr + j);
            if (hipGetLastError() != hipSuccess) return DGF_ERR_HIP;
            uint32_t h_changed[kChunk];
            if (hipMemcpyAsync(h_changed, ws.ctr, sizeof(h_changed), hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                return DGF_ERR_HIP;
            converged = h_changed[kChunk - 1] == 0u;
        }
        if (!converged) return DGF_ERR_UNSUPPORTED;
        hipLaunchKernelGGL(k_epic_graph, dim3(grid_for(N, 256)), dim3(256), 0, st, W, H, o.kappa,
                           (const uint64_t *)ws.keys, (const uint16_t *)ws.E, ws, err);
        if (hipGetLastError() != hipSuccess) return DGF_ERR_HIP;
        EpicFit F{};
        F.pts = points;
        F.flow = flow;
        F.status = status;
        F.keys = ws.keys;
        F.ws = ws;
        F.n = n;
        F.W = W;
        F.H = H;
        F.k = o.k;
        F.h = o.half_dist;
        F.dmax = (uint32_t)(64u * (uint32_t)o.half_dist);
        F.nbr = nbr;
        F.nbr_dist = nbr_dist;
        F.model_out = model;
        F.err = err;
        hipLaunchKernelGGL(k_epic_knn_fit, dim3((unsigned)n), dim3(64), 0, st, F);
        if (hipGetLastError() != hipSuccess) return DGF_ERR_HIP;
    }
    hipLaunchKernelGGL(k_epic_dense, dim3(grid_for(N, 256)), dim3(256), 0, st, W, H, (const uint64_t *)ws.keys,
                       (const float *)ws.model, dense, dense_pitch, labels, dist);
    if (hipGetLastError() != hipSuccess) return DGF_ERR_HIP;
    uint32_t h_err = 0;
    if (hipMemcpyAsync(&h_err, err, sizeof(h_err), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return DGF_ERR_HIP;
    return h_err ? DGF_ERR_CAPACITY : DGF_OK;
}

} // extern "C"
