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
//   k_epic_relax    32x64 tiles relaxed in LDS (Bellman-Ford sweeps over the tile, double
//                   buffered), exchanging border pixels with their neighbours through 64-bit
//                   atomics during the launch; launched until a launch changes nothing (host
//                   checks a counter every few launches: the one synchronisation of the call)
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
constexpr int kCand = 384;           // candidates one neighbour search can hold (about 210 needed at k 128)
constexpr int kHash = 512;           // LDS hash slots of one search (power of two, > kCand + kMaxDeg)
constexpr int kMaxK = 256;           // largest k
// relaxation tile: 32 x 64 crossed fewer tile borders than 32 x 32 on the benchmark frames
// (0.755 against 0.792 ms per 1242x375 frame); 64 x 64 tiles put 16 wavefronts behind each
// barrier and were slower (0.816 ms)
constexpr int kRTX = 32;             // relaxation tile width
constexpr int kRTY = 64;             // relaxation tile height
constexpr int kRTX2 = kRTX + 2;      // with the halo
constexpr int kRTY2 = kRTY + 2;
constexpr int kRelaxThreads = kRTX * kRTY / 4; // each lane owns 4 pixels of one column
static_assert(kRelaxThreads % 64 == 0 && kRelaxThreads <= 1024 && kRTY % (kRelaxThreads / kRTX) == 0, "tile shape");
constexpr int kExchange = 32;        // relaxation iterations between two halo exchanges
constexpr int kMaxIters = 8192;      // relaxation iterations per tile and launch
constexpr int kMaxPolls = 4096;      // halo polls of a still tile per launch
constexpr int kChunk = 4;            // relaxation launches between two convergence checks
constexpr int kMaxRelaxLaunches = 1 << 14;
constexpr int kDefaultAsyncRelax = 32; // dgf_epic_async's relaxation launches when given 0
constexpr uint64_t kNoKey = ~0ull;
constexpr uint64_t kDistCap = 0xFFFFFFFEull;
constexpr int kMaxEdge = 510;        // largest edge-map value

enum : uint32_t { kErrDegree = 1u, kErrCand = 2u };

struct EpicWs {
    uint64_t *keys;  // [H*W]
    uint16_t *E;     // [H*W]
    uint64_t *adj;   // [n][kMaxDeg]: (edge length << 32) | neighbour, kNoKey = empty slot
    float *model;    // [n][8]: affine coefficients (6), seed position (2)
    uint32_t *ctr;   // [kChunk] tiles changed per relaxation launch, [1] error bits, [1] least edge,
                     // [kChunk] busy count per relaxation launch, [1] the changed count of the
                     // launch before the current group of kChunk
    uint32_t *mail;  // [kChunk][tiles]: a neighbour published keys into this tile's halo
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
    char *keys = take(8 * N), *E = take(2 * N), *adj = take(8 * n * kMaxDeg);
    const int64_t tiles = (int64_t)((W + kRTX - 1) / kRTX) * ((H + kRTY - 1) / kRTY);
    char *model = take(32 * n), *ctr = take(4 * (2 * kChunk + 3)), *mail = take(4 * kChunk * tiles);
    if (ws) {
        ws->keys = (uint64_t *)keys;
        ws->E = (uint16_t *)E;
        ws->adj = (uint64_t *)adj;
        ws->model = (float *)model;
        ws->ctr = (uint32_t *)ctr;
        ws->mail = (uint32_t *)mail;
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
        if (i < S) ws.adj[i] = kNoKey;
        if (i < kChunk + 2) ws.ctr[i] = i == kChunk + 1 ? 0xFFFFFFFFu : 0u;
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

// Key of the path that reaches a pixel from a neighbour holding key kn with a step of cost c:
// the distance half saturates at all ones, so kNoKey stays kNoKey; a saturated distance is
// never a least one (every least distance is below kDistCap) and is replaced in time.
__device__ __forceinline__ uint64_t step_key(uint64_t kn, uint32_t c)
{
    const uint32_t hi = (uint32_t)(kn >> 32);
    uint32_t d = hi + c;
    d = d < hi ? 0xFFFFFFFFu : d;
    return ((uint64_t)d << 32) | (kn & 0xFFFFFFFFull);
}

// One relaxation launch over 32x64 tiles.  Each tile holds its pixels and a one-pixel halo in
// LDS (two buffers) and iterates key(p) = min(key(p), min over 4-neighbours q of key(q) +
// step(q, p)) -- one barrier per iteration, each lane owning 4 pixels whose step costs stay in
// registers.  Every kExchange iterations, and whenever it has stopped changing, a tile publishes
// its newly improved border pixels with 64-bit atomicMin and posts mail to each neighbour tile
// whose halo they touch; a tile with mail re-reads its halo.  Termination: `busy` counts the
// tiles that are working plus the mail not yet taken (a publisher adds one for each mailbox it
// fills, before it can itself go still), so it reaches zero only when no tile can change
// anything.  A still tile (with `wait`: the whole grid resident at once) polls its mailbox and
// the count, resuming on mail and leaving at zero; polls are bounded (kMaxPolls) so every tile
// exits.  Keys only decrease and always belong to a real path, so any interleaving converges to
// the exact least keys, and a launch in which no tile changes anything is at that fixed point.
// prev (nullable): the changed count of the launch before; when it is zero the distances are
// already at the fixed point and the launch returns at once (so a fixed number of launches can be
// enqueued without reading anything back).
__global__ __launch_bounds__(kRelaxThreads) void k_epic_relax(int W, int H, int kappa, uint64_t *keys,
                                                              const uint16_t *E, uint32_t *changed, uint32_t *busy,
                                                              uint32_t *mail, int wait, const uint32_t *prev)
{
    if (prev && *prev == 0u) return; // the same value in every block (an earlier kernel wrote it)
    __shared__ uint64_t K[2][kRTX2 * kRTY2];
    __shared__ uint16_t Es[kRTX2 * kRTY2];
    __shared__ uint32_t flags[2][kRelaxThreads / 64];
    __shared__ uint32_t sides, got_mail, count_zero;
    const int x0 = (int)blockIdx.x * kRTX - 1, y0 = (int)blockIdx.y * kRTY - 1;
    const int me = (int)(blockIdx.y * gridDim.x + blockIdx.x);
    const int nbr_tile[4] = {blockIdx.x > 0 ? me - 1 : -1, blockIdx.x + 1 < gridDim.x ? me + 1 : -1,
                             blockIdx.y > 0 ? me - (int)gridDim.x : -1,
                             blockIdx.y + 1 < gridDim.y ? me + (int)gridDim.x : -1};
    // the halo ring: 2 (kRTX + 2) + 2 kRTY cells (top row, bottom row, left column, right column)
    auto ring_cell = [&](int i) {
        if (i < kRTX2) return i;
        if (i < 2 * kRTX2) return (kRTY + 1) * kRTX2 + (i - kRTX2);
        i -= 2 * kRTX2;
        return i < kRTY ? (i + 1) * kRTX2 : (i - kRTY + 1) * kRTX2 + kRTX + 1;
    };
    auto global_of = [&](int c, uint32_t &q) {
        const int ly = c / kRTX2, lx = c - ly * kRTX2;
        const int gx = x0 + lx, gy = y0 + ly;
        q = (uint32_t)gy * (uint32_t)W + (uint32_t)gx;
        return gx >= 0 && gy >= 0 && gx < W && gy < H;
    };
    for (int c = threadIdx.x; c < kRTX2 * kRTY2; c += kRelaxThreads) {
        uint32_t q;
        uint64_t k = kNoKey;
        uint16_t e = 0;
        if (global_of(c, q)) {
            k = load_key(keys + q);
            e = E[q];
        }
        K[0][c] = k;
        K[1][c] = k;
        Es[c] = e;
    }
    if (threadIdx.x == 0) sides = 0u;
    __syncthreads();
    const int tx = threadIdx.x % kRTX, ty = threadIdx.x / kRTX;
    constexpr int kPix = kRTX * kRTY / kRelaxThreads;
    constexpr int kRowStep = kRelaxThreads / kRTX; // rows between a lane's pixels
    int cell[kPix];
    bool inside[kPix];
    uint64_t own[kPix], orig[kPix], pub[kPix];
    uint32_t cst[kPix][4]; // step costs from the left, right, upper and lower neighbour
    uint32_t side_of[kPix]; // which neighbour tiles' halos this pixel belongs to (bit per side)
#pragma unroll
    for (int j = 0; j < kPix; ++j) {
        const int lx = tx + 1, ly = ty + kRowStep * j + 1;
        const int c = ly * kRTX2 + lx;
        cell[j] = c;
        inside[j] = x0 + lx < W && y0 + ly < H;
        own[j] = orig[j] = pub[j] = K[0][c];
        const uint32_t e = (uint32_t)kappa + Es[c];
        cst[j][0] = e + Es[c - 1];
        cst[j][1] = e + Es[c + 1];
        cst[j][2] = e + Es[c - kRTX2];
        cst[j][3] = e + Es[c + kRTX2];
        side_of[j] = (lx == 1 ? 1u : 0u) | (lx == kRTX ? 2u : 0u) | (ly == 1 ? 4u : 0u) | (ly == kRTY ? 8u : 0u);
    }
    // re-read the halo ring into both buffers
    auto reload_halo = [&](int cur) {
        for (int i = threadIdx.x; i < 2 * kRTX2 + 2 * kRTY; i += kRelaxThreads) {
            const int c = ring_cell(i);
            uint32_t q;
            if (!global_of(c, q)) continue;
            const uint64_t k = load_key(keys + q);
            if (k < K[cur][c]) {
                K[0][c] = k;
                K[1][c] = k;
            }
        }
        __syncthreads();
    };
    // publish newly improved border pixels and post mail to the tiles whose halos they touch
    auto publish = [&]() {
        uint32_t my_sides = 0u;
#pragma unroll
        for (int j = 0; j < kPix; ++j) {
            if (inside[j] && side_of[j] && own[j] < pub[j]) {
                const int ly = ty + kRowStep * j + 1;
                const uint32_t q = (uint32_t)(y0 + ly) * (uint32_t)W + (uint32_t)(x0 + tx + 1);
                atomicMin((unsigned long long *)(keys + q), (unsigned long long)own[j]);
                pub[j] = own[j];
                my_sides |= side_of[j];
            }
        }
        if (my_sides) atomicOr(&sides, my_sides);
        __builtin_amdgcn_s_waitcnt(0); // the key updates are performed before any mail is posted
        __syncthreads();
        if (threadIdx.x < 4 && ((sides >> threadIdx.x) & 1u) && nbr_tile[threadIdx.x] >= 0)
            if (atomicExch(mail + nbr_tile[threadIdx.x], 1u) == 0u) atomicAdd(busy, 1u);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x == 0) sides = 0u;
    };
    // take this tile's mail; a working tile already holds a busy count and returns the one the
    // mail carried, a still tile takes it over
    auto take_mail = [&](bool still_now) {
        if (threadIdx.x == 0) {
            uint32_t m = 0u;
            if (__hip_atomic_load(mail + me, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) m = atomicExch(mail + me, 0u);
            if (m && !still_now) atomicSub(busy, 1u);
            got_mail = m;
        }
        __syncthreads();
        return got_mail != 0u;
    };
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int cur = 0, polls = 0;
    bool still = false;
    for (int it = 0; it < kMaxIters; ++it) {
        // all sixteen neighbour keys first (independent LDS reads, one wait), then the minima
        const uint64_t *Kc = K[cur];
        uint64_t nk[kPix][4];
#pragma unroll
        for (int j = 0; j < kPix; ++j) {
            const int c = cell[j];
            nk[j][0] = Kc[c - 1];
            nk[j][1] = Kc[c + 1];
            nk[j][2] = Kc[c - kRTX2];
            nk[j][3] = Kc[c + kRTX2];
        }
        bool ch = false;
#pragma unroll
        for (int j = 0; j < kPix; ++j) {
            uint64_t best = own[j];
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                const uint64_t v = step_key(nk[j][d], cst[j][d]);
                best = v < best ? v : best;
            }
            best = inside[j] ? best : own[j];
            ch |= best < own[j];
            own[j] = best;
            K[cur ^ 1][cell[j]] = best;
        }
        // one barrier: each wavefront posts whether any of its lanes changed anything
        const uint64_t changed_lanes = __ballot(ch);
        if (lane == 0) flags[it & 1][wave] = changed_lanes != 0ull;
        __syncthreads();
        bool any = false;
#pragma unroll
        for (int w = 0; w < kRelaxThreads / 64; ++w) any |= flags[it & 1][w] != 0u;
        cur ^= 1;
        if (any && (it + 1) % kExchange != 0) continue;
        publish();
        if (take_mail(false)) {
            reload_halo(cur);
            continue;
        }
        if (any) continue;
        // still
        if (threadIdx.x == 0) atomicSub(busy, 1u);
        still = true;
        if (!wait) break;
        bool resume = false;
        while (polls < kMaxPolls) {
            ++polls;
            __builtin_amdgcn_s_sleep(2);
            if (threadIdx.x == 0)
                count_zero = __hip_atomic_load(busy, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u;
            __syncthreads();
            const bool zero = count_zero != 0u;
            if (take_mail(true)) {
                resume = true;
                break;
            }
            if (zero) break;
        }
        if (!resume) break;
        still = false;
        reload_halo(cur);
    }
    // leave: return the busy count of a working tile and of any mail not taken
    bool wrote = false;
#pragma unroll
    for (int j = 0; j < kPix; ++j) {
        if (inside[j] && own[j] < orig[j]) {
            const int ly = ty + kRowStep * j + 1;
            const uint32_t q = (uint32_t)(y0 + ly) * (uint32_t)W + (uint32_t)(x0 + tx + 1);
            atomicMin((unsigned long long *)(keys + q), (unsigned long long)own[j]);
            wrote = true;
        }
    }
    if (threadIdx.x == 0) {
        if (!still) atomicSub(busy, 1u);
        if (atomicExch(mail + me, 0u)) atomicSub(busy, 1u);
    }
    if (__syncthreads_or(wrote) && threadIdx.x == 0) atomicAdd(changed, 1u);
}

// (one block) Keeps the changed count of the previous group's last launch (prev_last >= 0) in
// carry, then clears the counters of the next m launches.
__global__ void k_epic_clear_launch_counters(uint32_t *changed, uint32_t *busy, uint32_t *mail, int m,
                                             uint32_t tiles, uint32_t *carry, int prev_last)
{
    if (prev_last >= 0 && threadIdx.x == 0) *carry = changed[prev_last];
    __syncthreads();
    if ((int)threadIdx.x < m) {
        changed[threadIdx.x] = 0u;
        busy[threadIdx.x] = tiles;
    }
    for (int64_t i = threadIdx.x; i < (int64_t)m * tiles; i += blockDim.x) mail[i] = 0u;
}

// Insert (or lower) the edge s -> t of length w into s's adjacency row: a slot holds
// (length << 32) | t, so once t owns a slot a 64-bit atomicMin keeps the least length.
__device__ void adj_insert(const EpicWs &ws, uint32_t s, uint32_t t, uint32_t w, uint32_t *err)
{
    unsigned long long *row = (unsigned long long *)(ws.adj + (int64_t)s * kMaxDeg);
    const unsigned long long val = ((unsigned long long)w << 32) | t;
    for (int j = 0; j < kMaxDeg; ++j) {
        unsigned long long cur = __hip_atomic_load(row + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cur == kNoKey) {
            cur = atomicCAS(row + j, (unsigned long long)kNoKey, val);
            if (cur == kNoKey) return;
        }
        if ((uint32_t)cur == t) {
            atomicMin(row + j, val);
            return;
        }
    }
    atomicOr(err, kErrDegree);
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t w = __shfl_xor(v, o, 64);
        v = w < v ? w : v;
    }
    return v;
}

// Seed graph: every right / down pixel pair whose cells differ gives both cells an edge of
// length D(p) + step(p, q) + D(q); each row keeps the least length per neighbour.  Neighbouring
// lanes hold neighbouring pixels of a row, so runs of lanes often carry the same cell pair (a
// horizontal cell border seen by the down pairs): the first lane of each run inserts the run's
// least length for all of it.  Also the least edge length of the whole graph (one atomic per
// wavefront).
__global__ void k_epic_graph(int W, int H, int kappa, const uint64_t *keys, const uint16_t *E, EpicWs ws,
                             uint32_t *err, uint32_t *min_edge, const uint32_t *unsettled)
{
    if (unsettled && *unsettled) return; // the partition did not reach its fixed point
    const uint32_t N = (uint32_t)W * (uint32_t)H;
    const int lane = threadIdx.x & 63;
    uint32_t wmin = 0xFFFFFFFFu;
    // (the loop runs a whole wavefront at a time: blockDim and the stride are multiples of 64)
    for (uint32_t base = blockIdx.x * blockDim.x + (threadIdx.x & ~63u); base < N; base += gridDim.x * blockDim.x) {
        const uint32_t p = base + lane;
        const bool in = p < N;
        const uint32_t y = in ? p / (uint32_t)W : 0u, x = in ? p - y * (uint32_t)W : 0u;
        const uint64_t kp = in ? keys[p] : kNoKey;
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            const bool has = in && (d == 0 ? x + 1 < (uint32_t)W : y + 1 < (uint32_t)H);
            const uint32_t q = d == 0 ? p + 1 : p + (uint32_t)W;
            const uint64_t kq = has ? keys[q] : kNoKey;
            const uint32_t ls = (uint32_t)kp, lt = (uint32_t)kq;
            const bool edge = has && ls != lt;
            uint32_t w = 0xFFFFFFFFu;
            if (edge) {
                const uint64_t w64 = (kp >> 32) + (uint64_t)kappa + E[p] + E[q] + (kq >> 32);
                w = w64 < 0xFFFFFFFFull ? (uint32_t)w64 : 0xFFFFFFFFu;
            }
            const uint64_t pair = edge ? ((uint64_t)ls << 32) | lt : kNoKey;
            // least length over this lane's run of equal pairs (lanes lane, lane + 1, ...)
            uint32_t wr = w;
            bool along = edge;
            for (int j = 1; j < 64; ++j) {
                const uint64_t pj = __shfl_down(pair, j, 64);
                const uint32_t wj = __shfl_down(w, j, 64);
                along = along && lane + j < 64 && pj == pair;
                if (along) wr = wj < wr ? wj : wr;
                if (!__ballot(along)) break;
            }
            const uint64_t prev = __shfl_up(pair, 1, 64);
            const bool head = edge && (lane == 0 || prev != pair);
            if (head) {
                wmin = wr < wmin ? wr : wmin;
                adj_insert(ws, ls, lt, wr, err);
                adj_insert(ws, lt, ls, wr, err);
            }
        }
    }
    wmin = wave_min_u32(wmin);
    if (lane == 0 && wmin != 0xFFFFFFFFu) atomicMin(min_edge, wmin);
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
    const uint32_t *min_edge;
    const uint32_t *unsettled; // nullable: nonzero when the partition did not reach its fixed point
};

__device__ __forceinline__ double wave_sum_f64(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ int hash_slot(int32_t t) { return (int)(((uint32_t)t * 2654435761u) >> 23); }

// One wavefront per seed s: its k nearest seeds on the seed graph in increasing (distance, index)
// order, at graph distance <= 64 h, then the weighted least-squares affine model of the flow
// around s, in FP64.  The search settles in batches (Dijkstra with buckets as wide as the least
// edge length D of the graph): with dmin the least tentative distance of the frontier, every
// frontier node below dmin + D is final, since any other path to it leaves the settled set
// through a frontier node and adds at least D.  After each batch the settled set is exactly the
// nodes below dmin + D, so once it holds k nodes its k smallest are the answer.  Candidates, a
// hash index from node to candidate slot and the settled candidates' slots (16-bit) live in LDS:
// 9.3 KB per search, so 17 searches share a CU.
__global__ __launch_bounds__(64) void k_epic_knn_fit(EpicFit F)
{
    if (F.unsettled && *F.unsettled) return; // the partition did not reach its fixed point
    static_assert(kHash == 1 << 9, "hash_slot returns 9 bits");
    constexpr int kStageNodes = 8; // batch nodes whose adjacency rows are read together
    static_assert(kStageNodes * kMaxDeg >= kMaxK, "the sorted output reuses the staging arrays");
    __shared__ int32_t hkey[kHash];
    __shared__ int16_t hval[kHash];
    __shared__ int32_t cid[kCand];
    __shared__ uint32_t cdist[kCand];
    __shared__ uint8_t cdone[kCand];
    __shared__ int16_t sslot[kCand]; // candidate slots of the settled nodes, in settling order
    __shared__ int32_t it_t[kStageNodes * kMaxDeg];
    __shared__ uint32_t it_c[kStageNodes * kMaxDeg];
    int32_t *oid = it_t; // the k nearest, sorted (after the search, over the staging arrays)
    uint32_t *od = it_c;
    const int li = threadIdx.x;
    const uint64_t below = (1ull << li) - 1ull;
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
        const uint64_t bucket = *F.min_edge; // >= kappa >= 1 (all ones when there is no edge)
        __syncthreads();
        for (;;) {
            uint32_t lmin = 0xFFFFFFFFu;
            for (int j = li; j < m; j += 64)
                if (!cdone[j]) lmin = cdist[j] < lmin ? cdist[j] : lmin;
            const uint32_t dmin = wave_min_u32(lmin);
            if (dmin == 0xFFFFFFFFu) break; // frontier empty
            const uint64_t T = (uint64_t)dmin + bucket;
            const int b0 = cnt;
            for (int base = 0; base < m; base += 64) {
                const int j = base + li;
                const bool sel = j < m && !cdone[j] && (uint64_t)cdist[j] < T;
                const uint64_t bm = __ballot(sel);
                if (sel) {
                    sslot[cnt + __popcll(bm & below)] = (int16_t)j;
                    cdone[j] = 1;
                }
                cnt += __popcll(bm);
            }
            __syncthreads();
            if (cnt >= F.k) break;
            // relax the batch's edges, kStageNodes adjacency rows at a time
            for (int nb0 = b0; nb0 < cnt && !overflow; nb0 += kStageNodes) {
                const int nn = cnt - nb0 < kStageNodes ? cnt - nb0 : kStageNodes;
                uint64_t e[kStageNodes * kMaxDeg / 64];
                uint32_t dv[kStageNodes * kMaxDeg / 64];
#pragma unroll
                for (int r = 0; r < kStageNodes * kMaxDeg / 64; ++r) {
                    const int idx = li + 64 * r, node = idx / kMaxDeg, slot = idx - node * kMaxDeg;
                    e[r] = kNoKey;
                    dv[r] = 0u;
                    if (node < nn) {
                        const int cs = sslot[nb0 + node];
                        e[r] = F.ws.adj[(int64_t)cid[cs] * kMaxDeg + slot];
                        dv[r] = cdist[cs];
                    }
                }
                int ni = 0;
#pragma unroll
                for (int r = 0; r < kStageNodes * kMaxDeg / 64; ++r) {
                    const uint64_t c64 = e[r] == kNoKey ? ~0ull : (uint64_t)dv[r] + (e[r] >> 32);
                    const bool ok = c64 <= F.dmax;
                    const uint64_t bm = __ballot(ok);
                    if (ok) {
                        const int at = ni + __popcll(bm & below);
                        it_t[at] = (int32_t)(uint32_t)e[r];
                        it_c[at] = (uint32_t)c64;
                    }
                    ni += __popcll(bm);
                }
                __syncthreads();
                for (int ib = 0; ib < ni; ib += 64) {
                    const int i = ib + li;
                    const bool has = i < ni;
                    int32_t t = -1;
                    uint32_t c = 0u;
                    int hpos = -1;
                    bool is_new = false;
                    if (has) {
                        t = it_t[i];
                        c = it_c[i];
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
                    }
                    __syncthreads();
                    const uint64_t nbm = __ballot(is_new);
                    const int total = __popcll(nbm);
                    if (m + total > kCand) {
                        overflow = true;
                        break;
                    }
                    if (is_new) {
                        const int slot = m + __popcll(nbm & below);
                        hval[hpos] = (int16_t)slot;
                        cid[slot] = t;
                        cdist[slot] = 0xFFFFFFFFu;
                        cdone[slot] = 0;
                    }
                    m += total;
                    __syncthreads();
                    if (hpos >= 0) {
                        const int slot = hval[hpos];
                        if (!cdone[slot]) atomicMin(&cdist[slot], c);
                    }
                    __syncthreads();
                }
            }
            if (overflow) break;
        }
        __syncthreads();
        if (!overflow) {
            // the k smallest settled (distance, index) pairs, by rank
            for (int j = li; j < cnt; j += 64) {
                const int cj = sslot[j];
                const uint64_t kj = ((uint64_t)cdist[cj] << 32) | (uint32_t)cid[cj];
                int rank = 0;
                for (int i = 0; i < cnt; ++i) {
                    const int ci = sslot[i];
                    rank += (((uint64_t)cdist[ci] << 32) | (uint32_t)cid[ci]) < kj;
                }
                if (rank < F.k) {
                    oid[rank] = cid[cj];
                    od[rank] = cdist[cj];
                }
            }
            cnt = cnt < F.k ? cnt : F.k;
        }
        __syncthreads();
    }
    if (overflow && li == 0) atomicOr(F.err, kErrCand);
    if (!alive || overflow) cnt = 0;
    if (F.nbr)
        for (int j = li; j < F.k; j += 64) {
            F.nbr[s * F.k + j] = j < cnt ? oid[j] : -1;
            F.nbr_dist[s * F.k + j] = j < cnt ? od[j] : 0xFFFFFFFFu;
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
            const int32_t t = oid[j];
            const double w = exp2(-(double)od[j] / (double)F.h);
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
                             int32_t *labels, uint32_t *dist, const uint32_t *unsettled)
{
    if (unsettled && *unsettled) return; // the partition did not reach its fixed point
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

namespace dgf {
namespace {
// (one thread) The outcome of a call without host synchronisation: 0 done, 1 the partition did
// not reach its fixed point within the launches given, 2 a capacity limit (see dgf_epic).
__global__ void k_epic_status(uint32_t *out, const uint32_t *unsettled, const uint32_t *err)
{
    *out = (unsettled && *unsettled) ? 1u : (*err ? 2u : 0u);
}
} // namespace
} // namespace dgf

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

namespace {

// The body of dgf_epic (max_relax == 0: relaxation checked from the host until it settles, the
// outcome returned) and of dgf_epic_async (max_relax > 0 launches, the outcome left in
// *status_out on the device).
int epic_run(const dgf_image *I0, const float *points, const float *flow, const uint8_t *status, int64_t n,
             const dgf_epic_opts *opts, void *workspace, size_t ws_bytes, float *dense, int64_t dense_pitch,
             int32_t *labels, uint32_t *dist, int32_t *nbr, uint32_t *nbr_dist, float *model, void *stream,
             int max_relax, uint32_t *status_out)
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
    const uint32_t *unsettled = nullptr; // (the async form) the last relaxation launch's changed count
    if (n > 0) {
        hipLaunchKernelGGL(k_epic_seed, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, points, flow, status, n, W,
                           H, ws.keys);
        if (hipGetLastError() != hipSuccess) return DGF_ERR_HIP;
        const dim3 tiles((unsigned)((W + kRTX - 1) / kRTX), (unsigned)((H + kRTY - 1) / kRTY));
        const int64_t ntiles = (int64_t)tiles.x * tiles.y;
        // tiles may wait for each other only if the whole grid is resident at once
        int dev = 0, cus = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_epic_relax, kRelaxThreads, 0) != hipSuccess)
            return DGF_ERR_HIP;
        const int wait = ntiles <= (int64_t)cus * per_cu ? 1 : 0;
        uint32_t *busy = ws.ctr + kChunk + 2, *carry = ws.ctr + 2 * kChunk + 2;
        const bool sync = max_relax == 0;
        const int limit = sync ? kMaxRelaxLaunches : max_relax;
        bool converged = false;
        int last = 0; // the index of the last launch of the last group
        // when the tiles can wait for each other one launch usually reaches the fixed point, so
        // the first check comes after two launches (work + confirmation), later ones after kChunk;
        // a launch after one that changed nothing returns at once
        for (int base = 0, chunk = wait ? 2 : kChunk; base < limit && !converged; base += chunk, chunk = kChunk) {
            chunk = chunk < limit - base ? chunk : limit - base;
            hipLaunchKernelGGL(k_epic_clear_launch_counters, dim3(1), dim3(256), 0, st, ws.ctr, busy, ws.mail,
                               chunk, (uint32_t)ntiles, carry, base > 0 ? last : -1);
            for (int j = 0; j < chunk; ++j)
                hipLaunchKernelGGL(k_epic_relax, tiles, dim3(kRelaxThreads), 0, st, W, H, o.kappa, ws.keys,
                                   (const uint16_t *)ws.E, ws.ctr + j, busy + j, ws.mail + j * ntiles, wait,
                                   j > 0 ? (const uint32_t *)(ws.ctr + j - 1) : (base > 0 ? (const uint32_t *)carry : nullptr));
            if (hipGetLastError() != hipSuccess) return DGF_ERR_HIP;
            last = chunk - 1;
            if (sync) {
                uint32_t h_changed[kChunk];
                if (hipMemcpyAsync(h_changed, ws.ctr, sizeof(uint32_t) * chunk, hipMemcpyDeviceToHost, st) !=
                        hipSuccess ||
                    hipStreamSynchronize(st) != hipSuccess)
                    return DGF_ERR_HIP;
                converged = h_changed[chunk - 1] == 0u;
            }
        }
        if (sync && !converged) return DGF_ERR_UNSUPPORTED;
        unsettled = sync ? nullptr : ws.ctr + last;
        hipLaunchKernelGGL(k_epic_graph, dim3(grid_for(N, 256)), dim3(256), 0, st, W, H, o.kappa,
                           (const uint64_t *)ws.keys, (const uint16_t *)ws.E, ws, err, ws.ctr + kChunk + 1, unsettled);
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
        F.min_edge = ws.ctr + kChunk + 1;
        F.unsettled = unsettled;
        hipLaunchKernelGGL(k_epic_knn_fit, dim3((unsigned)n), dim3(64), 0, st, F);
        if (hipGetLastError() != hipSuccess) return DGF_ERR_HIP;
    }
    hipLaunchKernelGGL(k_epic_dense, dim3(grid_for(N, 256)), dim3(256), 0, st, W, H, (const uint64_t *)ws.keys,
                       (const float *)ws.model, dense, dense_pitch, labels, dist, unsettled);
    if (hipGetLastError() != hipSuccess) return DGF_ERR_HIP;
    if (max_relax > 0) {
        hipLaunchKernelGGL(k_epic_status, dim3(1), dim3(1), 0, st, status_out, unsettled, (const uint32_t *)err);
        return hipGetLastError() == hipSuccess ? DGF_OK : DGF_ERR_HIP;
    }
    uint32_t h_err = 0;
    if (hipMemcpyAsync(&h_err, err, sizeof(h_err), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return DGF_ERR_HIP;
    return h_err ? DGF_ERR_CAPACITY : DGF_OK;
}

} // namespace

int dgf_epic(const dgf_image *I0, const float *points, const float *flow, const uint8_t *status, int64_t n,
             const dgf_epic_opts *opts, void *workspace, size_t ws_bytes, float *dense, int64_t dense_pitch,
             int32_t *labels, uint32_t *dist, int32_t *nbr, uint32_t *nbr_dist, float *model, void *stream)
{
    return epic_run(I0, points, flow, status, n, opts, workspace, ws_bytes, dense, dense_pitch, labels, dist, nbr,
                    nbr_dist, model, stream, 0, nullptr);
}

int dgf_epic_async(const dgf_image *I0, const float *points, const float *flow, const uint8_t *status, int64_t n,
                   const dgf_epic_opts *opts, void *workspace, size_t ws_bytes, float *dense, int64_t dense_pitch,
                   int32_t *labels, uint32_t *dist, int32_t *nbr, uint32_t *nbr_dist, float *model,
                   int32_t max_relax, uint32_t *status_out, void *stream)
{
    if (max_relax < 0 || max_relax > kMaxRelaxLaunches || !status_out || (uintptr_t)status_out % 4 != 0)
        return DGF_ERR_INVALID_ARG;
    return epic_run(I0, points, flow, status, n, opts, workspace, ws_bytes, dense, dense_pitch, labels, dist, nbr,
                    nbr_dist, model, stream, max_relax ? max_relax : kDefaultAsyncRelax, status_out);
}

} // extern "C"
