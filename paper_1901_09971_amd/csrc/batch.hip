// batch.hip -- many frame pairs of uneven size and point count in one pass: a plan built once on
// the host (descriptor tables and every pyramid in one device allocation), then per run
//   * one launch making level 1 of all 2P frames beside the detection of all pairs (job tables,
//     per-pair window and stride), then one launch per coarser level covering all frames,
//   * a one-block kernel that clears the work counters (no memset node, so the sequence can be
//     captured in a graph and replayed),
//   * one persistent tracking launch: a resident-sized grid whose wavefronts pull work items
//     (a group of points of one pair) from per-XCD counters over contiguous item ranges, so the
//     pairs one XCD tracks stay in its own L2, and steal from the other ranges once theirs is
//     drained.
// Outputs of all pairs are concatenated in pair order.  The whole sequence can be captured once
// into a hipGraph and replayed with a single launch.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <new>
#include <vector>

#include "dgf_internal.hpp"
#include "dgf_tuning.hpp"

namespace dgf {

// Clears the kNumXcd work counters (one thread each; launched as one block of kNumXcd threads).
__global__ void k_clear_counters(uint32_t *c)
{
    if (threadIdx.x < kNumXcd) c[(size_t)threadIdx.x * kCounterStride] = 0u;
}

// Grid-stride clear of a float buffer (a kernel, not a memset, so a captured graph can hold it).
__global__ void k_zero_f32(float *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0.f;
}

} // namespace dgf

using namespace dgf;

struct dgf_batch {
    int P = 0, L = 0, s = 0, iters = 0, dtype = 0;
    dgf_track_opts opts{};
    TrackTuning tune{};
    std::vector<int64_t> pt_off, item_off;
    int64_t total_pts = 0, nitems = 0, grid_waves = 0;
    void *dmem = nullptr;
    LevelPair *d_lv = nullptr;
    std::vector<LevelPair> h_lv; // host copy of the level table
    int64_t *d_item_off = nullptr, *d_pt_off = nullptr;
    uint32_t *d_counter = nullptr;
    AdjPair *d_adj = nullptr; // per-pair frames and gradient-map offsets for the adjoint
    std::vector<int64_t> grad_off; // first float of each pair's dI0 (dI1 follows), P + 1 entries
    PyrJob *d_pyr = nullptr; // [(L-1)][2P]
    double *d_gm = nullptr;  // global-motion fit state (models, then partial sums), DGF_TRACK_GLOBAL only
    int gm_nblk = 0;
    DetectJob *d_det = nullptr;
    std::vector<int> pyr_w2, pyr_h2; // per level 1..L-1: largest output size over the frames
    int det_tiles_x = 0, det_tiles_y = 0;
    size_t det_lds = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

bool pair_ok(const dgf_pair_desc &d, int dtype)
{
    auto ok = [&](const dgf_image &im) {
        const int e = im.dtype == DGF_U8 ? 1 : (im.dtype == DGF_F32 ? 4 : 0);
        return im.data && im.width >= 1 && im.height >= 1 && e && im.dtype == dtype &&
               im.pitch_bytes >= (int64_t)im.width * e && im.pitch_bytes < (1 << 24) && im.height < (1 << 24) &&
               im.pitch_bytes <= (int64_t)INT32_MAX / im.height &&
               (e == 1 || (im.pitch_bytes % 4 == 0 && (uintptr_t)im.data % 4 == 0));
    };
    return ok(d.I0) && ok(d.I1) && d.I0.width == d.I1.width && d.I0.height == d.I1.height && d.window >= 1 &&
           d.window <= DGF_MAX_WINDOW && d.stride >= 1;
}

// Level 1 of every frame beside every pair's detection, then the coarser levels.
int launch_front(dgf_batch *b, float *points, hipStream_t st)
{
    BatchFront F{};
    F.pyr = b->d_pyr;
    F.det = b->d_det;
    F.nframes = 2 * b->P;
    F.npairs = b->P;
    F.L = b->L;
    for (int l = 1; l < b->L; ++l) {
        F.max_w2[l] = b->pyr_w2[l];
        F.max_h2[l] = b->pyr_h2[l];
    }
    F.det_tx = b->det_tiles_x;
    F.det_ty = b->det_tiles_y;
    F.det_lds = b->det_lds;
    return launch_front_batched(F, points, st) == hipSuccess ? DGF_OK : DGF_ERR_HIP;
}

// Work counters, then the persistent tracking launch (with the global prior: its first pass, the
// fit and fresh counters before it).
int launch_track_all(dgf_batch *b, const float *points, float *flow, uint8_t *status, int32_t *iters_out,
                     float *illum_out, hipStream_t st)
{
    hipLaunchKernelGGL(k_clear_counters, dim3(1), dim3(kNumXcd), 0, st, b->d_counter);
    if (hipGetLastError() != hipSuccess) return DGF_ERR_HIP;
    TrackParams P{};
    P.pts = points;
    P.n = b->total_pts;
    P.flow = flow;
    P.status = status;
    P.iters_out = iters_out;
    P.illum_out = illum_out;
    P.L = b->L;
    P.iters = b->iters;
    fill_track_geometry(P, b->s, b->tune.margin, b->tune.lpp, b->tune.kind);
    fill_track_constants(P, b->opts, b->s);
    P.npairs = b->P;
    P.persistent = 1;
    P.blv = b->d_lv;
    P.item_off = b->d_item_off;
    P.pt_off = b->d_pt_off;
    P.counter = b->d_counter;
    P.nitems = b->nitems;
    P.grid_waves = b->grid_waves;
    if (b->opts.flags & DGF_TRACK_GLOBAL) {
        // every pair's coarsest-level pass, every pair's global fit, fresh work counters, then the
        // tracking proper from each pair's fitted motion
        GmFit g{};
        g.pts = reinterpret_cast<const float2 *>(points);
        g.flow = reinterpret_cast<const float2 *>(flow);
        g.status = status;
        g.pt_off = b->d_pt_off;
        g.blv = b->d_lv;
        g.L = b->L;
        g.npairs = b->P;
        g.nblk = b->gm_nblk;
        g.c = kTukeyC * ldexp(1.0, b->L - 1);
        g.models = b->d_gm;
        g.part = (double *)((uint8_t *)b->d_gm + gm_models_bytes(b->P));
        P.lstop = b->L - 1;
        P.iters_out = nullptr;
        P.illum_out = nullptr;
        if (launch_track(P, b->tune, b->dtype, st) != hipSuccess) return DGF_ERR_HIP;
        if (launch_gm_fit(g, st) != hipSuccess) return DGF_ERR_HIP;
        hipLaunchKernelGGL(k_clear_counters, dim3(1), dim3(kNumXcd), 0, st, b->d_counter);
        if (hipGetLastError() != hipSuccess) return DGF_ERR_HIP;
        P.lstop = 0;
        P.gm_model = g.models;
        P.iters_out = iters_out;
        P.illum_out = illum_out;
    }
    return launch_track(P, b->tune, b->dtype, st) == hipSuccess ? DGF_OK : DGF_ERR_HIP;
}

int launch_all(dgf_batch *b, float *points, float *flow, uint8_t *status, int32_t *iters_out, float *illum_out,
               hipStream_t st)
{
    const int rc = launch_front(b, points, st);
    return rc != DGF_OK ? rc : launch_track_all(b, points, flow, status, iters_out, illum_out, st);
}

int check_run(const dgf_batch *b, const float *points, const float *flow, const uint8_t *status, const float *illum_out)
{
    if (!b) return DGF_ERR_INVALID_ARG;
    if (b->total_pts > 0 && (!points || !flow || !status)) return DGF_ERR_INVALID_ARG;
    if (illum_out && !(b->opts.flags & DGF_TRACK_ILLUM)) return DGF_ERR_INVALID_ARG;
    return DGF_OK;
}

} // namespace

extern "C" {

int dgf_batch_create(const dgf_pair_desc *pairs, int32_t npairs, int32_t levels, int32_t support, int32_t iters,
                     const dgf_track_opts *opts, dgf_batch **out)
{
    if (!out) return DGF_ERR_INVALID_ARG;
    *out = nullptr;
    if (!pairs || npairs < 1 || npairs > 65535) return DGF_ERR_INVALID_ARG;
    if (levels < 1 || levels > DGF_MAX_LEVELS || iters < 1) return DGF_ERR_INVALID_ARG;
    if (support < 1 || (support & 1) == 0 || support > DGF_MAX_SUPPORT) return DGF_ERR_INVALID_ARG;
    const int dtype = pairs[0].I0.dtype;
    for (int i = 0; i < npairs; ++i)
        if (!pair_ok(pairs[i], dtype)) return DGF_ERR_INVALID_ARG;
    dgf_track_opts o;
    const int orc = effective_track_opts(opts, support, &o);
    if (orc != DGF_OK) return orc;
    for (int i = 0; i < npairs; ++i)
        if (front_detect_lds(pairs[i].window, pairs[i].stride) > kMaxLdsPerBlock) return DGF_ERR_UNSUPPORTED;

    dgf_batch *b = new (std::nothrow) dgf_batch();
    if (!b) return DGF_ERR_INVALID_ARG;
    b->P = npairs;
    b->L = levels;
    b->s = support;
    b->iters = iters;
    b->dtype = dtype;
    b->opts = o;
    int64_t total_n = 0;
    for (int i = 0; i < npairs; ++i)
        total_n += dgf_detect_count(pairs[i].I0.width, pairs[i].I0.height, pairs[i].window, pairs[i].stride);
    b->tune = tuning_for(support, levels, dtype, total_n);
    if (o.flags & kRowRunFlags) b->tune = illum_tuning(support, b->tune);
    if (!track_shape_ok(support, b->tune)) {
        delete b;
        return DGF_ERR_UNSUPPORTED;
    }
    while (track_lds_bytes(support, b->tune) > kMaxLdsPerBlock && b->tune.wpb > 1) b->tune.wpb /= 2;
    if (track_lds_bytes(support, b->tune) > kMaxLdsPerBlock) {
        delete b;
        return DGF_ERR_UNSUPPORTED;
    }
    const int ppw = 64 / b->tune.lpp;

    // point and work-item prefix sums; detection jobs
    b->pt_off.assign(npairs + 1, 0);
    b->item_off.assign(npairs + 1, 0);
    std::vector<DetectJob> det(npairs);
    for (int i = 0; i < npairs; ++i) {
        const dgf_pair_desc &d = pairs[i];
        const int64_t n = dgf_detect_count(d.I0.width, d.I0.height, d.window, d.stride);
        b->pt_off[i + 1] = b->pt_off[i] + n;
        b->item_off[i + 1] = b->item_off[i] + (n + ppw - 1) / ppw;
        DetectJob j{};
        j.img = (const uint8_t *)d.I0.data;
        j.pitch = d.I0.pitch_bytes;
        j.W = d.I0.width;
        j.H = d.I0.height;
        j.win = d.window;
        j.stride = d.stride;
        j.nx = n ? (d.I0.width - d.window) / d.stride + 1 : 0;
        j.ny = n ? (d.I0.height - d.window) / d.stride + 1 : 0;
        j.out_off = b->pt_off[i];
        det[i] = j;
        b->det_tiles_x = std::max(b->det_tiles_x, (j.nx + 15) / 16);
        b->det_tiles_y = std::max(b->det_tiles_y, (j.ny + 15) / 16);
        b->det_lds = std::max(b->det_lds, front_detect_lds(d.window, d.stride));
    }
    b->total_pts = b->pt_off[npairs];
    b->nitems = b->item_off[npairs];
    if (dtype != DGF_U8) { // detection reads uint8 frames
        delete b;
        return DGF_ERR_UNSUPPORTED;
    }
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        delete b;
        return DGF_ERR_HIP;
    }
    // persistent grid: 32 wavefront slots per CU; waves beyond what fits start after the first
    // ones drain the queue and exit at once
    b->grid_waves = std::min<int64_t>(b->nitems, (int64_t)cus * 32);
    if (b->grid_waves < 1) b->grid_waves = 1;

    // largest size of every level over the frames
    b->pyr_w2.assign(levels, 0);
    b->pyr_h2.assign(levels, 0);
    for (int i = 0; i < npairs; ++i) {
        int W = pairs[i].I0.width, H = pairs[i].I0.height;
        for (int l = 1; l < levels; ++l) {
            W = (W + 1) / 2;
            H = (H + 1) / 2;
            b->pyr_w2[l] = std::max(b->pyr_w2[l], W);
            b->pyr_h2[l] = std::max(b->pyr_h2[l], H);
        }
    }

    // device layout: [level table][item_off][pt_off][counter][pyramid jobs][detect jobs]
    // [adjoint table][global-motion state][pyramids]
    std::vector<int64_t> pyr_bytes(npairs), pyr_base(npairs);
    int64_t sz = 0;
    const int64_t o_lv = sz;
    sz = align_up(sz + (int64_t)sizeof(LevelPair) * npairs * levels, 256);
    const int64_t o_item = sz;
    sz = align_up(sz + 8 * (npairs + 1), 256);
    const int64_t o_pt = sz;
    sz = align_up(sz + 8 * (npairs + 1), 256);
    const int64_t o_ctr = sz;
    sz = align_up(sz + 4 * kCounterStride * kNumXcd, 256);
    const int64_t o_pyrjobs = sz;
    sz = align_up(sz + (int64_t)sizeof(PyrJob) * 2 * npairs * std::max(levels - 1, 1), 256);
    const int64_t o_det = sz;
    sz = align_up(sz + (int64_t)sizeof(DetectJob) * npairs, 256);
    const int64_t o_adj = sz;
    sz = align_up(sz + (int64_t)sizeof(AdjPair) * npairs, 256);
    int64_t max_n = 0;
    for (int i = 0; i < npairs; ++i) max_n = std::max(max_n, b->pt_off[i + 1] - b->pt_off[i]);
    b->gm_nblk = gm_blocks(max_n);
    const int64_t o_gm = sz;
    if (o.flags & DGF_TRACK_GLOBAL) sz = align_up(sz + (int64_t)gm_state_bytes(npairs, b->gm_nblk), 256);
    for (int i = 0; i < npairs; ++i) {
        pyr_bytes[i] = (int64_t)dgf_pyramid_layout(pairs[i].I0.width, pairs[i].I0.height, levels, dtype, nullptr, nullptr);
        pyr_base[i] = sz;
        sz = align_up(sz + 2 * pyr_bytes[i], 256);
    }
    if (hipMalloc(&b->dmem, (size_t)sz) != hipSuccess) {
        b->dmem = nullptr;
        delete b;
        return DGF_ERR_HIP;
    }
    uint8_t *base = (uint8_t *)b->dmem;
    b->d_lv = (LevelPair *)(base + o_lv);
    b->d_item_off = (int64_t *)(base + o_item);
    b->d_pt_off = (int64_t *)(base + o_pt);
    b->d_counter = (uint32_t *)(base + o_ctr);
    b->d_pyr = (PyrJob *)(base + o_pyrjobs);
    b->d_det = (DetectJob *)(base + o_det);
    b->d_adj = (AdjPair *)(base + o_adj);
    if (o.flags & DGF_TRACK_GLOBAL) b->d_gm = (double *)(base + o_gm);

    // level table and pyramid jobs
    std::vector<LevelPair> lv((size_t)npairs * levels);
    std::vector<PyrJob> jobs((size_t)2 * npairs * std::max(levels - 1, 1));
    for (int i = 0; i < npairs; ++i) {
        int64_t off[DGF_MAX_LEVELS], pitch[DGF_MAX_LEVELS];
        dgf_pyramid_layout(pairs[i].I0.width, pairs[i].I0.height, levels, dtype, off, pitch);
        uint8_t *w0 = base + pyr_base[i], *w1 = w0 + pyr_bytes[i];
        LevelPair *L = &lv[(size_t)i * levels];
        L[0] = LevelPair{(const uint8_t *)pairs[i].I0.data, (const uint8_t *)pairs[i].I1.data, pairs[i].I0.pitch_bytes,
                         pairs[i].I1.pitch_bytes, pairs[i].I0.width, pairs[i].I0.height};
        int W = pairs[i].I0.width, H = pairs[i].I0.height;
        for (int l = 1; l < levels; ++l) {
            jobs[(size_t)(l - 1) * 2 * npairs + 2 * i] = PyrJob{L[l - 1].p0, w0 + off[l], L[l - 1].pitch0, pitch[l], W, H};
            jobs[(size_t)(l - 1) * 2 * npairs + 2 * i + 1] = PyrJob{L[l - 1].p1, w1 + off[l], L[l - 1].pitch1, pitch[l], W, H};
            W = (W + 1) / 2;
            H = (H + 1) / 2;
            L[l] = LevelPair{w0 + off[l], w1 + off[l], pitch[l], pitch[l], W, H};
        }
    }
    // adjoint table: level-0 frames, and each pair's two gradient maps (row pitch = width)
    std::vector<AdjPair> adj(npairs);
    b->grad_off.assign(npairs + 1, 0);
    for (int i = 0; i < npairs; ++i) {
        const dgf_pair_desc &d = pairs[i];
        const int64_t wh = (int64_t)d.I0.width * d.I0.height;
        const int64_t g0 = b->grad_off[i];
        adj[i] = AdjPair{(const uint8_t *)d.I0.data, (const uint8_t *)d.I1.data, d.I0.pitch_bytes, d.I1.pitch_bytes,
                         g0, g0 + wh, d.I0.width, d.I0.width, d.I0.width, d.I0.height};
        b->grad_off[i + 1] = g0 + 2 * wh;
    }
    b->h_lv = lv;
    bool ok = hipMemcpy(b->d_lv, lv.data(), sizeof(LevelPair) * lv.size(), hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(b->d_adj, adj.data(), sizeof(AdjPair) * adj.size(), hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(b->d_item_off, b->item_off.data(), 8 * (npairs + 1), hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(b->d_pt_off, b->pt_off.data(), 8 * (npairs + 1), hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(b->d_pyr, jobs.data(), sizeof(PyrJob) * jobs.size(), hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(b->d_det, det.data(), sizeof(DetectJob) * det.size(), hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) {
        (void)hipFree(b->dmem);
        delete b;
        return DGF_ERR_HIP;
    }
    *out = b;
    return DGF_OK;
}

int64_t dgf_batch_num_points(const dgf_batch *b) { return b ? b->total_pts : -1; }

int dgf_batch_point_offsets(const dgf_batch *b, int64_t *offsets)
{
    if (!b || !offsets) return DGF_ERR_INVALID_ARG;
    memcpy(offsets, b->pt_off.data(), sizeof(int64_t) * (b->P + 1));
    return DGF_OK;
}

int dgf_batch_run(dgf_batch *b, float *points, float *flow, uint8_t *status, int32_t *iters_out, float *illum_out,
                  void *stream)
{
    const int rc = check_run(b, points, flow, status, illum_out);
    if (rc != DGF_OK || b->total_pts == 0) return rc;
    return launch_all(b, points, flow, status, iters_out, illum_out, (hipStream_t)stream);
}

int dgf_batch_front(dgf_batch *b, float *points, void *stream)
{
    if (!b) return DGF_ERR_INVALID_ARG;
    if (b->total_pts > 0 && !points) return DGF_ERR_INVALID_ARG;
    if (b->total_pts == 0) return DGF_OK;
    return launch_front(b, points, (hipStream_t)stream);
}

int dgf_batch_track(dgf_batch *b, const float *points, float *flow, uint8_t *status, int32_t *iters_out,
                    float *illum_out, void *stream)
{
    const int rc = check_run(b, points, flow, status, illum_out);
    if (rc != DGF_OK || b->total_pts == 0) return rc;
    return launch_track_all(b, points, flow, status, iters_out, illum_out, (hipStream_t)stream);
}

int dgf_batch_capture(dgf_batch *b, float *points, float *flow, uint8_t *status, float *illum_out, void *stream)
{
    if (!b || !stream) return DGF_ERR_INVALID_ARG; // graphs are captured from a created stream
    const int crc = check_run(b, points, flow, status, illum_out);
    if (crc != DGF_OK) return crc;
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    if (b->total_pts == 0) return DGF_OK;
    hipStream_t st = (hipStream_t)stream;
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return DGF_ERR_HIP;
    const int rc = launch_all(b, points, flow, status, nullptr, illum_out, st);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &g);
    if (rc != DGF_OK || e != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        return rc != DGF_OK ? rc : DGF_ERR_HIP;
    }
    hipGraphExec_t ex = nullptr;
    if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return DGF_ERR_HIP;
    }
    b->graph = g;
    b->exec = ex;
    return DGF_OK;
}

int dgf_batch_replay(dgf_batch *b, void *stream)
{
    if (!b) return DGF_ERR_INVALID_ARG;
    if (b->total_pts == 0) return DGF_OK;
    if (!b->exec) return DGF_ERR_INVALID_ARG;
    return hipGraphLaunch(b->exec, (hipStream_t)stream) == hipSuccess ? DGF_OK : DGF_ERR_HIP;
}

int dgf_batch_level(const dgf_batch *b, int pair, int frame, int level, const uint8_t **data, int64_t *pitch_bytes,
                    int32_t *width, int32_t *height)
{
    if (!b || !data || !pitch_bytes || !width || !height) return DGF_ERR_INVALID_ARG;
    if (pair < 0 || pair >= b->P || (frame != 0 && frame != 1) || level < 0 || level >= b->L) return DGF_ERR_INVALID_ARG;
    const LevelPair &v = b->h_lv[(size_t)pair * b->L + level];
    *data = frame ? v.p1 : v.p0;
    *pitch_bytes = frame ? v.pitch1 : v.pitch0;
    *width = v.W;
    *height = v.H;
    return DGF_OK;
}

int64_t dgf_batch_grad_size(const dgf_batch *b, int64_t *offsets)
{
    if (!b) return -1;
    if (offsets) memcpy(offsets, b->grad_off.data(), sizeof(int64_t) * (b->P + 1));
    return b->grad_off[b->P];
}

int dgf_batch_backward(dgf_batch *b, const float *points, const float *flow, const uint8_t *status, const float *dflow,
                       const float *illum, float *grad, void *stream)
{
    if (!b) return DGF_ERR_INVALID_ARG;
    if (b->total_pts > 0 && (!points || !flow || !status || !dflow || !grad)) return DGF_ERR_INVALID_ARG;
    if (grad && (uintptr_t)grad % 4 != 0) return DGF_ERR_INVALID_ARG;
    if (b->opts.flags & DGF_TRACK_CROSS) return DGF_ERR_UNSUPPORTED; // cross-based supports are not differentiated
    const bool im = (b->opts.flags & DGF_TRACK_ILLUM) != 0;
    if (im && b->total_pts > 0 && !illum) return DGF_ERR_INVALID_ARG;
    if (!im && illum) return DGF_ERR_INVALID_ARG;
    if (b->total_pts == 0) return DGF_OK;
    hipStream_t st = (hipStream_t)stream;
    const int64_t ng = b->grad_off[b->P];
    const int64_t blocks = std::min<int64_t>((ng + 1023) / 1024, 8192);
    hipLaunchKernelGGL(k_zero_f32, dim3((unsigned)blocks), dim3(256), 0, st, grad, ng);
    if (hipGetLastError() != hipSuccess) return DGF_ERR_HIP;
    AdjParams A{};
    A.pairs = b->d_adj;
    A.pt_off = b->d_pt_off;
    A.npairs = b->P;
    A.grad0 = grad;
    A.grad1 = grad;
    A.s = b->s;
    A.r = b->s / 2;
    A.pts = points;
    A.flow = flow;
    A.dflow = dflow;
    A.status = status;
    A.illum = im ? illum : nullptr;
    A.n = b->total_pts;
    fill_adjoint_constants(A, b->opts);
    return launch_track_adjoint(A, b->dtype, st) == hipSuccess ? DGF_OK : DGF_ERR_HIP;
}

int dgf_batch_destroy(dgf_batch *b)
{
    if (!b) return DGF_OK;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    int rc = DGF_OK;
    if (b->dmem && hipFree(b->dmem) != hipSuccess) rc = DGF_ERR_HIP;
    delete b;
    return rc;
}

} // extern "C"
