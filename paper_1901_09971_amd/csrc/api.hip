// api.hip -- host side of the C ABI declared in include/degraf_flow.h: argument validation,
// pyramid/workspace layout and kernel launches on the caller's stream.  No call here allocates
// device memory or synchronises the host.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "dgf_internal.hpp"
#include "dgf_tuning.hpp"

using namespace dgf;

namespace {

int esize(int dtype) { return dtype == DGF_U8 ? 1 : (dtype == DGF_F32 ? 4 : 0); }

bool image_ok(const dgf_image *im)
{
    if (!im || !im->data) return false;
    if (im->width < 1 || im->height < 1) return false;
    const int e = esize(im->dtype);
    if (e == 0) return false;
    if (im->pitch_bytes < (int64_t)im->width * e) return false;
    if (im->dtype == DGF_F32 && ((uintptr_t)im->data % 4 != 0 || im->pitch_bytes % 4 != 0)) return false;
    // kernels address pixels with 24-bit row x pitch products and 32-bit byte offsets
    if (im->pitch_bytes >= (1 << 24) || im->height >= (1 << 24) || im->pitch_bytes > (int64_t)INT32_MAX / im->height)
        return false;
    return true;
}

int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

int hip_rc(hipError_t e) { return e == hipSuccess ? DGF_OK : DGF_ERR_HIP; }

} // namespace

extern "C" {

const char *dgf_strerror(int code)
{
    switch (code) {
    case DGF_OK: return "ok";
    case DGF_ERR_INVALID_ARG: return "invalid argument";
    case DGF_ERR_CAPACITY: return "output capacity too small";
    case DGF_ERR_UNSUPPORTED: return "unsupported configuration";
    case DGF_ERR_HIP: return "HIP runtime error";
    case DGF_ERR_WORKSPACE: return "workspace missing or too small";
    case DGF_ERR_SCRATCH: return "input larger than the static scratch of dgf_track_static";
    default: return "unknown error";
    }
}

int dgf_version(void) { return 100; }

int dgf_track_opts_default(dgf_track_opts *o)
{
    if (!o) return DGF_ERR_INVALID_ARG;
    o->sigma1 = 8.0f;
    o->sigma2 = 32.0f;
    o->eps_coarse = 1e-2f;
    o->eps_fine = 1e-4f;
    o->min_eig = 1e-4f * 255.0f * 255.0f;
    o->flags = 0;
    o->cross_tau = 25.0f;
    return DGF_OK;
}

int64_t dgf_detect_count(int32_t W, int32_t H, int32_t window, int32_t stride)
{
    if (window < 1 || stride < 1) return -1;
    if (W < window || H < window) return 0;
    return (int64_t)((W - window) / stride + 1) * (int64_t)((H - window) / stride + 1);
}

int dgf_detect(const dgf_image *I0, int32_t window, int32_t stride, float *points, uint8_t *sel, float *response,
               int64_t capacity, void *stream)
{
    if (!image_ok(I0) || I0->dtype != DGF_U8) return DGF_ERR_INVALID_ARG;
    if (window < 1 || window > DGF_MAX_WINDOW || stride < 1) return DGF_ERR_INVALID_ARG;
    const int64_t N = dgf_detect_count(I0->width, I0->height, window, stride);
    if (N == 0) return DGF_OK;
    if (!points) return DGF_ERR_INVALID_ARG;
    if (capacity < N) return DGF_ERR_CAPACITY;
    return hip_rc(launch_detect((const uint8_t *)I0->data, I0->pitch_bytes, I0->width, I0->height, window, stride, points,
                                sel, response, (hipStream_t)stream));
}

size_t dgf_pyramid_layout(int32_t W, int32_t H, int32_t levels, int32_t dtype, int64_t *offsets, int64_t *pitches)
{
    const int e = esize(dtype);
    if (W < 1 || H < 1 || levels < 1 || levels > DGF_MAX_LEVELS || e == 0) return 0;
    int64_t total = 0;
    if (offsets) offsets[0] = 0;
    if (pitches) pitches[0] = 0;
    for (int l = 1; l < levels; ++l) {
        W = (W + 1) / 2;
        H = (H + 1) / 2;
        const int64_t pitch = align_up((int64_t)W * e, 64);
        total = align_up(total, 256);
        if (offsets) offsets[l] = total;
        if (pitches) pitches[l] = pitch;
        total += pitch * H;
    }
    return (size_t)align_up(total, 256);
}

int dgf_pyramid(const dgf_image *src, int32_t levels, void *dst, size_t dst_bytes, void *stream)
{
    if (!image_ok(src) || levels < 1 || levels > DGF_MAX_LEVELS) return DGF_ERR_INVALID_ARG;
    int64_t off[DGF_MAX_LEVELS], pitch[DGF_MAX_LEVELS];
    const size_t need = dgf_pyramid_layout(src->width, src->height, levels, src->dtype, off, pitch);
    if (levels == 1) return DGF_OK;
    if (!dst || dst_bytes < need) return DGF_ERR_WORKSPACE;
    const uint8_t *prev = (const uint8_t *)src->data;
    int64_t prev_pitch = src->pitch_bytes;
    int W = src->width, H = src->height;
    if (src->dtype == DGF_U8) {
        const uint8_t *srcs[2] = {prev, nullptr};
        const int64_t sp[2] = {prev_pitch, 0};
        uint8_t *lvl[2][DGF_MAX_LEVELS] = {};
        for (int l = 1; l < levels; ++l) lvl[0][l] = (uint8_t *)dst + off[l];
        return launch_pyr_chains(srcs, sp, lvl, pitch, W, H, levels, 1, (hipStream_t)stream) == hipSuccess ? DGF_OK
                                                                                                          : DGF_ERR_HIP;
    }
    for (int l = 1; l < levels; ++l) {
        PyrJob j{prev, (uint8_t *)dst + off[l], prev_pitch, pitch[l], W, H};
        const hipError_t e = launch_pyr_level(&j, 1, src->dtype, (hipStream_t)stream);
        if (e != hipSuccess) return DGF_ERR_HIP;
        prev = (const uint8_t *)dst + off[l];
        prev_pitch = pitch[l];
        W = (W + 1) / 2;
        H = (H + 1) / 2;
    }
    return DGF_OK;
}

size_t dgf_track_workspace_bytes(int32_t W, int32_t H, int32_t levels, int32_t dtype)
{
    if (W < 1 || H < 1 || levels < 1 || levels > DGF_MAX_LEVELS || esize(dtype) == 0) return 0;
    // both pyramids, then the global-motion fit's state
    return 2 * dgf_pyramid_layout(W, H, levels, dtype, nullptr, nullptr) + gm_state_bytes(1, kGmMaxBlocks);
}

namespace {

int check_pair(const dgf_image *I0, const dgf_image *I1, int32_t levels)
{
    if (!image_ok(I0) || !image_ok(I1)) return DGF_ERR_INVALID_ARG;
    if (I0->width != I1->width || I0->height != I1->height || I0->dtype != I1->dtype) return DGF_ERR_INVALID_ARG;
    if (levels < 1 || levels > DGF_MAX_LEVELS) return DGF_ERR_INVALID_ARG;
    return DGF_OK;
}

// Level descriptors of both pyramids inside a track workspace (level 0 = the inputs).
void pyramid_levels(const dgf_image *I0, const dgf_image *I1, int32_t levels, const void *workspace, LevelPair *lv,
                    PyrJob *jobs /* nullable, [levels][2] */)
{
    int64_t off[DGF_MAX_LEVELS], pitch[DGF_MAX_LEVELS];
    const size_t pyr_bytes = dgf_pyramid_layout(I0->width, I0->height, levels, I0->dtype, off, pitch);
    uint8_t *ws0 = (uint8_t *)workspace;
    uint8_t *ws1 = ws0 ? ws0 + pyr_bytes : nullptr;
    lv[0] = LevelPair{(const uint8_t *)I0->data, (const uint8_t *)I1->data, I0->pitch_bytes, I1->pitch_bytes, I0->width,
                      I0->height};
    int W = I0->width, H = I0->height;
    for (int l = 1; l < levels; ++l) {
        if (jobs) {
            jobs[2 * l] = PyrJob{lv[l - 1].p0, ws0 + off[l], lv[l - 1].pitch0, pitch[l], W, H};
            jobs[2 * l + 1] = PyrJob{lv[l - 1].p1, ws1 + off[l], lv[l - 1].pitch1, pitch[l], W, H};
        }
        W = (W + 1) / 2;
        H = (H + 1) / 2;
        lv[l] = LevelPair{ws0 + off[l], ws1 + off[l], pitch[l], pitch[l], W, H};
    }
}

} // namespace

int dgf_track_pyramids(const dgf_image *I0, const dgf_image *I1, int32_t levels, void *workspace, size_t ws_bytes,
                       void *stream)
{
    const int rc = check_pair(I0, I1, levels);
    if (rc != DGF_OK) return rc;
    if (levels == 1) return DGF_OK;
    if (!workspace || ws_bytes < dgf_track_workspace_bytes(I0->width, I0->height, levels, I0->dtype))
        return DGF_ERR_WORKSPACE;
    LevelPair lv[DGF_MAX_LEVELS];
    PyrJob jobs[2 * DGF_MAX_LEVELS];
    pyramid_levels(I0, I1, levels, workspace, lv, jobs);
    if (I0->dtype == DGF_U8) {
        const uint8_t *srcs[2] = {lv[0].p0, lv[0].p1};
        const int64_t sp[2] = {lv[0].pitch0, lv[0].pitch1};
        uint8_t *lvl[2][DGF_MAX_LEVELS] = {};
        int64_t pitch[DGF_MAX_LEVELS] = {};
        for (int l = 1; l < levels; ++l) {
            lvl[0][l] = (uint8_t *)lv[l].p0;
            lvl[1][l] = (uint8_t *)lv[l].p1;
            pitch[l] = lv[l].pitch0;
        }
        return launch_pyr_chains(srcs, sp, lvl, pitch, I0->width, I0->height, levels, 2, (hipStream_t)stream) ==
                       hipSuccess
                   ? DGF_OK
                   : DGF_ERR_HIP;
    }
    for (int l = 1; l < levels; ++l) {
        const hipError_t e = launch_pyr_level(&jobs[2 * l], 2, I0->dtype, (hipStream_t)stream);
        if (e != hipSuccess) return DGF_ERR_HIP;
    }
    return DGF_OK;
}

int dgf_detect_pyramids(const dgf_image *I0, const dgf_image *I1, int32_t window, int32_t stride, int32_t levels,
                        void *workspace, size_t ws_bytes, float *points, uint8_t *sel, float *response,
                        int64_t capacity, void *stream)
{
    // everything both parts check, before anything is launched
    int rc = check_pair(I0, I1, levels);
    if (rc != DGF_OK) return rc;
    if (I0->dtype != DGF_U8) return DGF_ERR_INVALID_ARG;
    if (window < 1 || window > DGF_MAX_WINDOW || stride < 1) return DGF_ERR_INVALID_ARG;
    const int64_t n = dgf_detect_count(I0->width, I0->height, window, stride);
    if (n > 0 && !points) return DGF_ERR_INVALID_ARG;
    if (n > capacity) return DGF_ERR_CAPACITY;
    if (levels > 1 && (!workspace || ws_bytes < dgf_track_workspace_bytes(I0->width, I0->height, levels, I0->dtype)))
        return DGF_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    if (levels == 1 || n == 0 || !front_detect_fits(window, stride)) {
        if (n > 0) {
            rc = dgf_detect(I0, window, stride, points, sel, response, capacity, stream);
            if (rc != DGF_OK) return rc;
        }
        return dgf_track_pyramids(I0, I1, levels, workspace, ws_bytes, stream);
    }
    LevelPair lv[DGF_MAX_LEVELS];
    pyramid_levels(I0, I1, levels, workspace, lv, nullptr);
    const uint8_t *srcs[2] = {lv[0].p0, lv[0].p1};
    const int64_t sp[2] = {lv[0].pitch0, lv[0].pitch1};
    uint8_t *lvl[2][DGF_MAX_LEVELS] = {};
    int64_t pitch[DGF_MAX_LEVELS] = {};
    for (int l = 1; l < levels; ++l) {
        lvl[0][l] = (uint8_t *)lv[l].p0;
        lvl[1][l] = (uint8_t *)lv[l].p1;
        pitch[l] = lv[l].pitch0;
    }
    FrontDetect D{};
    D.img = (const uint8_t *)I0->data;
    D.pitch = I0->pitch_bytes;
    D.W = I0->width;
    D.H = I0->height;
    D.win = window;
    D.stride = stride;
    D.nx = (D.W - window) / stride + 1;
    D.ny = (D.H - window) / stride + 1;
    D.tiles_x = (D.nx + 15) / 16;
    D.tiles_y = (D.ny + 15) / 16;
    D.o = DetectOut{points, sel, response};
    return hip_rc(launch_pyr_chains(srcs, sp, lvl, pitch, I0->width, I0->height, levels, 2, st, &D));
}

} // extern "C"

namespace dgf {

// Validation shared by every tracking entry point; fills the effective options.
int validate_track(const dgf_image *I0, const dgf_image *I1, const float *points, int64_t n, int32_t levels,
                   int32_t support, int32_t iters, const dgf_track_opts *opts, const void *workspace, size_t ws_bytes,
                   const float *flow, const uint8_t *status, dgf_track_opts *o)
{
    const int rc = validate_track_args(I0, I1, points, n, levels, support, iters, opts, flow, status, o);
    if (rc != DGF_OK) return rc;
    if ((levels > 1 || (o->flags & DGF_TRACK_GLOBAL)) &&
        (!workspace || ws_bytes < dgf_track_workspace_bytes(I0->width, I0->height, levels, I0->dtype)))
        return DGF_ERR_WORKSPACE;
    return DGF_OK;
}

int validate_track_args(const dgf_image *I0, const dgf_image *I1, const float *points, int64_t n, int32_t levels,
                        int32_t support, int32_t iters, const dgf_track_opts *opts, const float *flow,
                        const uint8_t *status, dgf_track_opts *o)
{
    int rc = check_pair(I0, I1, levels);
    if (rc != DGF_OK) return rc;
    if (iters < 1) return DGF_ERR_INVALID_ARG;
    if (support < 1 || (support & 1) == 0 || support > DGF_MAX_SUPPORT) return DGF_ERR_INVALID_ARG;
    if (n < 0) return DGF_ERR_INVALID_ARG;
    if (n > 0 && (!points || !flow || !status)) return DGF_ERR_INVALID_ARG;
    return effective_track_opts(opts, support, o);
}

int effective_track_opts(const dgf_track_opts *opts, int32_t support, dgf_track_opts *o)
{
    if (opts) {
        *o = *opts;
        if ((o->flags & ~kTrackFlags) != 0) return DGF_ERR_UNSUPPORTED;
        if ((o->flags & kRowRunFlags) && run_shape_lanes(support) == 0) return DGF_ERR_UNSUPPORTED;
    } else {
        dgf_track_opts_default(o);
    }
    if (!(o->sigma1 >= 0.f) || !(o->sigma2 >= 0.f) || !(o->eps_coarse >= 0.f) || !(o->eps_fine >= 0.f) ||
        isnan(o->min_eig))
        return DGF_ERR_INVALID_ARG;
    if (isinf(o->sigma2) && !isinf(o->sigma1)) return DGF_ERR_INVALID_ARG; // no finite inner band with infinite outer
    if ((o->flags & DGF_TRACK_CROSS) && !(o->cross_tau >= 0.f && isfinite(o->cross_tau))) return DGF_ERR_INVALID_ARG;
    return DGF_OK;
}

// Global-motion fit state in a track workspace: after both pyramids.
GmFit gm_fit_for(const dgf_image *I0, int32_t levels, const void *workspace, const float *points,
                 const float *flow, const uint8_t *status, int64_t n)
{
    const size_t pyr = dgf_pyramid_layout(I0->width, I0->height, levels, I0->dtype, nullptr, nullptr);
    uint8_t *base = (uint8_t *)workspace + 2 * pyr;
    GmFit g{};
    g.pts = reinterpret_cast<const float2 *>(points);
    g.flow = reinterpret_cast<const float2 *>(flow);
    g.status = status;
    g.n = n;
    g.W = I0->width;
    g.H = I0->height;
    g.L = levels;
    g.npairs = 1;
    g.nblk = gm_blocks(n);
    g.c = kTukeyC * ldexp(1.0, levels - 1);
    g.models = reinterpret_cast<double *>(base);
    g.part = reinterpret_cast<double *>(base + gm_models_bytes(1));
    return g;
}

// Tracking on pyramids already in `workspace`, with an explicit launch shape (validated).
int track_run_with(const dgf_image *I0, const dgf_image *I1, const float *points, int64_t n, int32_t levels,
                   int32_t support, int32_t iters, const dgf_track_opts &o, const void *workspace, float *flow,
                   uint8_t *status, int32_t *iters_out, TrackTuning tune, hipStream_t st, float *illum_out)
{
    if (o.flags & kRowRunFlags) tune = illum_tuning(support, tune);
    if (!track_shape_ok(support, tune)) return DGF_ERR_UNSUPPORTED;
    while (track_lds_bytes(support, tune) > kMaxLdsPerBlock && tune.wpb > 1) tune.wpb /= 2;
    if (track_lds_bytes(support, tune) > kMaxLdsPerBlock) return DGF_ERR_UNSUPPORTED;
    if (n == 0) return DGF_OK;
    TrackParams P{};
    pyramid_levels(I0, I1, levels, workspace, P.lv, nullptr);
    P.pts = points;
    P.n = n;
    P.flow = flow;
    P.status = status;
    P.iters_out = iters_out;
    P.illum_out = illum_out;
    P.L = levels;
    P.iters = iters;
    fill_track_geometry(P, support, tune.margin, tune.lpp, tune.kind);
    fill_track_constants(P, o, support);
    if (o.flags & DGF_TRACK_GLOBAL) {
        // first pass on the coarsest level alone (into the outputs), the global fit into the
        // workspace, then the tracking proper from the fitted motion
        const GmFit g = gm_fit_for(I0, levels, workspace, points, flow, status, n);
        P.lstop = levels - 1;
        P.iters_out = nullptr;
        P.illum_out = nullptr;
        if (launch_track(P, tune, I0->dtype, st) != hipSuccess) return DGF_ERR_HIP;
        if (launch_gm_fit(g, st) != hipSuccess) return DGF_ERR_HIP;
        P.lstop = 0;
        P.gm_model = g.models;
        P.iters_out = iters_out;
        P.illum_out = illum_out;
    }
    return hip_rc(launch_track(P, tune, I0->dtype, st));
}

} // namespace dgf

extern "C" {

int dgf_track_run(const dgf_image *I0, const dgf_image *I1, const float *points, int64_t n, int32_t levels,
                  int32_t support, int32_t iters, const dgf_track_opts *opts, const void *workspace, size_t ws_bytes,
                  float *flow, uint8_t *status, int32_t *iters_out, float *illum_out, void *stream)
{
    dgf_track_opts o;
    const int rc = validate_track(I0, I1, points, n, levels, support, iters, opts, workspace, ws_bytes, flow, status, &o);
    if (rc != DGF_OK) return rc;
    if (illum_out && !(o.flags & DGF_TRACK_ILLUM)) return DGF_ERR_INVALID_ARG;
    return track_run_with(I0, I1, points, n, levels, support, iters, o, workspace, flow, status, iters_out,
                          tuning_for(support, levels, I0->dtype, n), (hipStream_t)stream, illum_out);
}

int dgf_track(const dgf_image *I0, const dgf_image *I1, const float *points, int64_t n, int32_t levels,
              int32_t support, int32_t iters, const dgf_track_opts *opts, void *workspace, size_t ws_bytes,
              float *flow, uint8_t *status, int32_t *iters_out, float *illum_out, void *stream)
{
    // validate everything first, so that an error launches nothing
    int rc = dgf_track_run(I0, I1, points, 0, levels, support, iters, opts, workspace, ws_bytes, flow, status,
                           iters_out, illum_out, stream);
    if (rc != DGF_OK) return rc;
    if (n < 0) return DGF_ERR_INVALID_ARG;
    if (n > 0 && (!points || !flow || !status)) return DGF_ERR_INVALID_ARG;
    if (n == 0) return DGF_OK;
    rc = dgf_track_pyramids(I0, I1, levels, workspace, ws_bytes, stream);
    if (rc != DGF_OK) return rc;
    return dgf_track_run(I0, I1, points, n, levels, support, iters, opts, workspace, ws_bytes, flow, status,
                         iters_out, illum_out, stream);
}

} // extern "C"
