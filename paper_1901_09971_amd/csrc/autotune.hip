// autotune.hip -- picks the tracker launch shape by timing every compiled candidate on the
// caller's own frames and points, installs the fastest for (support, element type), and keeps a
// small JSON cache so that later processes skip the search.
//
// Candidates: kernel kind (row-run layout where compiled for the support, else the generic slot
// layout) x lanes per point {16, 32, 64} x wavefronts per workgroup {1, 2, 4} x I1 tile margin
// {1, 2, 3, 4, 6}.  Every candidate computes the same result (the launch shape does not enter the
// arithmetic), so the search only changes speed.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <string>
#include <vector>

#include "dgf_internal.hpp"
#include "dgf_tuning.hpp"

using namespace dgf;

namespace {

std::string cache_key(int support, int levels, int dtype, int64_t n, int32_t flags)
{
    hipDeviceProp_t prop{};
    int dev = 0;
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        arch = prop.gcnArchName;
        const size_t c = arch.find(':');
        if (c != std::string::npos) arch = arch.substr(0, c);
    }
    int64_t bucket = 1;
    while (bucket < n) bucket <<= 1;
    char buf[160];
    snprintf(buf, sizeof buf, "%s:s%d:L%d:%s:n%lld%s%s%s", arch.c_str(), support, levels, dtype == DGF_U8 ? "u8" : "f32",
             (long long)bucket, (flags & DGF_TRACK_ILLUM) ? ":illum" : "", (flags & DGF_TRACK_CROSS) ? ":cross" : "",
             (flags & DGF_TRACK_GLOBAL) ? ":gm" : "");
    return buf;
}

struct CacheEntry {
    dgf_tuning t;
};

// The cache file holds one JSON object with one entry per line:
//   "gfx950:s21:L5:u8:n32768": {"lanes_per_point": 64, "waves_per_group": 1, "margin": 2, "kernel": 0, "ms": 0.3740},
std::map<std::string, dgf_tuning> read_cache(const char *path)
{
    std::map<std::string, dgf_tuning> m;
    FILE *f = fopen(path, "r");
    if (!f) return m;
    char line[512];
    while (fgets(line, sizeof line, f)) {
        char key[200];
        dgf_tuning t{};
        if (sscanf(line, " \"%199[^\"]\": {\"lanes_per_point\": %d, \"waves_per_group\": %d, \"margin\": %d, \"kernel\": %d, "
                         "\"ms\": %f}",
                   key, &t.lanes_per_point, &t.waves_per_group, &t.margin, &t.kernel, &t.ms) == 6)
            m[key] = t;
    }
    fclose(f);
    return m;
}

bool write_cache(const char *path, const std::map<std::string, dgf_tuning> &m)
{
    std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return false;
    fprintf(f, "{\n");
    size_t i = 0;
    for (const auto &kv : m) {
        const dgf_tuning &t = kv.second;
        fprintf(f, "  \"%s\": {\"lanes_per_point\": %d, \"waves_per_group\": %d, \"margin\": %d, \"kernel\": %d, \"ms\": %.4f}%s\n",
                kv.first.c_str(), t.lanes_per_point, t.waves_per_group, t.margin, t.kernel, t.ms,
                ++i < m.size() ? "," : "");
    }
    fprintf(f, "}\n");
    const bool ok = fclose(f) == 0;
    return ok && rename(tmp.c_str(), path) == 0;
}

TrackTuning to_internal(const dgf_tuning &t) { return TrackTuning{t.lanes_per_point, t.waves_per_group, t.margin, t.kernel}; }

dgf_tuning to_public(const TrackTuning &t, float ms) { return dgf_tuning{t.lpp, t.wpb, t.margin, t.kind, ms}; }

} // namespace

extern "C" {

int dgf_get_tuning(int32_t support, int32_t levels, int32_t dtype, int64_t n, dgf_tuning *out)
{
    if (!out || support < 1 || (support & 1) == 0 || support > DGF_MAX_SUPPORT) return DGF_ERR_INVALID_ARG;
    if (dtype != DGF_U8 && dtype != DGF_F32) return DGF_ERR_INVALID_ARG;
    *out = to_public(tuning_for(support, levels, dtype, n), -1.0f);
    return DGF_OK;
}

int dgf_set_tuning(int32_t support, int32_t dtype, const dgf_tuning *t)
{
    if (!t || support < 1 || (support & 1) == 0 || support > DGF_MAX_SUPPORT) return DGF_ERR_INVALID_ARG;
    if (dtype != DGF_U8 && dtype != DGF_F32) return DGF_ERR_INVALID_ARG;
    const TrackTuning tt = to_internal(*t);
    if (!tuning_valid(tt, support)) return DGF_ERR_UNSUPPORTED;
    set_tuning(support, dtype, tt);
    return DGF_OK;
}

int dgf_autotune(const dgf_image *I0, const dgf_image *I1, const float *points, int64_t n, int32_t levels,
                 int32_t support, int32_t iters, const dgf_track_opts *opts, void *workspace, size_t ws_bytes,
                 float *flow, uint8_t *status, const char *cache_path, dgf_tuning *out, void *stream)
{
    dgf_track_opts o;
    int rc = validate_track(I0, I1, points, n, levels, support, iters, opts, workspace, ws_bytes, flow, status, &o);
    if (rc != DGF_OK) return rc;
    if (n < 1) return DGF_ERR_INVALID_ARG;
    // the illumination model, cross-based supports and the global prior are cached under their own keys
    const std::string key = cache_key(support, levels, I0->dtype, n, o.flags);
    std::map<std::string, dgf_tuning> cache;
    if (cache_path) {
        cache = read_cache(cache_path);
        auto it = cache.find(key);
        if (it != cache.end() && tuning_valid(to_internal(it->second), support)) {
            // a cache hit installs the stored shape and still leaves what a timed call leaves:
            // the pyramids in the workspace and a tracking result made with that shape
            set_tuning(support, I0->dtype, to_internal(it->second));
            if (out) *out = it->second;
            rc = dgf_track_pyramids(I0, I1, levels, workspace, ws_bytes, stream);
            if (rc != DGF_OK) return rc;
            return track_run_with(I0, I1, points, n, levels, support, iters, o, workspace, flow, status, nullptr,
                                  to_internal(it->second), (hipStream_t)stream);
        }
    }
    hipStream_t st = (hipStream_t)stream;
    rc = dgf_track_pyramids(I0, I1, levels, workspace, ws_bytes, stream);
    if (rc != DGF_OK) return rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return DGF_ERR_HIP;
    std::vector<TrackTuning> cand;
    for (int kind = 0; kind <= 1; ++kind)
        for (int lpp : {16, 32, 64})
            for (int wpb : {1, 2, 4})
                for (int m : {1, 2, 3, 4, 6}) {
                    const TrackTuning t{lpp, wpb, m, kind};
                    if (kind == 0 && !run_shape_compiled(lpp, support)) continue;
                    if (kind == 1 && (o.flags & kRowRunFlags)) continue;
                    if (!tuning_valid(t, support) || track_lds_bytes(support, t) > kMaxLdsPerBlock) continue;
                    cand.push_back(t);
                }
    float best_ms = INFINITY;
    TrackTuning best = tuning_for(support, levels, I0->dtype, n);
    for (const TrackTuning &t : cand) {
        rc = track_run_with(I0, I1, points, n, levels, support, iters, o, workspace, flow, status, nullptr, t, st);
        if (rc != DGF_OK) break;
        (void)hipEventRecord(e0, st);
        for (int r = 0; r < 3; ++r) {
            rc = track_run_with(I0, I1, points, n, levels, support, iters, o, workspace, flow, status, nullptr, t, st);
            if (rc != DGF_OK) break;
        }
        (void)hipEventRecord(e1, st);
        if (rc != DGF_OK || hipEventSynchronize(e1) != hipSuccess) {
            rc = rc != DGF_OK ? rc : DGF_ERR_HIP;
            break;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        ms /= 3.0f;
        if (ms < best_ms) {
            best_ms = ms;
            best = t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != DGF_OK) return rc;
    set_tuning(support, I0->dtype, best);
    const dgf_tuning pub = to_public(best, best_ms);
    if (out) *out = pub;
    if (cache_path) {
        cache[key] = pub;
        write_cache(cache_path, cache); // a cache that cannot be written is not an error
    }
    return DGF_OK;
}

} // extern "C"
