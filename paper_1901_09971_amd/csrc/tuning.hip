// tuning.hip -- tracker launch shapes: heuristic defaults plus a small table of entries that
// the autotuner (or the caller) installs per (support, dtype).
#include <math.h>
#include <mutex>
#include <stdio.h>
#include <stdlib.h>

#include "dgf_tuning.hpp"

namespace dgf {

namespace {

struct Entry {
    int support, dtype;
    TrackTuning t;
};

std::mutex g_mu;
Entry g_table[64];
int g_count = 0;

TrackTuning heuristic(int support)
{
    const int px = support * support;
    TrackTuning t;
    t.wpb = 1;
    t.margin = 2;
    t.kind = 0;
    if (run_shape_compiled(64, support)) {
        t.lpp = 64;
    } else if (run_shape_compiled(32, support)) {
        t.lpp = 32;
    } else if (run_shape_compiled(16, support)) {
        t.lpp = 16;
    } else {
        t.lpp = px >= 200 ? 64 : (px >= 64 ? 32 : 16);
    }
    return t;
}

} // namespace

bool tuning_valid(const TrackTuning &t, int support)
{
    if (t.lpp != 16 && t.lpp != 32 && t.lpp != 64) return false;
    if (t.wpb != 1 && t.wpb != 2 && t.wpb != 4) return false;
    if (t.margin < 1 || t.margin > 16) return false;
    if (t.kind != 0 && t.kind != 1) return false;
    return track_shape_ok(support, t);
}

void set_tuning(int support, int dtype, const TrackTuning &t)
{
    std::lock_guard<std::mutex> g(g_mu);
    for (int i = 0; i < g_count; ++i)
        if (g_table[i].support == support && g_table[i].dtype == dtype) {
            g_table[i].t = t;
            return;
        }
    if (g_count < 64) g_table[g_count++] = Entry{support, dtype, t};
}

bool get_installed(int support, int dtype, TrackTuning *out)
{
    std::lock_guard<std::mutex> g(g_mu);
    for (int i = 0; i < g_count; ++i)
        if (g_table[i].support == support && g_table[i].dtype == dtype) {
            *out = g_table[i].t;
            return true;
        }
    return false;
}

TrackTuning tuning_for(int support, int levels, int dtype, int64_t n)
{
    (void)levels;
    (void)n;
    // DGF_TUNE="lpp,wpb,margin[,kind]" takes precedence (launch-shape experiments and tests)
    if (const char *env = getenv("DGF_TUNE")) {
        TrackTuning e{0, 0, 0, 0};
        const int k = sscanf(env, "%d,%d,%d,%d", &e.lpp, &e.wpb, &e.margin, &e.kind);
        if (k >= 3 && tuning_valid(e, support)) return e;
    }
    TrackTuning t;
    if (get_installed(support, dtype, &t)) return t;
    t = heuristic(support);
    if (!tuning_valid(t, support)) {
        t.lpp = 64;
        t.kind = 1;
    }
    return t;
}

void fill_track_constants(TrackParams &P, const dgf_track_opts &o, int support)
{
    P.s1 = o.sigma1;
    P.s2 = o.sigma2;
    P.illum = (o.flags & DGF_TRACK_ILLUM) ? 1 : 0;
    if (isinf(o.sigma1)) {
        P.mode = ROBUST_L2; // |r| <= inf always: every weight is 1
        P.cmid = 0.0f;
    } else if (o.sigma1 > 0.f && o.sigma2 > o.sigma1 && isfinite(o.sigma2)) {
        P.mode = ROBUST_HAMPEL;
        P.cmid = o.sigma1 / (o.sigma2 - o.sigma1);
    } else {
        P.mode = ROBUST_HARD; // empty middle band, or sigma1 = 0 (psi is 0 off r = 0): w = 1 for |r| <= sigma1, else 0
        P.cmid = 0.0f;
    }
    P.cs2 = P.cmid * o.sigma2;
    P.eps2c = o.eps_coarse * o.eps_coarse;
    P.eps2f = o.eps_fine * o.eps_fine;
    P.min_eig_s2 = o.min_eig * (float)(support * support);
    P.min_eig = o.min_eig;
    P.cross = (o.flags & DGF_TRACK_CROSS) ? 1 : 0;
    P.tau = o.cross_tau;
    P.lstop = 0;
    P.gm_model = nullptr;
}

} // namespace dgf
