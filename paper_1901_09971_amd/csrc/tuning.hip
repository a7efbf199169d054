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
    t.lpp = px >= 200 ? 64 : (px >= 64 ? 32 : 16);
    t.wpb = 4;
    t.margin = 4;
    return t;
}

} // namespace

bool tuning_valid(const TrackTuning &t, int support)
{
    if (t.lpp != 16 && t.lpp != 32 && t.lpp != 64) return false;
    if (t.wpb != 1 && t.wpb != 2 && t.wpb != 4) return false;
    if (t.margin < 1 || t.margin > 16) return false;
    return pick_ppl_max(support, t.lpp) > 0;
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
    TrackTuning t;
    if (get_installed(support, dtype, &t)) return t;
    t = heuristic(support);
    // DGF_TUNE="lpp,wpb,margin" overrides the heuristic (launch-shape experiments)
    if (const char *env = getenv("DGF_TUNE")) {
        TrackTuning e = t;
        if (sscanf(env, "%d,%d,%d", &e.lpp, &e.wpb, &e.margin) == 3 && tuning_valid(e, support)) t = e;
    }
    if (!tuning_valid(t, support)) t.lpp = 64;
    return t;
}

void fill_track_constants(TrackParams &P, const dgf_track_opts &o, int support)
{
    P.s1 = o.sigma1;
    P.s2 = o.sigma2;
    P.cmid = (o.sigma2 > o.sigma1 && isfinite(o.sigma2)) ? o.sigma1 / (o.sigma2 - o.sigma1) : 0.0f;
    P.eps2c = o.eps_coarse * o.eps_coarse;
    P.eps2f = o.eps_fine * o.eps_fine;
    P.min_eig_s2 = o.min_eig * (float)(support * support);
}

} // namespace dgf
