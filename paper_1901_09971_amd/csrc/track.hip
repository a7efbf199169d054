// track.hip -- host side of the tracker: launch geometry, shape selection and dispatch to the
// kernel instantiations in track_u8.hip / track_f32.hip (generic kernel: track_kernel.hpp) and
// track_run_*.hip (row-run kernel: track_run_kernel.hpp).
#include "track_run_kernel.hpp"

namespace dgf {

hipError_t launch_track_u8(const TrackParams &P, int lpp, int ppl, int tp, int wpb, hipStream_t st);
hipError_t launch_track_f32(const TrackParams &P, int lpp, int ppl, int tp, int wpb, hipStream_t st);
// row-run instantiations, one file per (element type, cross-based supports, batch plan)
using RunLaunch = hipError_t (*)(const TrackParams &, int, int, int, hipStream_t);
hipError_t launch_track_run_u8(const TrackParams &P, int lpp, int s, int wpb, hipStream_t st);
hipError_t launch_track_run_u8_batch(const TrackParams &P, int lpp, int s, int wpb, hipStream_t st);
hipError_t launch_track_run_u8_cross(const TrackParams &P, int lpp, int s, int wpb, hipStream_t st);
hipError_t launch_track_run_u8_cross_batch(const TrackParams &P, int lpp, int s, int wpb, hipStream_t st);
hipError_t launch_track_run_f32(const TrackParams &P, int lpp, int s, int wpb, hipStream_t st);
hipError_t launch_track_run_f32_batch(const TrackParams &P, int lpp, int s, int wpb, hipStream_t st);
hipError_t launch_track_run_f32_cross(const TrackParams &P, int lpp, int s, int wpb, hipStream_t st);
hipError_t launch_track_run_f32_cross_batch(const TrackParams &P, int lpp, int s, int wpb, hipStream_t st);

bool run_shape_compiled(int lpp, int s)
{
#define DGF_HAS(L_, SEG_, R_, TP_, S_, X_)                                                                             \
    if (lpp == L_ && s == S_) return true;
    DGF_TRACK_RUN_SHAPES(DGF_HAS, float)
#undef DGF_HAS
    return false;
}

int run_shape_lanes(int s)
{
    for (int lpp : {64, 32, 16})
        if (run_shape_compiled(lpp, s)) return lpp;
    return 0;
}

TrackTuning illum_tuning(int s, TrackTuning t)
{
    if (t.kind != 0 || !run_shape_compiled(t.lpp, s)) {
        t.kind = 0;
        t.lpp = run_shape_lanes(s);
    }
    return t;
}

namespace {

bool shape_compiled(int lpp, int ppl, int tp)
{
#define DGF_HAS(L_, P_, T_, X_)                                                                                        \
    if (lpp == L_ && ppl == P_ && tp == T_) return true;
    DGF_TRACK_SHAPES(DGF_HAS, float)
#undef DGF_HAS
    return false;
}

} // namespace

int tile_pitch(int s) { return s <= 21 ? 32 : 64; }

// I1 tile pitch of a row-run shape (see DGF_TRACK_RUN_SHAPES)
int run_shape_pitch(int lpp, int s)
{
#define DGF_HAS(L_, SEG_, R_, TP_, S_, X_)                                                                             \
    if (lpp == L_ && s == S_) return TP_;
    DGF_TRACK_RUN_SHAPES(DGF_HAS, float)
#undef DGF_HAS
    return 0;
}

// Row pitch of the raw / resampled I0 tiles: s + 3, moved off multiples of 4 so that the rows
// touched by one wavefront land in different LDS banks.
int raw_pitch(int s)
{
    const int rw = s + 3;
    return (rw % 4 == 0) ? rw + 2 : rw;
}

int pick_ppl_max(int s, int lpp)
{
    const int ppl = (s * s + lpp - 1) / lpp;
    return shape_compiled(lpp, ppl, tile_pitch(s)) ? ppl : -1;
}

bool track_shape_ok(int s, const TrackTuning &T)
{
    if (T.kind == 0 && run_shape_compiled(T.lpp, s)) return true;
    return pick_ppl_max(s, T.lpp) > 0;
}

int clamp_margin(int s, int margin, int tp)
{
    const int mmax = (tp - s - 1) / 2;
    return margin < 1 ? 1 : (margin > mmax ? mmax : margin);
}

void fill_track_geometry(TrackParams &P, int s, int margin, int lpp, int kind)
{
    const int tp = (kind == 0 && run_shape_compiled(lpp, s)) ? run_shape_pitch(lpp, s) : tile_pitch(s);
    P.s = s;
    P.r = s / 2;
    P.M = clamp_margin(s, margin, tp);
    P.TW = s + 1 + 2 * P.M;
    P.RW = s + 3;
    P.RPP = raw_pitch(s);
    // raw patch, resampled (s + 2)^2 grid, and the cross-based support's arms (2 (s + 2) + 2 ints)
    const int tmpl = P.RW * P.RPP + (s + 2) * P.RPP + 2 * (s + 2) + 2;
    const int iter = P.TW * tp;
    P.tile_floats = tmpl > iter ? tmpl : iter;
    P.invBW = 1.0f / (float)(s + 2);
    P.ppl = (s * s + lpp - 1) / lpp;
}

size_t track_lds_bytes(int s, const TrackTuning &T)
{
    TrackParams P{};
    fill_track_geometry(P, s, T.margin, T.lpp, T.kind);
    return (size_t)T.wpb * (64 / T.lpp) * P.tile_floats * sizeof(float);
}

hipError_t launch_track(const TrackParams &P, const TrackTuning &T, int dtype, hipStream_t st)
{
    if (P.n <= 0) return hipSuccess;
    if (T.kind == 0 && run_shape_compiled(T.lpp, P.s)) {
        static const RunLaunch run[2][2][2] = {
            {{launch_track_run_u8, launch_track_run_u8_batch}, {launch_track_run_u8_cross, launch_track_run_u8_cross_batch}},
            {{launch_track_run_f32, launch_track_run_f32_batch},
             {launch_track_run_f32_cross, launch_track_run_f32_cross_batch}}};
        return run[dtype == DGF_U8 ? 0 : 1][P.cross ? 1 : 0][P.npairs ? 1 : 0](P, T.lpp, P.s, T.wpb, st);
    }
    const int tp = tile_pitch(P.s);
    if (!shape_compiled(T.lpp, P.ppl, tp)) return hipErrorInvalidValue;
    if (dtype == DGF_U8) return launch_track_u8(P, T.lpp, P.ppl, tp, T.wpb, st);
    return launch_track_f32(P, T.lpp, P.ppl, tp, T.wpb, st);
}

} // namespace dgf
