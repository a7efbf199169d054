// dgf_tuning.hpp -- launch-shape selection for the tracker (lanes per point, waves per
// workgroup, I1 tile margin) and the derived per-launch constants.
#pragma once

#include "dgf_internal.hpp"

namespace dgf {

// Tuning used for a (support, levels, dtype, n) request: an entry installed by the autotuner or
// by dgf_set_tuning for this support and dtype if there is one, else a shape heuristic.
TrackTuning tuning_for(int support, int levels, int dtype, int64_t n);

// Robust-norm and stopping constants of a launch, from the caller's options.
void fill_track_constants(TrackParams &P, const dgf_track_opts &o, int support);

bool tuning_valid(const TrackTuning &t, int support);

// Argument validation shared by the tracking entry points (fills the effective options), and
// tracking on already-built pyramids with an explicit launch shape.
int validate_track(const dgf_image *I0, const dgf_image *I1, const float *points, int64_t n, int32_t levels,
                   int32_t support, int32_t iters, const dgf_track_opts *opts, const void *workspace, size_t ws_bytes,
                   const float *flow, const uint8_t *status, dgf_track_opts *o);
// The same checks without the workspace (for dgf_track_static, whose pyramids need none).
int validate_track_args(const dgf_image *I0, const dgf_image *I1, const float *points, int64_t n, int32_t levels,
                        int32_t support, int32_t iters, const dgf_track_opts *opts, const float *flow,
                        const uint8_t *status, dgf_track_opts *o);
// Options in effect for a tracking call (defaults when opts is null), checked against the support.
int effective_track_opts(const dgf_track_opts *opts, int32_t support, dgf_track_opts *o);
int track_run_with(const dgf_image *I0, const dgf_image *I1, const float *points, int64_t n, int32_t levels,
                   int32_t support, int32_t iters, const dgf_track_opts &o, const void *workspace, float *flow,
                   uint8_t *status, int32_t *iters_out, TrackTuning tune, hipStream_t st, float *illum_out = nullptr);
void set_tuning(int support, int dtype, const TrackTuning &t);
GmFit gm_fit_for(const dgf_image *I0, int32_t levels, const void *workspace, const float *points,
                 const float *flow, const uint8_t *status, int64_t n);
bool get_installed(int support, int dtype, TrackTuning *out);

} // namespace dgf
