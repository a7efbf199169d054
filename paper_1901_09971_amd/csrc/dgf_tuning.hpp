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
void set_tuning(int support, int dtype, const TrackTuning &t);
bool get_installed(int support, int dtype, TrackTuning *out);

} // namespace dgf
