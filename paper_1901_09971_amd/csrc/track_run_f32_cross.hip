// track_run_f32_cross.hip -- single-pair, cross-based-support instantiations of the row-run tracker
// kernel for float images (kernel: track_run_kernel.hpp; the other forms have files of their own,
// so that they compile in parallel).
#include "track_run_kernel.hpp"

namespace dgf {

DGF_DEFINE_TRACK_RUN_LAUNCH(launch_track_run_f32_cross, float, true, false)

} // namespace dgf
