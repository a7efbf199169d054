// track_run_u8_batch.hip -- batch-plan (persistent), square-window instantiations of the row-run
// tracker kernel for uint8_t images (kernel: track_run_kernel.hpp; the other forms have files of
// their own, so that they compile in parallel).
#include "track_run_kernel.hpp"

namespace dgf {

DGF_DEFINE_TRACK_RUN_LAUNCH(launch_track_run_u8_batch, uint8_t, false, true)

} // namespace dgf
