// track_run_u8_batch.hip -- batch-plan (persistent) instantiations of the row-run tracker kernel
// for uint8_t images.
#include "track_run_kernel.hpp"

namespace dgf {

hipError_t launch_track_run_u8_batch(const TrackParams &P, int lpp, int s, int wpb, hipStream_t st)
{
#define DGF_CASE(L_, SEG_, R_, TP_, S_, X_)                                                                            \
    if (lpp == L_ && s == S_)                                                                                          \
        return P.illum ? launch_track_run_t<L_, SEG_, R_, TP_, S_, X_, true, true>(P, wpb, st)                             \
                       : launch_track_run_t<L_, SEG_, R_, TP_, S_, X_, false, true>(P, wpb, st);
    DGF_TRACK_RUN_SHAPES(DGF_CASE, uint8_t)
#undef DGF_CASE
    return hipErrorInvalidValue;
}

} // namespace dgf
