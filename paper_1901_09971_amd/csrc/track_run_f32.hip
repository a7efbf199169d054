// track_run_f32.hip -- single-pair instantiations of the row-run tracker kernel for float images
// (batch plans: track_run_f32_batch.hip).
#include "track_run_kernel.hpp"

namespace dgf {

hipError_t launch_track_run_f32_batch(const TrackParams &P, int lpp, int s, int wpb, hipStream_t st);

hipError_t launch_track_run_f32(const TrackParams &P, int lpp, int s, int wpb, hipStream_t st)
{
    if (P.npairs) return launch_track_run_f32_batch(P, lpp, s, wpb, st);
#define DGF_CASE(L_, SEG_, R_, TP_, S_, X_)                                                                            \
    if (lpp == L_ && s == S_)                                                                                          \
        return P.illum ? launch_track_run_t<L_, SEG_, R_, TP_, S_, X_, true, false>(P, wpb, st)                            \
                       : launch_track_run_t<L_, SEG_, R_, TP_, S_, X_, false, false>(P, wpb, st);
    DGF_TRACK_RUN_SHAPES(DGF_CASE, float)
#undef DGF_CASE
    return hipErrorInvalidValue;
}

} // namespace dgf
