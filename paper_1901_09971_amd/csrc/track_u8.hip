// track_u8.hip -- instantiations of the tracker kernel for uint8_t images (one translation unit per
// element type so the two sets compile in parallel).
#include "track_kernel.hpp"

namespace dgf {

hipError_t launch_track_u8(const TrackParams &P, int lpp, int ppl, int tp, int wpb, hipStream_t st)
{
#define DGF_CASE(L_, P_, T_, X_)                                                                                     \
    if (lpp == L_ && ppl == P_ && tp == T_) return launch_track_t<L_, P_, T_, X_>(P, wpb, st);
    DGF_TRACK_SHAPES(DGF_CASE, uint8_t)
#undef DGF_CASE
    return hipErrorInvalidValue;
}

} // namespace dgf
