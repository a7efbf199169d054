// dgf_internal.hpp -- device helpers and launch descriptors shared by the gfx950 kernels of the
// DeGraF detector / robust local flow tracker.  Internal to the HIP library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "degraf_flow.h"

namespace dgf {

// ------------------------------------------------------------------------------------------
// small device helpers
// ------------------------------------------------------------------------------------------

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Orders LDS writes and reads among the lanes of one wavefront.  LDS requests of one wave are
// served in issue order; the fences stop the compiler from moving accesses across this point.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ bool wave_any(bool p) { return __builtin_amdgcn_ballot_w64(p) != 0ull; }

template <int CTRL>
__device__ __forceinline__ float dpp(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}

__device__ __forceinline__ float readlane(float v, int l)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

// Sum of v over the LPP-lane group the calling lane belongs to (groups are aligned blocks of
// LPP lanes), returned to every lane of the group.  Must be called with all 64 lanes active.
// Rows of 16 lanes are reduced with DPP butterflies; rows are combined through readlane.
template <int LPP>
__device__ __forceinline__ float group_sum(float v)
{
    v += dpp<0xB1>(v);  // quad_perm [1,0,3,2]
    v += dpp<0x4E>(v);  // quad_perm [2,3,0,1]
    v += dpp<0x141>(v); // row_half_mirror
    v += dpp<0x140>(v); // row_mirror
    if constexpr (LPP == 16) {
        return v;
    } else {
        const float r0 = readlane(v, 0), r1 = readlane(v, 16), r2 = readlane(v, 32), r3 = readlane(v, 48);
        if constexpr (LPP == 32) {
            return (threadIdx.x & 32) ? (r2 + r3) : (r0 + r1);
        } else {
            return (r0 + r1) + (r2 + r3);
        }
    }
}

template <typename PixT>
__device__ __forceinline__ float load_px(const uint8_t *base, int64_t pitch, int x, int y)
{
    return (float)reinterpret_cast<const PixT *>(base + (int64_t)y * pitch)[x];
}

// ------------------------------------------------------------------------------------------
// launch descriptors
// ------------------------------------------------------------------------------------------

struct LevelPair {
    const uint8_t *p0; // I0 level (row 0)
    const uint8_t *p1; // I1 level (row 0)
    int64_t pitch0, pitch1;
    int32_t W, H;
};

struct TrackParams {
    LevelPair lv[DGF_MAX_LEVELS];
    const float *pts;
    int64_t n;
    float *flow;
    uint8_t *status;
    int32_t *iters_out;
    int32_t L, s, r, iters;
    int32_t ppl;         // pixel slots per lane actually used (ceil(s^2 / LPP))
    int32_t M;           // I1 tile margin, px on each side
    int32_t TW;          // I1 tile width = s + 1 + 2M
    int32_t RW;          // raw I0 tile width = s + 3
    int32_t tile_floats; // LDS floats per point = max(RW^2, TW^2)
    float invTW, invRW;
    float s1, s2, cmid;  // robust thresholds and sigma1 / (sigma2 - sigma1) (0 if unused)
    float eps2c, eps2f;  // squared stopping thresholds
    float min_eig_s2;    // min_eig * s^2
};

struct TrackTuning {
    int lpp;     // lanes per point: 16, 32 or 64
    int wpb;     // waves per workgroup: 1, 2, 4
    int margin;  // I1 tile margin M
};

struct PyrJob {
    const uint8_t *src;
    uint8_t *dst;
    int64_t src_pitch, dst_pitch;
    int32_t W, H; // source size; destination is ceil(W/2) x ceil(H/2)
};

// launchers (return hipSuccess or the launch error)
hipError_t launch_detect(const uint8_t *img, int64_t pitch, int W, int H, int win, int stride, float *pts,
                         uint8_t *sel, float *resp, hipStream_t st);
hipError_t launch_pyr_level(const PyrJob *jobs, int njobs, int dtype, hipStream_t st);
hipError_t launch_track(const TrackParams &P, const TrackTuning &T, int dtype, hipStream_t st);
int pick_ppl_max(int s, int lpp);
constexpr size_t kMaxLdsPerBlock = 64 * 1024;
// LDS bytes of one tracker workgroup for this support and launch shape
size_t track_lds_bytes(int s, const TrackTuning &T);
void fill_track_geometry(TrackParams &P, int s, int margin, int lpp);

} // namespace dgf
