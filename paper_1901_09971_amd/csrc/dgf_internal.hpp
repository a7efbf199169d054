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
// Rows of 16 lanes are reduced with DPP butterflies; rows are then combined with the gfx950
// row-swap permutes (v_permlane16_swap / v_permlane32_swap), whose two outputs always add up to
// the pairwise row sums, so the result is independent of which rows the swap exchanges.
// One cross-row step of a group sum: after the 16-lane stage, LPP = 32 adds the partner row of
// each 32-lane half (v_permlane16_swap), LPP = 64 adds the other half (v_permlane32_swap).
template <int LPP>
__device__ __forceinline__ float group_sum_cross(float v)
{
    const unsigned u = __builtin_bit_cast(unsigned, v);
    if constexpr (LPP == 32) {
        const auto p = __builtin_amdgcn_permlane16_swap(u, u, false, false);
        return __builtin_bit_cast(float, (unsigned)p[0]) + __builtin_bit_cast(float, (unsigned)p[1]);
    } else {
        const auto p = __builtin_amdgcn_permlane32_swap(u, u, false, false);
        return __builtin_bit_cast(float, (unsigned)p[0]) + __builtin_bit_cast(float, (unsigned)p[1]);
    }
}

template <int LPP>
__device__ __forceinline__ float group_sum(float v)
{
    v += dpp<0xB1>(v);  // quad_perm [1,0,3,2]
    v += dpp<0x4E>(v);  // quad_perm [2,3,0,1]
    v += dpp<0x141>(v); // row_half_mirror
    v += dpp<0x140>(v); // row_mirror
    if constexpr (LPP >= 32) {
        const unsigned u = __builtin_bit_cast(unsigned, v);
        const auto p = __builtin_amdgcn_permlane16_swap(u, u, false, false);
        v = __builtin_bit_cast(float, (unsigned)p[0]) + __builtin_bit_cast(float, (unsigned)p[1]);
    }
    if constexpr (LPP == 64) {
        const unsigned u = __builtin_bit_cast(unsigned, v);
        const auto p = __builtin_amdgcn_permlane32_swap(u, u, false, false);
        v = __builtin_bit_cast(float, (unsigned)p[0]) + __builtin_bit_cast(float, (unsigned)p[1]);
    }
    return v;
}

// Bitwise OR of v over the LPP-lane group of the calling lane (the pattern of group_sum).  Must be
// called with all 64 lanes active.
template <int CTRL>
__device__ __forceinline__ unsigned dppu(unsigned v)
{
    return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}

template <int LPP>
__device__ __forceinline__ unsigned group_or(unsigned v)
{
    v |= dppu<0xB1>(v);
    v |= dppu<0x4E>(v);
    v |= dppu<0x141>(v);
    v |= dppu<0x140>(v);
    if constexpr (LPP >= 32) {
        const auto p = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        v = (unsigned)p[0] | (unsigned)p[1];
    }
    if constexpr (LPP == 64) {
        const auto p = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        v = (unsigned)p[0] | (unsigned)p[1];
    }
    return v;
}

// Sums of five values over all 64 lanes, returned wave-uniform.  Transposed reduction for four of
// them: the half- and row-swap permutes add two different values in one step (each half, then
// each row, keeps a different value), so one register remains for the in-row DPP butterflies.
// The fifth takes the in-row butterflies and then two row broadcasts (row 0 into row 1 and row
// 2 into row 3, then row 1 into rows 2 and 3), which leave its sum in lane 63.
__device__ __forceinline__ void wave_sum5(float &a, float &b, float &c, float &d, float &e)
{
    auto swap32 = [](float x, float y) {
        const auto p = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(unsigned, x), __builtin_bit_cast(unsigned, y),
                                                        false, false);
        return __builtin_bit_cast(float, (unsigned)p[0]) + __builtin_bit_cast(float, (unsigned)p[1]);
    };
    auto swap16 = [](float x, float y) {
        const auto p = __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(unsigned, x), __builtin_bit_cast(unsigned, y),
                                                        false, false);
        return __builtin_bit_cast(float, (unsigned)p[0]) + __builtin_bit_cast(float, (unsigned)p[1]);
    };
    // lanes 0-31 / 32-63 now hold half-sums of (a | d), (b | e)
    const float x1 = swap32(a, d), x2 = swap32(b, e);
    // rows 0..3 of y1 hold 16-lane partials of a, b, d, e
    float y1 = swap16(x1, x2), y2 = c;
    y1 += dpp<0xB1>(y1);
    y2 += dpp<0xB1>(y2);
    y1 += dpp<0x4E>(y1);
    y2 += dpp<0x4E>(y2);
    y1 += dpp<0x141>(y1);
    y2 += dpp<0x141>(y2);
    y1 += dpp<0x140>(y1);
    y2 += dpp<0x140>(y2);
    // rows 1 and 3 add lane 15 / 47 (row_bcast:15), rows 2 and 3 then lane 31 (row_bcast:31); the
    // other rows keep their value.  Written out because the compiler turns a DPP add on some rows
    // into a zeroed copy, a DPP move and an add.  The s_nops give the two wait states a DPP read
    // needs after a vector write of its source (also for a DPP read of the result after the
    // block, which the compiler's hazard check cannot see); the block touches registers only.
    asm("s_nop 1\n\t"
        "v_add_f32_dpp %0, %0, %0 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_add_f32_dpp %0, %0, %0 row_bcast:31 row_mask:0xc bank_mask:0xf\n\t"
        "s_nop 1"
        : "+v"(y2));
    a = readlane(y1, 0);
    b = readlane(y1, 16);
    d = readlane(y1, 32);
    e = readlane(y1, 48);
    c = readlane(y2, 63);
}

__device__ __forceinline__ bool wave_all(bool p) { return __builtin_amdgcn_ballot_w64(!p) == 0ull; }

// DeGraF centroid of one w x w window from its integer sums (Section 2 "Point detection", Eq. 1
// and 2): S = sum I, Mi = sum i I, Mj = sum j I (i row, j column within the window), m = max I.
// The negative weights 1 + m - I give S- = (1 + m) w^2 - S and moments (1 + m) w (w(w-1)/2) - M;
// the negative centroid is taken when S- > S.  (ox, oy) is the chosen centroid within the window,
// resp the distance between the two centroids.
struct DgfCentroid {
    float ox, oy, resp;
    bool neg;
};

__device__ __forceinline__ DgfCentroid degraf_centroid(int S, int Mi, int Mj, int m, int win)
{
    const int wh = win * win;
    const int mom = win * (win * (win - 1) / 2); // sum over the window of a row (or column) index
    const int S_neg = (1 + m) * wh - S;
    const int Mi_neg = (1 + m) * mom - Mi;
    const int Mj_neg = (1 + m) * mom - Mj;
    const bool neg = S_neg > S;
    const float cnx = (float)Mj_neg / (float)S_neg, cny = (float)Mi_neg / (float)S_neg;
    float cpx, cpy;
    if (S > 0) {
        cpx = (float)Mj / (float)S;
        cpy = (float)Mi / (float)S;
    } else {
        cpx = 0.5f * (float)(win - 1);
        cpy = cpx;
    }
    DgfCentroid d;
    d.ox = neg ? cnx : cpx;
    d.oy = neg ? cny : cpy;
    d.neg = neg;
    d.resp = sqrtf((cpx - cnx) * (cpx - cnx) + (cpy - cny) * (cpy - cny));
    return d;
}

// Lane layout for staging a rectangle `cols` floats wide with the LPP lanes of one point.  With
// cols <= LPP, rpp = LPP / cols rows go per pass and lane li keeps column c = li mod cols of row
// r0 = li / cols (lanes with r0 >= rpp stay idle); a wider rectangle takes one row per pass and
// lane li keeps columns li, li + LPP, ...  `cols` is a launch constant, so this runs once per
// launch.
struct StageLanes {
    int rpp, r0, c;
    int li;
};

template <int LPP>
__device__ __forceinline__ StageLanes stage_lanes(int cols, int li)
{
    StageLanes sl;
    if (cols <= LPP) {
        sl.rpp = LPP / cols;
        sl.r0 = li / cols;
        sl.c = li - sl.r0 * cols;
    } else {
        sl.rpp = 1;
        sl.r0 = 0;
        sl.c = li;
    }
    sl.li = li;
    return sl;
}

// Copies the rows x cols rectangle of a level image whose top-left pixel is (ox, oy) into LDS
// (row pitch lp floats), replicating the image border.  Every address is clamped into the image,
// so the loads run unpredicated and kStageBatch of them are in flight before the first LDS write;
// only the writes check the row count.  Byte offsets are 24-bit row x pitch products in 32 bits
// off a scalar global base: the host rejects pitches of 2^24 bytes or more and images of 2 GiB or
// more.
//
// A uint8 rectangle at most 32 texels wide that lies inside the image with three columns to spare
// on the left and four on the right (no border to replicate) goes four texels per lane: eight
// lanes per row, lane li keeping columns 4 (li mod 8) .. + 3 of row li / 8 of each pass; two
// aligned dword loads per lane cut out its four bytes with v_alignbyte (rows need not be dword
// aligned), and kStageBatch4 passes' loads are in flight before the first write.  Every byte those
// loads touch lies on an image row between columns ox - 3 and ox + 4 ceil(cols / 4) + 3.
constexpr int kStageBatch = 2;
constexpr int kStageBatch4 = 2;

template <int LPP, typename PixT>
__device__ __forceinline__ void stage_rect(float *lds, int lp, const uint8_t *base, int64_t pitch, int W, int H, int ox,
                                           int oy, int rows, int cols, const StageLanes &sl)
{
    typedef const __attribute__((address_space(1))) uint8_t gbyte;
    typedef const __attribute__((address_space(1))) uint32_t gword;
    gbyte *gb = (gbyte *)base;
    const uint32_t pb = (uint32_t)pitch, hm1 = (uint32_t)(H - 1);
    if constexpr (sizeof(PixT) == 1) {
        constexpr int rpp4 = LPP / 8;
        if (cols <= 32 && ox >= 3 && oy >= 0 && ox + 4 * ((cols + 3) >> 2) + 4 <= W && oy + rows <= H) {
            const int r04 = sl.li >> 3, c4 = (sl.li & 7) << 2;
            if (c4 >= cols) return;
            const uint32_t mis = (uint32_t)(uintptr_t)base & 3u, cx = (uint32_t)(ox + c4);
            const bool full = c4 + 4 <= cols;
            for (int y0 = r04; y0 < rows; y0 += kStageBatch4 * rpp4) {
                uint32_t lo[kStageBatch4], hi[kStageBatch4], sh[kStageBatch4];
#pragma unroll
                for (int k = 0; k < kStageBatch4; ++k) {
                    const int y = min(y0 + k * rpp4, rows - 1);
                    const uint32_t off = __umul24((uint32_t)(oy + y), pb) + cx;
                    sh[k] = (off + mis) & 3u;
                    gword *p = (gword *)(gb + (off - sh[k]));
                    lo[k] = p[0];
                    hi[k] = p[1];
                }
#pragma unroll
                for (int k = 0; k < kStageBatch4; ++k) {
                    const int y = y0 + k * rpp4;
                    if (y < rows) {
                        const uint32_t v = __builtin_amdgcn_alignbyte(hi[k], lo[k], sh[k]);
                        float *d = lds + y * lp + c4;
                        const float f0 = (float)(v & 255u), f1 = (float)((v >> 8) & 255u),
                                    f2 = (float)((v >> 16) & 255u), f3 = (float)(v >> 24);
                        if (full) {
                            d[0] = f0;
                            d[1] = f1;
                            d[2] = f2;
                            d[3] = f3;
                        } else {
                            d[0] = f0;
                            if (c4 + 1 < cols) d[1] = f1;
                            if (c4 + 2 < cols) d[2] = f2;
                        }
                    }
                }
            }
            return;
        }
    }
    if (sl.r0 >= sl.rpp) return;
    for (int c = sl.c; c < cols; c += LPP) { // a single pass when cols <= LPP
        const uint32_t cx = (uint32_t)clampi(ox + c, 0, W - 1) * (uint32_t)sizeof(PixT);
        for (int y0 = sl.r0; y0 < rows; y0 += kStageBatch * sl.rpp) {
            float v[kStageBatch];
#pragma unroll
            for (int k = 0; k < kStageBatch; ++k) {
                const uint32_t cy = min((uint32_t)max(oy + y0 + k * sl.rpp, 0), hm1);
                v[k] = (float)*reinterpret_cast<const __attribute__((address_space(1))) PixT *>(gb + (__umul24(cy, pb) + cx));
            }
#pragma unroll
            for (int k = 0; k < kStageBatch; ++k) {
                const int y = y0 + k * sl.rpp;
                if (y < rows) lds[y * lp + c] = v[k];
            }
        }
    }
}

// Steps of stage_u8_w64 (below) for one lane: NS steps of 8 rows from byte offset a0 (aligned)
// with shift sh off the aligned base gb, B steps' loads in flight.  WHOLE: every group writes
// all four words (the row's last group fits the LDS row); otherwise the row's last group writes
// only the words it owns.
template <int NS, int B, bool EXACT, bool WHOLE>
__device__ __forceinline__ void stage_u8_w64_steps(float *lds, int lp, const __attribute__((address_space(1))) uint8_t *gb,
                                                   uint32_t pb, uint32_t a0, uint32_t alast, uint32_t sh, int r0,
                                                   int c4, int rows, int cols)
{
    typedef const __attribute__((address_space(1))) uint32_t gword;
#pragma unroll
    for (int k0 = 0; k0 < NS; k0 += B) {
        uint32_t lo[B], hi[B];
#pragma unroll
        for (int k = k0; k < k0 + B && k < NS; ++k) {
            uint32_t a = a0 + (uint32_t)(8 * k) * pb;
            if (!EXACT) a = min(a, alast);
            gword *p = (gword *)(gb + a);
            lo[k - k0] = p[0];
            hi[k - k0] = p[1];
        }
#pragma unroll
        for (int k = k0; k < k0 + B && k < NS; ++k) {
            if (EXACT || r0 + 8 * k < rows) {
                const uint32_t v = __builtin_amdgcn_alignbyte(hi[k - k0], lo[k - k0], sh);
                float *d = lds + (r0 + 8 * k) * lp + c4;
                const float f0 = (float)(v & 255u), f1 = (float)((v >> 8) & 255u), f2 = (float)((v >> 16) & 255u),
                            f3 = (float)(v >> 24);
                if (WHOLE || c4 + 4 <= cols) {
                    d[0] = f0;
                    d[1] = f1;
                    d[2] = f2;
                    d[3] = f3;
                } else {
                    d[0] = f0;
                    if (c4 + 1 < cols) d[1] = f1;
                    if (c4 + 2 < cols) d[2] = f2;
                }
            }
        }
    }
}

// stage_rect's interior case for a rectangle staged by a whole wavefront (64 lanes) from a uint8
// image: the same values, with the steps unrolled.  Qualifies when rows <= 8 NS, cols <= 32 and
// the rectangle lies inside the image with every row's dword pairs inside the row (stage_rect's
// own interior test); returns false, staging nothing, otherwise.  Eight lanes per row, four bytes
// per lane, row r0 + 8 k in step k.  The base pointer is moved back to a 4-byte boundary once;
// 8 k rows further on the byte shift is the same (8 pitch is a multiple of 4), so a step costs an
// offset add, one v_alignbyte and four conversions.  The loads are unpredicated and go out B steps
// at a time, all of a batch before its first LDS write: a step past the rectangle's last row loads
// that row again and writes nothing.  When the row's last group of four fits the LDS row pitch it
// writes all four words (the extra ones land in the row's padding, which no reader looks at).
// CROWS = 8 NS tells that rows always equals it (no clamp, no write test).
template <int NS, int B, int CROWS = 0>
__device__ __forceinline__ bool stage_u8_w64(float *lds, int lp, const uint8_t *base, int64_t pitch, int W, int H,
                                             int ox, int oy, int rows, int cols, int li)
{
    constexpr bool exact = CROWS == 8 * NS;
    if (!(rows <= 8 * NS && cols <= 32 && ox >= 3 && oy >= 0 && ox + 4 * ((cols + 3) >> 2) + 4 <= W && oy + rows <= H))
        return false;
    typedef const __attribute__((address_space(1))) uint8_t gbyte;
    const int r0 = li >> 3, c4 = (li & 7) << 2;
    if (c4 >= cols || r0 >= rows) return true;
    const uint32_t mis = (uint32_t)(uintptr_t)base & 3u;
    gbyte *gb = (gbyte *)(base - mis); // 4-byte aligned
    const uint32_t pb = (uint32_t)pitch;
    // byte offset of the lane's first pixel off the aligned base (step 0), its shift and the
    // aligned offset; then the aligned offset of the lane's pixel in the rectangle's last row
    const uint32_t o0 = __umul24((uint32_t)(oy + r0), pb) + (uint32_t)(ox + c4) + mis;
    const uint32_t sh = o0 & 3u, a0 = o0 - sh;
    const uint32_t alast = exact ? 0u : a0 + __umul24((uint32_t)(rows - 1 - r0), pb);
    if (4 * ((cols + 3) >> 2) <= lp)
        stage_u8_w64_steps<NS, B, exact, true>(lds, lp, gb, pb, a0, alast, sh, r0, c4, rows, cols);
    else
        stage_u8_w64_steps<NS, B, exact, false>(lds, lp, gb, pb, a0, alast, sh, r0, c4, rows, cols);
    return true;
}

// i / d for 0 <= i < 2^16 and 1 <= d < 2^8, with inv = 1 / d: (i + 1/2) / d is at least 1 / (2 d)
// away from the next integer and the float product errs by far less, so the truncation is exact.
__device__ __forceinline__ int div_small(int i, float inv) { return (int)(((float)i + 0.5f) * inv); }

// Block-wide copy of the w x h byte rectangle whose top-left pixel is (x, y) of a uint8 image
// (row pitch `pitch` bytes, width W; the rectangle lies inside the image) into LDS with row pitch
// lp, a multiple of 4 at least 4 ceil(w / 4), from a 4-byte aligned base.  Four bytes per lane
// and step, from two aligned dwords of the image row cut by v_alignbyte; kB steps' loads are
// issued before the first LDS write.  A group whose dword pair would leave the row loads an
// in-row pair instead (branch-free, so no load waits on another) and is redone byte by byte
// afterwards; rows narrower than 11 bytes go byte by byte throughout.  Bytes w .. 4 ceil(w / 4) - 1
// of an LDS row receive copies of row bytes (clamped).
template <int kB>
__device__ __forceinline__ void stage_u8_block(uint8_t *lds, int lp, const uint8_t *img, int64_t pitch, int W, int x,
                                              int y, int w, int h)
{
    typedef const __attribute__((address_space(1))) uint8_t gbyte;
    typedef const __attribute__((address_space(1))) uint32_t gword;
    const int n4 = (w + 3) >> 2, G = n4 * h, nt = (int)blockDim.x;
    const float inv = 1.0f / (float)n4;
    const uint32_t mis = (uint32_t)(uintptr_t)img & 3u;
    gbyte *gb = (gbyte *)img;
    auto bytes = [&](int64_t row, int c) {
        uint32_t t = 0u;
#pragma unroll
        for (int b = 0; b < 4; ++b) t |= (uint32_t)gb[row + min(x + c + b, W - 1)] << (8 * b);
        return t;
    };
    if (W < 11) {
        for (int g = (int)threadIdx.x; g < G; g += nt) {
            const int r = div_small(g, inv), c = 4 * (g - r * n4);
            *reinterpret_cast<uint32_t *>(lds + r * lp + c) = bytes((int64_t)(y + r) * pitch, c);
        }
        return;
    }
    for (int g0 = (int)threadIdx.x; g0 < G; g0 += kB * nt) {
        uint32_t lo[kB], hi[kB], sh[kB];
        unsigned edge = 0u;
#pragma unroll
        for (int k = 0; k < kB; ++k) {
            const int g = min(g0 + k * nt, G - 1);
            const int r = div_small(g, inv), c = 4 * (g - r * n4);
            const int64_t row = (int64_t)(y + r) * pitch;
            const int s = (int)((row + x + c + mis) & 3);
            int a = x + c - s; // image column of the first aligned dword: a is in [-3, W - 1]
            const bool fits = a >= 0 && a + 8 <= W;
            // else the nearest aligned pair inside the row (one exists when W >= 11)
            a = a < 0 ? a + 4 : a;
            a = a + 8 > W ? a - 4 * ((a + 11 - W) >> 2) : a;
            gword *p = (gword *)(gb + (row + a));
            lo[k] = p[0];
            hi[k] = p[1];
            sh[k] = (uint32_t)s;
            edge |= (fits ? 0u : 1u) << k;
        }
#pragma unroll
        for (int k = 0; k < kB; ++k) {
            const int g = g0 + k * nt;
            if (g < G) {
                const int r = div_small(g, inv), c = 4 * (g - r * n4);
                *reinterpret_cast<uint32_t *>(lds + r * lp + c) = __builtin_amdgcn_alignbyte(hi[k], lo[k], sh[k]);
            }
        }
        if (edge) {
#pragma unroll
            for (int k = 0; k < kB; ++k) {
                const int g = g0 + k * nt;
                if (g < G && ((edge >> k) & 1u)) {
                    const int r = div_small(g, inv), c = 4 * (g - r * n4);
                    *reinterpret_cast<uint32_t *>(lds + r * lp + c) = bytes((int64_t)(y + r) * pitch, c);
                }
            }
        }
    }
}

// ---- detection tiles (shared by the detection launches and the fused front-end launch) -------

struct DetectOut {
    float *pts;
    uint8_t *sel;
    float *resp;
};

__device__ __forceinline__ void finish_window(int S, int Mi, int Mj, int m, int win, int x0, int y0, int64_t n,
                                              DetectOut o)
{
    const DgfCentroid d = degraf_centroid(S, Mi, Mj, m, win);
    reinterpret_cast<float2 *>(o.pts)[n] = make_float2((float)x0 + d.ox, (float)y0 + d.oy);
    if (o.sel) o.sel[n] = (uint8_t)d.neg;
    if (o.resp) o.resp[n] = d.resp;
}

// LDS-tiled form: TX x TY windows per workgroup (tile (tile_x, tile_y) of the window grid), one
// lane per window, the covered pixels staged in `tile` (row pitch rounded up to 4 bytes, 4-byte
// aligned).  n0 offsets the output (batched form: points of a pair start at its offset in the
// concatenated output).
template <int TX, int TY>
__device__ __forceinline__ void detect_tile(uint8_t *tile, int tile_x, int tile_y, const uint8_t *__restrict__ img,
                                            int64_t pitch, int W, int H, int win, int stride, int nx, int ny, int64_t n0,
                                            DetectOut o)
{
    const int wx0 = tile_x * TX, wy0 = tile_y * TY;
    const int ox = wx0 * stride, oy = wy0 * stride;
    const int RW = (TX - 1) * stride + win, RH = (TY - 1) * stride + win, RP = (RW + 3) & ~3;
    const int rw = min(RW, W - ox), rh = min(RH, H - oy);
    stage_u8_block<4>(tile, RP, img, pitch, W, ox, oy, rw, rh);
    __syncthreads();
    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    const int kx = wx0 + tx, ky = wy0 + ty;
    if (ty >= TY || kx >= nx || ky >= ny) return; // (blocks may have more lanes than windows)
    const uint8_t *w0 = tile + ty * stride * RP + tx * stride;
    int S = 0, Mi = 0, Mj = 0, m = 0;
    for (int i = 0; i < win; ++i) {
        int rs = 0, rj = 0;
        for (int j = 0; j < win; ++j) {
            const int v = w0[i * RP + j];
            rs += v;
            rj += j * v;
            m = max(m, v);
        }
        S += rs;
        Mi += i * rs;
        Mj += rj;
    }
    finish_window(S, Mi, Mj, m, win, kx * stride, ky * stride, n0 + (int64_t)ky * nx + kx, o);
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
    float *illum_out;    // illumination model: (m, c) per point (nullable)
    int32_t L, s, r, iters;
    int32_t ppl;         // pixel slots per lane actually used (ceil(s^2 / LPP))
    int32_t M;           // I1 tile margin, px on each side
    int32_t TW;          // I1 tile width = s + 1 + 2M (row pitch in LDS: the kernel's TP)
    int32_t RW;          // raw I0 tile width = s + 3
    int32_t RPP;         // LDS row pitch of the raw / resampled I0 tiles (>= RW, chosen to spread banks)
    int32_t tile_floats; // LDS floats per point = max(RW RPP + (s+2) RPP, TW * TP)
    float invBW;         // 1 / (s + 2)
    int32_t mode;        // ROBUST_L2, ROBUST_HAMPEL or ROBUST_HARD
    int32_t illum;       // 1: gain / offset illumination model (4x4 system per iteration)
    float s1, s2, cmid;  // robust thresholds and sigma1 / (sigma2 - sigma1) (0 if unused)
    float cs2;           // cmid * sigma2
    float eps2c, eps2f;  // squared stopping thresholds
    float min_eig_s2;    // min_eig * s^2
    float min_eig;       // per support pixel (cross-based supports divide by their own size)
    int32_t cross;       // 1: adaptive cross-based supports with threshold tau
    float tau;
    int32_t lstop;       // last (finest) level run: 0, or L - 1 for the global prior's first pass
    const double *gm_model; // nullable: global affine motion per pair, [npairs or 1][6], starts the coarsest level
    // batched form (npairs = 0 for a single pair): per-pair level table, prefix sums of per-pair
    // work items (groups of points of one pair handled by one wavefront) and of per-pair points
    int32_t npairs;
    int32_t persistent;  // 1: waves pull items from the per-XCD counters until all ranges are drained
    const LevelPair *blv; // [npairs][L]
    const int64_t *item_off, *pt_off; // [npairs + 1] each
    uint32_t *counter;
    int64_t nitems;
    int64_t grid_waves; // batched form: wavefronts to launch (persistent: a resident-sized grid)
};

// One wavefront's unit of work: a group of up to 64 / LPP consecutive points of one pair.
struct WorkItem {
    int64_t pidx; // global point index of this lane's point
    int pair;
    bool valid;   // this lane's point exists
    bool done;    // no work left for the wavefront
};

template <int PPW, bool BATCH = true>
__device__ __forceinline__ WorkItem work_item(const TrackParams &P, int64_t item, int q)
{
    WorkItem w;
    if (!BATCH || P.npairs == 0) {
        w.done = item * PPW >= P.n;
        w.pair = 0;
        // last point first: in the detector's row-major order that issues the bottom image rows
        // first, which in a forward-moving camera's view hold the nearest scene, the largest
        // motions and the points that run out of iterations; started early, they no longer
        // form the launch's tail (12 % shorter on the 1242x375 driving pair, outputs identical)
        const int64_t rr = item * PPW + q;
        w.valid = rr < P.n;
        w.pidx = w.valid ? P.n - 1 - rr : 0;
        return w;
    }
    w.done = item >= P.nitems;
    w.pair = 0;
    w.pidx = 0;
    w.valid = false;
    if (w.done) return w;
    int lo = 0, hi = P.npairs - 1; // last pair whose first item is <= item
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (P.item_off[mid] <= item)
            lo = mid;
        else
            hi = mid - 1;
    }
    const int64_t local = (item - P.item_off[lo]) * PPW + q;
    w.pair = lo;
    w.valid = local < P.pt_off[lo + 1] - P.pt_off[lo];
    w.pidx = P.pt_off[lo] + local;
    return w;
}

// The hardware hands the blocks of a launch to the eight XCDs in turn (block b runs on XCD b mod 8)
// and every XCD has an L2 of its own.
constexpr int kNumXcd = 8;

// Plain row-run launches hand each XCD runs of kXcdRun consecutive points: the blocks of XCD x
// take runs x, x + 8, x + 16, ... in their launch order, so a point's flow and status lines are
// written back from one L2 rather than from up to eight, and the launch order still takes the
// points from the last one back in steps of 8 kXcdRun.  The grid is a whole number of such groups
// of 8 runs (plain_blocks); waves past the last point find nothing to do.  PPW points per wave,
// wpb waves per block, both powers of two with wpb PPW <= kXcdRun.
constexpr int kXcdRun = 64;

template <int PPW>
__device__ __forceinline__ int64_t plain_item(unsigned b, int wave, int wpb)
{
    const int ppb = wpb * PPW;                         // points per block
    const int kb_log = __builtin_ctz(kXcdRun / ppb);    // blocks per run, log2
    const unsigned x = b % kNumXcd, j = b / kNumXcd;    // XCD, and the block's rank on it
    const int64_t run = (int64_t)(j >> kb_log) * kNumXcd + x;
    return (run * kXcdRun + (int64_t)(j & ((1u << kb_log) - 1)) * ppb) / PPW + wave;
}

inline int64_t plain_blocks(int64_t blocks, int wpb, int ppw)
{
    const int64_t group = (int64_t)kNumXcd * (kXcdRun / (wpb * ppw));
    return (blocks + group - 1) / group * group;
}

// Persistent form: the items are split into kNumXcd contiguous ranges, one per XCD, each with a
// counter of its own (kCounterStride words apart, so they sit in different cache lines).  A
// wavefront takes items from the range of the XCD it runs on and, once that range is drained, from
// the next ones in turn; it leaves after all of them are.  Every wavefront therefore ends after at
// most (its items + kNumXcd) counter bumps, and every item is handed out exactly once.  `visit` is
// wavefront-uniform (all lanes take lane 0's counter value).
constexpr int kCounterStride = 64;

__device__ __forceinline__ int64_t next_item(const TrackParams &P, int home, int &visit)
{
    while (visit < kNumXcd) {
        const int k = (home + visit) % kNumXcd;
        const int64_t lo = P.nitems * k / kNumXcd, hi = P.nitems * (k + 1) / kNumXcd;
        unsigned v = 0u;
        if ((threadIdx.x & 63) == 0) v = atomicAdd(P.counter + (size_t)k * kCounterStride, 1u);
        const int64_t item = lo + (int64_t)__builtin_amdgcn_readfirstlane(v);
        if (item < hi) return item;
        ++visit;
    }
    return P.nitems;
}

__device__ __forceinline__ uint32_t uniform_u32(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }

__device__ __forceinline__ uint64_t uniform_u64(uint64_t v)
{
    return (uint64_t)uniform_u32((uint32_t)v) | ((uint64_t)uniform_u32((uint32_t)(v >> 32)) << 32);
}

// Level descriptors of the pair a wavefront works on.  The value is the same in every lane; the
// readfirstlanes tell the compiler so, and keep base pointers and sizes in scalar registers (the
// table is read through a generic pointer, kernel argument or device memory, which it cannot
// prove uniform on its own).
template <bool BATCH = true>
__device__ __forceinline__ LevelPair level_of(const TrackParams &P, int pair, int l)
{
    const LevelPair v = (BATCH && P.npairs) ? P.blv[pair * P.L + l] : P.lv[l];
    LevelPair u;
    u.p0 = reinterpret_cast<const uint8_t *>(uniform_u64(reinterpret_cast<uint64_t>(v.p0)));
    u.p1 = reinterpret_cast<const uint8_t *>(uniform_u64(reinterpret_cast<uint64_t>(v.p1)));
    u.pitch0 = (int64_t)uniform_u64((uint64_t)v.pitch0);
    u.pitch1 = (int64_t)uniform_u64((uint64_t)v.pitch1);
    u.W = (int)uniform_u32((uint32_t)v.W);
    u.H = (int)uniform_u32((uint32_t)v.H);
    return u;
}

// How the robust weight w = psi(r)/r is evaluated (chosen on the host from sigma1, sigma2):
//   ROBUST_L2     both thresholds infinite: w = 1 everywhere (plain least squares)
//   ROBUST_HAMPEL 0 < sigma1 < sigma2 finite: w = hampel_weight(r) below
//   ROBUST_HARD   sigma1 >= sigma2, or sigma1 = 0: w = 1 for |r| <= sigma1, else 0
enum { ROBUST_L2 = 0, ROBUST_HAMPEL = 1, ROBUST_HARD = 2 };

// Symmetric 4x4 system M x = v by an LDL^T factorisation; m holds the upper triangle row by row
// (m00 m01 m02 m03 m11 m12 m13 m22 m23 m33).  Returns det M (the product of the pivots); when a
// pivot is not positive, x is not finite.  x may be null (determinant only).
__device__ __forceinline__ float ldl4(const float *m, const float *v, float *x)
{
    const float d0 = m[0];
    const float i0 = __builtin_amdgcn_rcpf(d0);
    const float l10 = m[1] * i0, l20 = m[2] * i0, l30 = m[3] * i0;
    const float d1 = fmaf(-l10, m[1], m[4]);
    const float i1 = __builtin_amdgcn_rcpf(d1);
    const float l21 = fmaf(-l20, m[1], m[5]) * i1, l31 = fmaf(-l30, m[1], m[6]) * i1;
    const float d2 = fmaf(-l21 * l21, d1, fmaf(-l20, m[2], m[7]));
    const float i2 = __builtin_amdgcn_rcpf(d2);
    const float l32 = fmaf(-l31 * l21, d1, fmaf(-l30, m[2], m[8])) * i2;
    const float d3 = fmaf(-l32 * l32, d2, fmaf(-l31 * l31, d1, fmaf(-l30, m[3], m[9])));
    const float i3 = __builtin_amdgcn_rcpf(d3);
    if (x) {
        const bool ok = d0 > 0.f && d1 > 0.f && d2 > 0.f && d3 > 0.f;
        const float y0 = v[0], y1 = fmaf(-l10, y0, v[1]), y2 = fmaf(-l21, y1, fmaf(-l20, y0, v[2]));
        const float y3 = fmaf(-l32, y2, fmaf(-l31, y1, fmaf(-l30, y0, v[3])));
        const float x3 = y3 * i3, x2 = fmaf(-l32, x3, y2 * i2);
        const float x1 = fmaf(-l31, x3, fmaf(-l21, x2, y1 * i1));
        const float x0 = fmaf(-l30, x3, fmaf(-l20, x2, fmaf(-l10, x1, y0 * i0)));
        const float bad = __builtin_nanf("");
        x[0] = ok ? x0 : bad;
        x[1] = ok ? x1 : bad;
        x[2] = ok ? x2 : bad;
        x[3] = ok ? x3 : bad;
    }
    return d0 * d1 * d2 * d3;
}

// IRLS weight of the middle-band norm, psi(r) / r = clamp(cs2 / |r| - cmid, 0, 1) with
// cmid = sigma1 / (sigma2 - sigma1) and cs2 = cmid sigma2: exactly 1 over the inner band
// (cs2 / sigma1 - cmid = 1), falling to 0 at sigma2.  At r = 0 the reciprocal is infinite and the
// clamp gives the limit 1.  Needs sigma1 > 0 (otherwise cs2 = 0 and 0 * inf is undefined).
__device__ __forceinline__ float hampel_weight(float r, float cs2, float cmid)
{
    return __builtin_amdgcn_fmed3f(fmaf(cs2, __builtin_amdgcn_rcpf(fabsf(r)), -cmid), 0.f, 1.f);
}

// Level-0 frames of one pair and where its gradient maps live: dI0 = grad0 + g0 and
// dI1 = grad1 + g1 (the kernel's base pointers), row pitch gpitch floats.
struct AdjPair {
    const uint8_t *I0, *I1;
    int64_t pitch0, pitch1; // bytes
    int64_t g0, g1;         // float offsets of the two gradient maps
    int64_t gpitch0, gpitch1;
    int32_t W, H;
};

struct AdjParams {
    AdjPair one;           // single-pair form (npairs == 0)
    const AdjPair *pairs;  // batched form: per-pair table (device)
    const int64_t *pt_off; // batched form: first point of each pair, npairs + 1 entries (device)
    int32_t npairs;
    float *grad0, *grad1;  // gradient base pointers
    int32_t s, r;
    const float *pts, *flow, *dflow;
    const uint8_t *status;
    float *dpoints;        // nullable: dL/dp per point (written)
    const float *illum;    // illumination model: (m, c) per point from the forward pass, else null
    int64_t n;
    float s1, s2, dpsi_mid; // thresholds and the middle-band slope -sigma1 / (sigma2 - sigma1)
    int32_t mode;
    int64_t perm_mul;       // block b takes point (b perm_mul) mod n; set by the launch
};

struct DetectGradParams {
    const uint8_t *img;
    int64_t pitch;
    int32_t W, H, win, stride, nx;
    const uint8_t *sel;
    const float *dpoints;
    float *dI;
    int64_t dpitch; // floats
    int64_t n;
};
hipError_t launch_detect_backward(const DetectGradParams &G, hipStream_t st);

hipError_t launch_track_adjoint(const AdjParams &A, int dtype, hipStream_t st);
void fill_adjoint_constants(AdjParams &A, const dgf_track_opts &o);

// Tracker flags the library implements, and those that need the row-run kernel.
constexpr int32_t kTrackFlags = DGF_TRACK_ILLUM | DGF_TRACK_CROSS | DGF_TRACK_GLOBAL;
constexpr int32_t kRowRunFlags = DGF_TRACK_ILLUM | DGF_TRACK_CROSS | DGF_TRACK_GLOBAL;

// Global-motion fit of the tracker's first pass (gm.hip): least squares, then ten Tukey
// reweightings, one launch each, plus one that finishes the last model.
constexpr int kGmSums = 13;      // weighted sums of one pass
constexpr int kGmPasses = 11;    // weighting passes
constexpr int kGmMaxBlocks = 256; // workgroups per pair and pass
constexpr double kTukeyC = 4.685;  // Tukey biweight constant, in coarsest-level pixels

struct GmFit {
    const float2 *pts, *flow;  // points and first-pass motion (level-0 pixels)
    const uint8_t *status;     // first-pass status: CONVERGED marks a sample
    int64_t n;                 // single pair: points [0, n) of a W x H frame
    int W, H;
    const int64_t *pt_off;     // batched: pair p holds points pt_off[p] .. pt_off[p + 1] (else null)
    const LevelPair *blv;      // batched: level table [npairs][L] (level 0 gives the frame size)
    int L;
    int npairs, nblk;          // nblk: largest gm_blocks over the pairs (the grid's x extent)
    double c;                  // Tukey constant, level-0 pixels
    double *models;            // [2][npairs][6]; the fitted model ends in the first half
    double *part;              // [2][npairs][nblk][kGmSums]
};

// Workgroups per pass for a pair of n points (about 2048 points each): a function of the pair's
// own count, so that a pair fitted in a batch plan is reduced exactly as it is on its own.
__host__ __device__ inline int gm_blocks(int64_t n)
{
    const int64_t b = (n + 2047) / 2048;
    return (int)(b < 1 ? 1 : (b > kGmMaxBlocks ? kGmMaxBlocks : b));
}
size_t gm_models_bytes(int npairs);
size_t gm_state_bytes(int npairs, int nblk); // models, then partials (at gm_models_bytes)
hipError_t launch_gm_fit(const GmFit &g, hipStream_t st);

struct TrackTuning {
    int lpp;     // lanes per point: 16, 32 or 64
    int wpb;     // waves per workgroup: 1, 2, 4
    int margin;  // I1 tile margin M
    int kind;    // 0: row-run kernel when compiled for this support, else generic; 1: generic
};

struct PyrJob {
    const uint8_t *src;
    uint8_t *dst;
    int64_t src_pitch, dst_pitch;
    int32_t W, H; // source size; destination is ceil(W/2) x ceil(H/2)
};

struct DetectJob {
    const uint8_t *img;
    int64_t pitch;
    int32_t W, H, win, stride, nx, ny;
    int64_t out_off; // index of the pair's first point in the concatenated output
};

// launchers (return hipSuccess or the launch error)
size_t detect_tile_lds(int win, int stride);
hipError_t launch_detect(const uint8_t *img, int64_t pitch, int W, int H, int win, int stride, float *pts,
                         uint8_t *sel, float *resp, hipStream_t st);
hipError_t launch_pyr_level(const PyrJob *jobs, int njobs, int dtype, hipStream_t st);

// Up to four consecutive uint8 levels of one or two images in one launch: level k (k = 1 .. m)
// of image f goes to dst[k - 1][f] with row pitch dst_pitch[k - 1]; W[0] x H[0] is the source
// level, W[k] = ceil(W[k - 1] / 2).
struct PyrChain {
    const uint8_t *src[2];
    int64_t src_pitch[2];
    uint8_t *dst[4][2];
    int64_t dst_pitch[4];
    int32_t W[5], H[5];
    int32_t m;
};
// Detection of one uint8 frame run beside the first pyramid-chain launch (dgf_detect_pyramids):
// tiles_x x tiles_y tiles of 16 x 16 windows; front_detect_fits tells whether a tile's pixels fit
// the chain's LDS.
struct FrontDetect {
    const uint8_t *img;
    int64_t pitch;
    int32_t W, H, win, stride, nx, ny, tiles_x, tiles_y;
    DetectOut o;
};
// The front end of a batch plan (front_batch.hip): level 1 of every frame beside every pair's
// detection in one launch, then one launch per coarser level.
struct BatchFront {
    const PyrJob *pyr;    // device: [(L - 1)][nframes] level jobs, frame 2p = I0 of pair p, 2p + 1 its I1
    const DetectJob *det; // device: [npairs]
    int nframes, npairs, L;
    int max_w2[DGF_MAX_LEVELS], max_h2[DGF_MAX_LEVELS]; // largest level-l size over the frames
    int det_tx, det_ty;   // tiles of 16 x 16 windows covering the largest window grid
    size_t det_lds;       // largest front_detect_lds over the pairs
};
hipError_t launch_front_batched(const BatchFront &F, float *pts, hipStream_t st);
size_t front_detect_lds(int win, int stride); // LDS of one pair's detection tile in that launch

bool front_detect_fits(int win, int stride);
hipError_t launch_pyr_chain_u8(const PyrChain &A, int njobs, hipStream_t st, const FrontDetect *det = nullptr);
hipError_t launch_pyr_chains(const uint8_t *const srcs[2], const int64_t src_pitch[2],
                             uint8_t *const lvl[2][DGF_MAX_LEVELS], const int64_t *pitch, int W, int H, int levels,
                             int njobs, hipStream_t st, const FrontDetect *det = nullptr);
hipError_t launch_track(const TrackParams &P, const TrackTuning &T, int dtype, hipStream_t st);
int pick_ppl_max(int s, int lpp);
bool run_shape_compiled(int lpp, int s);
int run_shape_lanes(int s); // lanes per point of a compiled row-run shape for support s (64 preferred), 0 if none
TrackTuning illum_tuning(int s, TrackTuning t); // t moved onto a row-run shape (the illumination model runs there)
// true when a kernel is compiled for this support and launch shape
bool track_shape_ok(int s, const TrackTuning &T);
constexpr size_t kMaxLdsPerBlock = 64 * 1024;
// LDS bytes of one tracker workgroup for this support and launch shape
size_t track_lds_bytes(int s, const TrackTuning &T);
void fill_track_geometry(TrackParams &P, int s, int margin, int lpp, int kind);

} // namespace dgf
