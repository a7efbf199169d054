// track_run_kernel.hpp -- the tracker of track_kernel.hpp with a row-run pixel layout (device code).
//
// Same method, same arithmetic per support pixel; only the assignment of support pixels to
// lanes differs.  The support rows are cut into runs of R consecutive pixels (R divides s), and
// each lane owns SEG runs.  Consequences on CDNA4:
//   * the I1 samples of a run come from R + 1 columns of two tile rows: R + 1 ds_read2_b32 with
//     immediate offsets off one base address per run (vertical lerp first, then horizontal, so
//     neighbouring pixels share their taps);
//   * the template of a run is built in registers from a 4 x (R + 3) patch of the raw I0 tile:
//     value and central differences at +-1 px are read off the bilinearly resampled patch;
//   * per-pixel state is just template value and gradient (3 registers), so 16 or 32 lanes per
//     point fit, and the per-iteration reduction and 2x2 solve are amortised over 14-28 pixels
//     per lane instead of 7.
#pragma once

#include "track_kernel.hpp"

namespace dgf {

// Five group sums at once, stage by stage, so that no DPP read waits on the add just before it.
template <int LPP>
__device__ __forceinline__ void group_sum5(float &a, float &b, float &c, float &d, float &e)
{
#define DGF_STAGE(CTRL)                                                                                                \
    {                                                                                                                  \
        const float ta = dpp<CTRL>(a), tb = dpp<CTRL>(b), tc = dpp<CTRL>(c), td = dpp<CTRL>(d), te = dpp<CTRL>(e);     \
        a += ta;                                                                                                       \
        b += tb;                                                                                                       \
        c += tc;                                                                                                       \
        d += td;                                                                                                       \
        e += te;                                                                                                       \
    }
    if constexpr (LPP == 64) {
        wave_sum5(a, b, c, d, e);
        return;
    }
    DGF_STAGE(0xB1)
    DGF_STAGE(0x4E)
    DGF_STAGE(0x141)
    DGF_STAGE(0x140)
#undef DGF_STAGE
    if constexpr (LPP == 32) {
        a = group_sum_cross<32>(a);
        b = group_sum_cross<32>(b);
        c = group_sum_cross<32>(c);
        d = group_sum_cross<32>(d);
        e = group_sum_cross<32>(e);
    }
}

// Adaptive cross-based support, decided on the level image's own pixels at floor(p) + k for the
// support offsets extended by one, k in [-r-1, r+1]^2 (the first G = s + 2 rows and columns of the
// raw patch, pitch RP; centre c = G / 2): exact comparisons for integer frames, where the
// interpolated template would put many differences exactly on tau.  Per row the horizontal arm
// around the row's centre-column pixel (pixels within tau of it, run outward until the first that
// is not), and the vertical arm of the centre.  Rows are shared out over the group's lanes; the
// arms go to `arms` in LDS: left[y], right[y] as arms[2 y], arms[2 y + 1] (0 .. c), up and down in
// arms[2 G], arms[2 G + 1].  Needs G <= 32 (row flags as a 32-bit mask).
template <int LPP, int G, int RP>
__device__ __forceinline__ void cross_arms(const float *raw, int *arms, float tau, int li)
{
    static_assert(G <= 32, "cross-based supports need s + 2 <= 32");
    constexpr int c = G / 2;
    const float centre = raw[c * RP + c];
    unsigned vbits = 0u; // bit y: centre-column pixel of row y within tau of the centre
    for (int y = li; y < G; y += LPP) {
        const float *row = raw + y * RP;
        const float a = row[c];
        unsigned ok = 0u;
#pragma unroll
        for (int x = 0; x < G; ++x) ok |= (fabsf(row[x] - a) <= tau ? 1u : 0u) << x;
        const unsigned above = ok >> (c + 1), below = ok << (32 - c);
        arms[2 * y] = min(__builtin_clz(~below), c);
        arms[2 * y + 1] = min(__builtin_ctz(~above), c);
        vbits |= (fabsf(a - centre) <= tau ? 1u : 0u) << y;
    }
    // the vertical arm from the group's row flags
    const unsigned all = (unsigned)group_or<LPP>(vbits);
    if (li == 0) {
        arms[2 * G] = min(__builtin_clz(~(all << (32 - c))), c);
        arms[2 * G + 1] = min(__builtin_ctz(~(all >> (c + 1))), c);
    }
}

// The integer value of a wave-uniform integral float (a floor), decoded from its bits by scalar
// instructions (one vector read-first-lane): exact below 2^23 in magnitude, +-2^23 beyond and for
// non-finite values, which keeps every tile offset far from integer overflow (staging clamps each
// address into the image).
__device__ __forceinline__ int uniform_floor_int(float f)
{
    const int b = __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, f));
    const int e = ((b >> 23) & 0xFF) - 127; // unbiased exponent; -127 for +-0
    const int mag = e < 0 ? 0 : e >= 23 ? (1 << 23) : (((b & 0x7FFFFF) | 0x800000) >> (23 - e));
    return b < 0 ? -mag : mag;
}

// A square rectangle (rows = cols) of at most 8 NS rows into LDS (B steps' loads in flight;
// CROWS: its row count when fixed at compile time): the unrolled whole-wavefront form for uint8
// images where it qualifies, stage_rect otherwise, its lane layout worked out there and then
// (border tiles are rare, and the layout would otherwise hold registers for the whole launch).
template <int LPP, typename PixT, int NS, int B, int CROWS = 0>
__device__ __forceinline__ void stage_tile(float *lds, int lp, const uint8_t *base, int64_t pitch, int W, int H, int ox,
                                           int oy, int rows, int cols, int li)
{
    if constexpr (LPP == 64 && sizeof(PixT) == 1)
        if (stage_u8_w64<NS, B, CROWS>(lds, lp, base, pitch, W, H, ox, oy, rows, cols, li)) return;
    stage_rect<LPP, PixT>(lds, lp, base, pitch, W, H, ox, oy, rows, cols, stage_lanes<LPP>(cols, li));
}

// True when the flag is set on any lane of the wavefront.  With one point per wavefront (64 lanes
// per point) every lane holds the same value, so the flag itself decides the branch: no ballot,
// whose lowering would spend two vector instructions turning a mask back into a condition.
template <int LPP>
__device__ __forceinline__ bool group_any(bool p)
{
    if constexpr (LPP == 64)
        return p;
    else
        return wave_any(p);
}

// The 64-lane form without the illumination model is held to 80 VGPRs (six waves per SIMD): it is
// issue bound, and the sixth wave pays.  MODE (ROBUST_L2 / HAMPEL / HARD), CROSS (adaptive
// cross-based supports) and BATCH (a batch plan's persistent launch rather than one pair) are
// compile-time, so a single-pair square-window launch carries no batch bookkeeping, no per-pixel
// support mask and no branch on the robust norm.
template <int LPP, int SEG, int R, int TP, int S, typename PixT, bool IM, int MODE, bool CROSS, bool BATCH>
__global__ __launch_bounds__(256, (LPP == 64 && !IM) ? 6 : 1) void k_track_run(TrackParams P)
{
    constexpr int PPW = 64 / LPP;
    constexpr int PPL = SEG * R;
    extern __shared__ float smem[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wpb = blockDim.x >> 6;
    const int q = lane / LPP;
    const int li = lane - q * LPP;
    float *tile = smem + (size_t)(wave * PPW + q) * P.tile_floats;

    // support s x s, raw I0 patch (s + 3)^2 with row pitch RP (the host's raw_pitch(s)), resampled
    // grid (s + 2)^2 below it with the same pitch
    constexpr int s = S, r = S / 2, RW = S + 3, RP = (RW % 4 == 0) ? RW + 2 : RW, G = S + 2;
    static_assert(S % R == 0, "runs must tile the support rows");
    const int TW = P.TW, M = P.M;
    constexpr int nseg_row = s / R; // runs per support row
    constexpr int nseg = s * nseg_row;

    // run geometry: sb = row * TP + col0 of the run's first pixel in the I1 tile, rc = row << 8 |
    // col0; unused runs point at 0 and carry zero gradients
    int sb[SEG], rc[SEG];
    unsigned vmask = 0u;
#pragma unroll
    for (int j = 0; j < SEG; ++j) {
        const int g = j * LPP + li;
        const bool vg = g < nseg;
        const int gg = vg ? g : 0;
        const int row = gg / nseg_row;
        const int col0 = (gg - row * nseg_row) * R;
        sb[j] = row * TP + col0;
        // one register holding the whole offset: the run's tile address is then a single
        // shift-and-add off the wave's tile origin (the compiler would otherwise keep the row
        // and column terms apart and add them in every iteration)
        asm("" : "+v"(sb[j]));
        rc[j] = (row << 8) | col0;
        vmask |= (vg ? 1u : 0u) << j;
    }

    float T[PPL], GX[PPL], GY[PPL];

    // Plain launches give each XCD runs of 64 consecutive points in turn (plain_item; the points
    // are taken from the last one back, see work_item): every image band is still spread over all
    // eight XCDs, which balances the uneven per-point work, while each point's output lines are
    // written from one L2.  (Giving each XCD one band cut L2 fills 4.6x on the 1242x375 benchmark
    // pair but made the launch 25% longer.)  Persistent launches pull from the queue of their own
    // XCD first.
    const int home = (int)(blockIdx.x % kNumXcd);
    int visit = 0;
    int64_t item = (BATCH && P.persistent) ? next_item(P, home, visit)
                   : (!BATCH || P.npairs == 0) ? plain_item<PPW>(blockIdx.x, wave, wpb)
                                               : (int64_t)blockIdx.x * wpb + wave;
    for (;;) {
    const WorkItem wi = work_item<PPW, BATCH>(P, item, q);
    if (wi.done) break;
    const int64_t pidx = wi.pidx;
    const int pair = wi.pair;
    const bool valid = wi.valid;
    float px = 0.f, py = 0.f;
    if (valid) {
        const float2 pp = reinterpret_cast<const float2 *>(P.pts)[pidx];
        px = pp.x;
        py = pp.y;
    }
    const LevelPair LV0 = level_of<BATCH>(P, pair, 0);
    const int W0 = LV0.W, H0 = LV0.H;
    int status = -1;
    float ux = 0.f, uy = 0.f;
    if (valid && !(px >= 0.f && py >= 0.f && px <= (float)(W0 - 1) && py <= (float)(H0 - 1))) status = DGF_ST_OUT_OF_BOUNDS;
    bool active = valid && status < 0;
    if (!active) {
        px = 0.f;
        py = 0.f;
    }
    float gX = 0.f, gY = 0.f; // guess of the current level
    float hX = 0.f, hY = 0.f; // guess plus the steps taken on it so far (g + d)
    if (P.gm_model && active) {
        // global-motion prior: the coarsest level starts from the fitted affine motion at the point
        const double *A = P.gm_model + (BATCH ? 6 * pair : 0);
        const double x = (double)px - 0.5 * (W0 - 1), y = (double)py - 0.5 * (H0 - 1);
        const double itop = __builtin_ldexp(1.0, 1 - P.L); // coarsest-level pixels per level-0 pixel
        gX = (float)(fma(A[0], x, fma(A[1], y, A[2])) * itop);
        gY = (float)(fma(A[3], x, fma(A[4], y, A[5])) * itop);
    }
    bool conv0 = false;
    int it_total = 0;
    float im_m = 0.f, im_c = 0.f; // illumination model: gain change and offset, carried across levels


    for (int l = P.L - 1; l >= P.lstop; --l) {
        if (!group_any<LPP>(active)) break;
        const LevelPair LV = level_of<BATCH>(P, pair, l);
        const int Wl = LV.W, Hl = LV.H;
        const float sc = __builtin_ldexpf(1.0f, -l);
        const float plx = px * sc, ply = py * sc;
        const float pbx = floorf(plx), pby = floorf(ply);
        const float pfx = plx - pbx, pfy = ply - pby;
        const int ibx = (int)pbx - r, iby = (int)pby - r;

        // ---- template: raw I0_l patch (s+3)^2 with replicated border, row pitch RP
        wave_sync();
        stage_tile<LPP, PixT, (RW + 7) / 8, (RW + 7) / 8, RW>(tile, RP, LV.p0, LV.pitch0, Wl, Hl, ibx - 1, iby - 1, RW, RW, li);
        wave_sync();
        // Bilinear resample of the raw patch on the (s + 2)^2 grid of support offsets -r-1 .. r+1
        // (every sample shares the point's fraction): lanes take runs of kRes grid columns of one
        // grid row, a vertical lerp per raw column and a horizontal lerp between neighbours.
        float *grid = tile + RW * RP;
        {
            constexpr int kRes = 12, runs_row = (G + kRes - 1) / kRes;
            for (int u = li; u < G * runs_row; u += LPP) {
                const int gi = u / runs_row, c0 = (u - gi * runs_row) * kRes;
                const float *q = tile + gi * RP + c0;
                float v[kRes + 1];
#pragma unroll
                for (int cc = 0; cc <= kRes; ++cc) v[cc] = fmaf(pfy, q[RP + cc] - q[cc], q[cc]);
                float *o = grid + gi * RP + c0;
#pragma unroll
                for (int cc = 0; cc < kRes; ++cc)
                    if (c0 + cc < G) o[cc] = fmaf(pfx, v[cc + 1] - v[cc], v[cc]);
            }
        }
        wave_sync();
        // support of this level: bit j*R+p of pm for pixel p of run j (unused runs are out); the
        // square window is every pixel of the used runs
        unsigned pm = 0u;
#pragma unroll
        for (int j = 0; j < SEG; ++j)
            if ((vmask >> j) & 1u) pm |= ((1u << R) - 1u) << (j * R);
        auto in_support = [&](int j) -> bool {
            if constexpr (CROSS)
                return (pm >> j) & 1u;
            else
                return (vmask >> (j / R)) & 1u;
        };
        if constexpr (CROSS) {
            // adaptive cross-based support: a pixel stays when it and its four neighbours lie in
            // the cross region (no template gradient straddles the region's edge)
            int *arms = reinterpret_cast<int *>(grid + G * RP);
            cross_arms<LPP, G, RP>(tile, arms, P.tau, li);
            wave_sync();
            constexpr int c = G / 2;
            const int up = arms[2 * G], down = arms[2 * G + 1];
#pragma unroll
            for (int j = 0; j < SEG; ++j) {
                const int y = (rc[j] >> 8) + 1, x0 = (rc[j] & 255) + 1;
                const bool rowok = (y - 1 >= c - up) && (y + 1 <= c + down);
                const int lo = max(c - arms[2 * y] + 1, max(c - arms[2 * y - 2], c - arms[2 * y + 2]));
                const int hi = min(c + arms[2 * y + 1] - 1, min(c + arms[2 * y - 1], c + arms[2 * y + 3]));
#pragma unroll
                for (int p = 0; p < R; ++p)
                    if (!(rowok && x0 + p >= lo && x0 + p <= hi)) pm &= ~(1u << (j * R + p));
            }
        }
        // template value and central differences at +-1 px of the resampled patch.  Pixels out of
        // the support get half = 0, so their gradients vanish (unused runs read run 0's pixels,
        // so a non-finite pixel there reaches the sums through run 0 anyway).
#pragma unroll
        for (int j = 0; j < SEG; ++j) {
            const int row = rc[j] >> 8, col0 = rc[j] & 255;
            const float *gm = grid + row * RP + col0 + 1;      // grid row of support row - 1
            const float *g0 = gm + RP, *gp = gm + 2 * RP;        // support row, support row + 1
#pragma unroll
            for (int p = 0; p < R; ++p) {
                const float half = in_support(j * R + p) ? 0.5f : 0.f;
                T[j * R + p] = g0[p];
                GX[j * R + p] = half * (g0[p + 1] - g0[p - 1]);
                GY[j * R + p] = half * (gp[p] - gm[p]);
            }
        }
        float a = 0.f, b = 0.f, c = 0.f, sT = 0.f, nsup = 0.f;
#pragma unroll
        for (int j = 0; j < PPL; ++j) {
            a = fmaf(GX[j], GX[j], a);
            b = fmaf(GX[j], GY[j], b);
            c = fmaf(GY[j], GY[j], c);
            if constexpr (IM) sT += in_support(j) ? T[j] : 0.f;
        }
        if constexpr (CROSS) nsup = (float)__builtin_popcount(pm);
        group_sum5<LPP>(a, b, c, sT, nsup);
        if constexpr (!CROSS) nsup = (float)(s * s);
        // Illumination model: the template is centred and scaled over the support, T' = (T - Tm) / Ts,
        // and the iteration runs in (d, ga, gb) with ga = (1 + m) Ts and gb = (1 + m) Tm + c, a linear
        // change of the gain / offset parameters that leaves the Gauss-Newton iterates in d unchanged
        // and conditions the 4x4 system.  M0 is its unweighted matrix for phi = (g, -T', -1).
        float Tm = 0.f, Ts = 1.f, ga = 0.f, gb = 0.f, det0_im = 0.f;
        float M0[10];
        if constexpr (IM) {
            const float nv = nsup;
            Tm = sT / nv;
            float S2 = 0.f, Sgxd = 0.f, Sgyd = 0.f, Sgx = 0.f, Sgy = 0.f;
#pragma unroll
            for (int j = 0; j < PPL; ++j) {
                const float dv = in_support(j) ? T[j] - Tm : 0.f;
                S2 = fmaf(dv, dv, S2);
                Sgxd = fmaf(GX[j], dv, Sgxd);
                Sgyd = fmaf(GY[j], dv, Sgyd);
                Sgx += GX[j];
                Sgy += GY[j];
            }
            group_sum5<LPP>(S2, Sgxd, Sgyd, Sgx, Sgy);
            Ts = sqrtf(S2 / nv);
            if (!(Ts > 1e-6f)) Ts = 1.f;
            const float iTs = 1.f / Ts;
#pragma unroll
            for (int j = 0; j < PPL; ++j) T[j] = (T[j] - Tm) * iTs;
            M0[0] = a;
            M0[1] = b;
            M0[2] = -Sgxd * iTs;
            M0[3] = -Sgx;
            M0[4] = c;
            M0[5] = -Sgyd * iTs;
            M0[6] = -Sgy;
            M0[7] = S2 * iTs * iTs;
            M0[8] = 0.f; // sum of T' over the support
            M0[9] = nv;
            det0_im = ldl4(M0, nullptr, nullptr);
            ga = (1.f + im_m) * Ts;
            gb = fmaf(1.f + im_m, Tm, im_c);
        }
        const float lam = 0.5f * (a + c) - sqrtf(fmaf(b, b, 0.25f * (a - c) * (a - c)));
        // too flat to invert: a coarse level runs no iteration and passes the guess on; at
        // level 0 the point is ill-conditioned with u = g.  (An empty cross-based support is flat,
        // and with the illumination model one of fewer than four pixels: four unknowns.)
        const bool flat = active && !(CROSS ? (nsup >= (IM ? 4.f : 1.f) && lam >= P.min_eig * nsup)
                                            : lam >= P.min_eig_s2);
        if (flat && l == P.lstop) {
            status = DGF_ST_ILL_CONDITIONED;
            ux = gX;
            uy = gY;
            active = false;
        }
        const float det0 = fmaf(a, c, -b * b);
        const float eps2 = (l > 0) ? P.eps2c : P.eps2f;

        // ---- iterations
        hX = gX;
        hY = gY;
        bool lvl_active = active && !flat, lvl_conv = false;
        // below this the weighted system falls back to least squares
        const float det_floor = 1e-6f * (IM ? det0_im : det0);
        int ox1 = 0, oy1 = 0;
        for (int it = 0; it < P.iters; ++it) {
            if (!group_any<LPP>(lvl_active)) break;
            const float tx = pfx + hX, ty = pfy + hY;
            const float flx = floorf(tx), fly = floorf(ty);
            const float fx = tx - flx, fy = ty - fly;
            // integer part, kept finite and small for the tile arithmetic (a non-finite guess only
            // occurs on a point already stopped, whose samples are discarded)
            int ix, iy;
            if constexpr (LPP == 64) {
                // one point per wavefront: the position is wave-uniform, and scalar code decodes
                // the integer from the floor's bits
                ix = uniform_floor_int(flx);
                iy = uniform_floor_int(fly);
            } else {
                ix = (int)__builtin_amdgcn_fmed3f(flx, -1048576.f, 1048576.f);
                iy = (int)__builtin_amdgcn_fmed3f(fly, -1048576.f, 1048576.f);
            }
            const int bx = ibx + ix, by = iby + iy;
            int dxo = bx - ox1, dyo = by - oy1;
            const bool inr = dxo >= 0 && dxo <= 2 * M && dyo >= 0 && dyo <= 2 * M;
            if (group_any<LPP>((it == 0) || (lvl_active && !inr))) {
                wave_sync();
                ox1 = bx - M;
                oy1 = by - M;
                stage_tile<LPP, PixT, (TP + 7) / 8, 2>(tile, TP, LV.p1, LV.pitch1, Wl, Hl, ox1, oy1, TW, TW, li);
                wave_sync();
                dxo = M;
                dyo = M;
            } else if (!inr) {
                dxo = 0;
                dyo = 0;
            }
            const float *tb = tile + dyo * TP + dxo;

            // residuals of every pixel of this lane's runs
            // bilinear weights shared by every sample of this iteration; each residual is a chain
            // of four FMAs started from -T
            const float w11 = fx * fy, w10 = fmaf(-fx, fy, fx), w01 = fmaf(-fx, fy, fy), w00 = (1.f - fx) - w01;
            float RES[PPL];
#pragma unroll
            for (int j = 0; j < SEG; ++j) {
                const float *rp = tb + sb[j];
                float t0[R + 1], t1[R + 1];
#pragma unroll
                for (int cc = 0; cc < R + 1; ++cc) {
                    t0[cc] = rp[cc];
                    t1[cc] = rp[TP + cc];
                }
#pragma unroll
                for (int p = 0; p < R; ++p) {
                    float v;
                    if constexpr (IM)
                        v = fmaf(w00, t0[p], -fmaf(ga, T[j * R + p], gb));
                    else
                        v = fmaf(w00, t0[p], -T[j * R + p]);
                    v = fmaf(w10, t0[p + 1], v);
                    v = fmaf(w01, t1[p], v);
                    RES[j * R + p] = fmaf(w11, t1[p + 1], v);
                }
            }

            float sx, sy, sa = 0.f, sb = 0.f;
            if constexpr (IM) {
                // phi = (g, -T', -1) per pixel: A = sum w phi phi^T (upper triangle), V = sum w r phi
                // with the signs applied after the reduction; invalid runs have weight 0
                float A[10], V[4], x[4]; // step = A^-1 (-sum w r phi) with phi = (g, -T', -1)
                float q0 = 0.f, q1 = 0.f, q2 = 0.f, q3 = 0.f;
                if constexpr (MODE == ROBUST_L2) {
#pragma unroll
                    for (int j = 0; j < PPL; ++j) {
                        const float w = in_support(j) ? 1.f : 0.f;
                        const float rw = RES[j] * w;
                        q0 = fmaf(rw, GX[j], q0);
                        q1 = fmaf(rw, GY[j], q1);
                        q2 = fmaf(rw, T[j], q2);
                        q3 += rw;
                    }
                    float z0 = 0.f;
                    group_sum5<LPP>(q0, q1, q2, q3, z0);
#pragma unroll
                    for (int e = 0; e < 10; ++e) A[e] = M0[e];
                    V[0] = -q0;
                    V[1] = -q1;
                    V[2] = q2;
                    V[3] = q3;
                    ldl4(A, V, x);
                } else {
                    float s00 = 0.f, s01 = 0.f, s11 = 0.f, s02 = 0.f, s12 = 0.f, s03 = 0.f, s13 = 0.f, s22 = 0.f,
                          s23 = 0.f, s33 = 0.f;
#pragma unroll
                    for (int j = 0; j < PPL; ++j) {
                        float w = (MODE == ROBUST_HAMPEL) ? hampel_weight(RES[j], P.cs2, P.cmid)
                                                          : ((fabsf(RES[j]) <= P.s1) ? 1.f : 0.f);
                        w = in_support(j) ? w : 0.f;
                        const float wgx = w * GX[j], wgy = w * GY[j], wt = w * T[j];
                        s00 = fmaf(wgx, GX[j], s00);
                        s01 = fmaf(wgx, GY[j], s01);
                        s11 = fmaf(wgy, GY[j], s11);
                        s02 = fmaf(wgx, T[j], s02);
                        s12 = fmaf(wgy, T[j], s12);
                        s03 += wgx;
                        s13 += wgy;
                        s22 = fmaf(wt, T[j], s22);
                        s23 += wt;
                        s33 += w;
                        q0 = fmaf(RES[j], wgx, q0);
                        q1 = fmaf(RES[j], wgy, q1);
                        q2 = fmaf(RES[j], wt, q2);
                        q3 = fmaf(RES[j], w, q3);
                    }
                    float z0 = 0.f;
                    group_sum5<LPP>(s00, s01, s11, s02, s12);
                    group_sum5<LPP>(s03, s13, s22, s23, s33);
                    group_sum5<LPP>(q0, q1, q2, q3, z0);
                    A[0] = s00;
                    A[1] = s01;
                    A[2] = -s02;
                    A[3] = -s03;
                    A[4] = s11;
                    A[5] = -s12;
                    A[6] = -s13;
                    A[7] = s22;
                    A[8] = s23;
                    A[9] = s33;
                    // the factorisation that gives det A also solves for the step; only lanes
                    // that fall back need a second one
                    V[0] = -q0;
                    V[1] = -q1;
                    V[2] = q2;
                    V[3] = q3;
                    const float detw = ldl4(A, V, x);
                    const bool fb = lvl_active && !(detw > det_floor);
                    if (group_any<LPP>(fb)) { // too many down-weighted pixels: least-squares step
                        float u0 = 0.f, u1 = 0.f, u2 = 0.f, u3 = 0.f, z1 = 0.f;
#pragma unroll
                        for (int j = 0; j < PPL; ++j) {
                            const float rv = in_support(j) ? RES[j] : 0.f;
                            u0 = fmaf(rv, GX[j], u0);
                            u1 = fmaf(rv, GY[j], u1);
                            u2 = fmaf(rv, T[j], u2);
                            u3 += rv;
                        }
                        group_sum5<LPP>(u0, u1, u2, u3, z1);
                        if (fb) {
#pragma unroll
                            for (int e = 0; e < 10; ++e) A[e] = M0[e];
                            V[0] = -u0;
                            V[1] = -u1;
                            V[2] = u2;
                            V[3] = u3;
                        }
                        ldl4(A, V, x);
                    }
                }
                // the d rows of the model's system carry (1 + m) = ga / Ts; the unscaled system
                // solved here gives (1 + m) d, scaled back by Ts / ga (one reciprocal: correctly
                // rounded divisions cost about ten instructions each; ga = 0 still gives a
                // non-finite step)
                const float ik = Ts * __builtin_amdgcn_rcpf(ga);
                sx = x[0] * ik;
                sy = x[1] * ik;
                sa = x[2];
                sb = x[3];
            } else {
                float G11, G12, G22, B1 = 0.f, B2 = 0.f, det;
                if constexpr (MODE == ROBUST_L2) {
    #pragma unroll
                    for (int j = 0; j < PPL; ++j) {
                        B1 = fmaf(RES[j], GX[j], B1);
                        B2 = fmaf(RES[j], GY[j], B2);
                    }
                    float z0 = 0.f, z1 = 0.f, z2 = 0.f;
                    group_sum5<LPP>(B1, B2, z0, z1, z2);
                    G11 = a;
                    G12 = b;
                    G22 = c;
                    det = det0;
                } else {
                    G11 = 0.f;
                    G12 = 0.f;
                    G22 = 0.f;
                    if constexpr (MODE == ROBUST_HAMPEL) {
    #pragma unroll
                        for (int j = 0; j < PPL; ++j) {
                            const float w = hampel_weight(RES[j], P.cs2, P.cmid);
                            const float wgx = w * GX[j], wgy = w * GY[j];
                            G11 = fmaf(wgx, GX[j], G11);
                            G12 = fmaf(wgx, GY[j], G12);
                            G22 = fmaf(wgy, GY[j], G22);
                            B1 = fmaf(RES[j], wgx, B1);
                            B2 = fmaf(RES[j], wgy, B2);
                        }
                    } else {
    #pragma unroll
                        for (int j = 0; j < PPL; ++j) {
                            const float w = (fabsf(RES[j]) <= P.s1) ? 1.f : 0.f;
                            const float wgx = w * GX[j], wgy = w * GY[j];
                            G11 = fmaf(wgx, GX[j], G11);
                            G12 = fmaf(wgx, GY[j], G12);
                            G22 = fmaf(wgy, GY[j], G22);
                            B1 = fmaf(RES[j], wgx, B1);
                            B2 = fmaf(RES[j], wgy, B2);
                        }
                    }
                    group_sum5<LPP>(G11, G12, G22, B1, B2);
                    det = fmaf(G11, G22, -G12 * G12);
                    const bool fb = lvl_active && !(det > det_floor);
                    if (group_any<LPP>(fb)) {
                        float C1 = 0.f, C2 = 0.f;
    #pragma unroll
                        for (int j = 0; j < PPL; ++j) {
                            C1 = fmaf(RES[j], GX[j], C1);
                            C2 = fmaf(RES[j], GY[j], C2);
                        }
                        float z0 = 0.f, z1 = 0.f, z2 = 0.f;
                        group_sum5<LPP>(C1, C2, z0, z1, z2);
                        if (fb) {
                            G11 = a;
                            G12 = b;
                            G22 = c;
                            B1 = C1;
                            B2 = C2;
                            det = det0;
                        }
                    }
                }
                const float inv = __builtin_amdgcn_rcpf(det);
                sx = fmaf(G12, B2, -G22 * B1) * inv;
                sy = fmaf(G12, B1, -G11 * B2) * inv;
            }
            if (lvl_active) {
                ++it_total;
                if (!(isfinite(sx) && isfinite(sy) && isfinite(sa) && isfinite(sb))) {
                    status = DGF_ST_NOT_CONVERGED;
                    ux = __builtin_nanf("");
                    uy = __builtin_nanf("");
                    active = false;
                    lvl_active = false;
                } else {
                    hX += sx;
                    hY += sy;
                    if constexpr (IM) {
                        ga += sa;
                        gb += sb;
                    }
                    if (fmaf(sx, sx, sy * sy) < eps2) {
                        lvl_conv = true;
                        lvl_active = false;
                    }
                }
            }
        }
        if constexpr (IM) {
            if (active && !flat) { // back to (m, c), which carry over to the next level
                im_m = ga / Ts - 1.f;
                im_c = gb - ga * Tm / Ts;
                if (l > P.lstop && !(1.f + im_m >= 0.25f && 1.f + im_m <= 4.f)) {
                    // a runaway gain (towards 0, where the motion drops out of the model) ends the point
                    status = DGF_ST_NOT_CONVERGED;
                    ux = __builtin_nanf("");
                    uy = __builtin_nanf("");
                    active = false;
                }
            }
        }
        if (l > P.lstop) {
            if (active) {
                gX = 2.f * hX;
                gY = 2.f * hY;
            }
        } else {
            conv0 = lvl_conv;
        }
    }

    if (valid && li == 0) {
        if (status < 0) {
            ux = hX;
            uy = hY;
            if (!conv0 || (IM && !(1.f + im_m >= 0.5f && 1.f + im_m <= 2.f))) {
                // (illumination model: a gain outside [1/2, 2] is a contrast change, not a match)
                status = DGF_ST_NOT_CONVERGED;
            } else if (P.lstop > 0) {
                // a pass that stops above level 0 (the global prior's first pass) reports the
                // step test only, with the motion in level-0 pixels
                status = DGF_ST_CONVERGED;
                ux = ldexpf(ux, P.lstop);
                uy = ldexpf(uy, P.lstop);
            } else {
                const float qx = px + ux, qy = py + uy;
                status = (qx >= 0.f && qy >= 0.f && qx <= (float)(W0 - 1) && qy <= (float)(H0 - 1)) ? DGF_ST_CONVERGED
                                                                                                 : DGF_ST_OUT_OF_BOUNDS;
            }
        }
        reinterpret_cast<float2 *>(P.flow)[pidx] = make_float2(ux, uy);
        P.status[pidx] = (uint8_t)status;
        if (P.iters_out) P.iters_out[pidx] = it_total;
        if constexpr (IM) {
            if (P.illum_out) reinterpret_cast<float2 *>(P.illum_out)[pidx] = make_float2(im_m, im_c);
        }
    }
    if (!(BATCH && P.persistent)) break;
    item = next_item(P, home, visit);
    } // work loop
}

template <int LPP, int SEG, int R, int TP, int S, typename PixT, bool IM, bool CROSS, bool BATCH>
hipError_t launch_track_run_t(const TrackParams &P, int wpb, hipStream_t st)
{
    constexpr int PPW = 64 / LPP;
    const int64_t waves = P.npairs ? P.grid_waves : (P.n + PPW - 1) / PPW;
    const int64_t blocks = P.npairs ? (waves + wpb - 1) / wpb : plain_blocks((waves + wpb - 1) / wpb, wpb, PPW);
    const size_t lds = (size_t)wpb * PPW * P.tile_floats * sizeof(float);
    const dim3 grid((unsigned)blocks), block(64 * wpb);
    if (P.mode == ROBUST_L2)
        hipLaunchKernelGGL((k_track_run<LPP, SEG, R, TP, S, PixT, IM, ROBUST_L2, CROSS, BATCH>), grid, block, lds, st, P);
    else if (P.mode == ROBUST_HAMPEL)
        hipLaunchKernelGGL((k_track_run<LPP, SEG, R, TP, S, PixT, IM, ROBUST_HAMPEL, CROSS, BATCH>), grid, block, lds, st,
                           P);
    else
        hipLaunchKernelGGL((k_track_run<LPP, SEG, R, TP, S, PixT, IM, ROBUST_HARD, CROSS, BATCH>), grid, block, lds, st, P);
    return hipGetLastError();
}

// Dispatcher of one instantiation file: element type, cross-based supports or not, single pair
// or batch plan; the support shape and the illumination model are picked at run time.
#define DGF_DEFINE_TRACK_RUN_LAUNCH(NAME, PIXT, CROSS, BATCH)                                                          \
    hipError_t NAME(const TrackParams &P, int lpp, int s, int wpb, hipStream_t st)                                     \
    {                                                                                                                  \
        DGF_TRACK_RUN_SHAPES(DGF_TRACK_RUN_CASE_##CROSS##_##BATCH, PIXT)                                               \
        return hipErrorInvalidValue;                                                                                   \
    }
#define DGF_TRACK_RUN_CASE(L_, SEG_, R_, TP_, S_, X_, C_, B_)                                                          \
    if (lpp == L_ && s == S_)                                                                                          \
        return P.illum ? launch_track_run_t<L_, SEG_, R_, TP_, S_, X_, true, C_, B_>(P, wpb, st)                       \
                       : launch_track_run_t<L_, SEG_, R_, TP_, S_, X_, false, C_, B_>(P, wpb, st);
#define DGF_TRACK_RUN_CASE_false_false(L_, SEG_, R_, TP_, S_, X_) DGF_TRACK_RUN_CASE(L_, SEG_, R_, TP_, S_, X_, false, false)
#define DGF_TRACK_RUN_CASE_false_true(L_, SEG_, R_, TP_, S_, X_) DGF_TRACK_RUN_CASE(L_, SEG_, R_, TP_, S_, X_, false, true)
#define DGF_TRACK_RUN_CASE_true_false(L_, SEG_, R_, TP_, S_, X_) DGF_TRACK_RUN_CASE(L_, SEG_, R_, TP_, S_, X_, true, false)
#define DGF_TRACK_RUN_CASE_true_true(L_, SEG_, R_, TP_, S_, X_) DGF_TRACK_RUN_CASE(L_, SEG_, R_, TP_, S_, X_, true, true)

// Row-run shapes compiled per element type: (LPP, SEG, R, TP, support s).  SEG runs of R pixels
// per lane cover the s * (s / R) runs of an s x s support.  The odd tile pitch TP = 31 spreads
// the runs of consecutive rows over different LDS banks (a pitch of 32 maps them onto 3;
// a pitch of 43, conflict-free for the 64-lane form in a bank model, measured slower and no fewer
// conflict cycles).
#define DGF_TRACK_RUN_SHAPES(X, PixT)                                                                                  \
    X(64, 1, 7, 31, 21, PixT) X(32, 2, 7, 31, 21, PixT) X(16, 4, 7, 31, 21, PixT) X(32, 1, 3, 31, 9, PixT)             \
    X(16, 2, 3, 31, 9, PixT) X(32, 2, 5, 31, 15, PixT) X(16, 3, 5, 31, 15, PixT) X(16, 1, 11, 31, 11, PixT)           \
    X(16, 1, 7, 31, 7, PixT) X(16, 1, 5, 31, 5, PixT)

} // namespace dgf
