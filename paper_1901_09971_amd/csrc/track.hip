// track.hip -- pyramidal robust local optical flow tracking on gfx950.
//
// Per point, coarse to fine (the tracker of DeGraF-Flow Section 2, "Sparse point tracking"; a
// Lucas-Kanade derivative, Section 1): a support of s x s pixels around p_l = p / 2^l is sampled
// bilinearly in I0_l (template T_k and central-difference gradient g_k), then iteratively
// re-weighted Gauss-Newton steps on the 2x2 normal equations
//     (sum w_k g_k g_k^T) step = -sum w_k r_k g_k,   r_k = I1_l(p_l + k + guess + d) - T_k,
//     w_k = psi(r_k) / r_k
// move d until |step| < eps_l; the level result seeds the next level as 2 (guess + d).
//
// Mapping onto CDNA4:
//   * One point per group of LPP lanes (LPP = 16, 32 or 64, so 4, 2 or 1 points per wavefront).
//     Support pixel k goes to lane k mod LPP, slot k / LPP; each lane keeps its slots' template
//     value and gradient in registers for the whole level.
//   * The I1 samples of one iteration all share the same fractional offset (the support moves
//     rigidly), so the four bilinear weights are computed once per point and iteration.  The I1
//     neighbourhood of the support is staged in LDS as a (s + 1 + 2M)^2 float tile with a margin
//     of M pixels; it is re-staged only when the integer part of the displacement drifts more
//     than M pixels.  Each support pixel then costs two ds_read2_b32 and about twenty VALU ops.
//   * The five sums of the normal equations are reduced across the LPP lanes with DPP row
//     butterflies plus readlane (no LDS round trip); the 2x2 solve is done redundantly by every
//     lane of the point, so no broadcast is needed.
//   * Points that have stopped (converged at this level, ill-conditioned, out of bounds) keep
//     executing with their updates masked until every point of the wavefront has stopped.
//   * Coordinates keep the integer part and the fraction apart (floor(p_l) plus a small offset),
//     so the bilinear weights do not lose precision at x ~ 2000.
// No MFMA: each point's system is 2x2, not a dense contraction.
#include "dgf_internal.hpp"

namespace dgf {

template <int LPP, int PPLMAX, typename PixT>
__global__ __launch_bounds__(256) void k_track(TrackParams P)
{
    constexpr int PPW = 64 / LPP;
    extern __shared__ float smem[];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wpb = blockDim.x >> 6;
    const int q = lane / LPP;
    const int li = lane - q * LPP;
    const int64_t pidx = ((int64_t)blockIdx.x * wpb + wave) * PPW + q;
    float *tile = smem + (size_t)(wave * PPW + q) * P.tile_floats;

    const int s = P.s, r = P.r, S2 = s * s, TW = P.TW, RW = P.RW, M = P.M, ppl = P.ppl;

    const bool valid = pidx < P.n;
    float px = 0.f, py = 0.f;
    if (valid) {
        const float2 pp = reinterpret_cast<const float2 *>(P.pts)[pidx];
        px = pp.x;
        py = pp.y;
    }
    const int W0 = P.lv[0].W, H0 = P.lv[0].H;
    int status = -1; // -1: still running
    float ux = 0.f, uy = 0.f;
    if (valid && !(px >= 0.f && py >= 0.f && px <= (float)(W0 - 1) && py <= (float)(H0 - 1))) status = DGF_ST_OUT_OF_BOUNDS;
    bool active = valid && status < 0;
    if (!active) { // keep the arithmetic of idle lanes finite and in range
        px = 0.f;
        py = 0.f;
    }
    float gX = 0.f, gY = 0.f, dX = 0.f, dY = 0.f;
    bool conv0 = false;
    int it_total = 0;

    float T[PPLMAX], GX[PPLMAX], GY[PPLMAX];
    int off[PPLMAX];

    for (int l = P.L - 1; l >= 0; --l) {
        if (!wave_any(active)) break;
        const LevelPair LV = P.lv[l];
        const int Wl = LV.W, Hl = LV.H;
        const float sc = __builtin_ldexpf(1.0f, -l);
        const float plx = px * sc, ply = py * sc;
        const float pbx = floorf(plx), pby = floorf(ply);
        const float pfx = plx - pbx, pfy = ply - pby;
        const int ibx = (int)pbx - r, iby = (int)pby - r; // integer origin of the support

        // ---- template: stage I0_l over the support plus a one-pixel ring, (s+3)^2 floats
        wave_sync();
        for (int c = li; c < RW * RW; c += LPP) {
            const int ty = (int)(((float)c + 0.5f) * P.invRW);
            const int tx = c - ty * RW;
            tile[c] = load_px<PixT>(LV.p0, LV.pitch0, clampi(ibx - 1 + tx, 0, Wl - 1), clampi(iby - 1 + ty, 0, Hl - 1));
        }
        wave_sync();
        const float w00 = (1.f - pfx) * (1.f - pfy), w10 = pfx * (1.f - pfy);
        const float w01 = (1.f - pfx) * pfy, w11 = pfx * pfy;
        float a = 0.f, b = 0.f, c = 0.f;
#pragma unroll
        for (int j = 0; j < PPLMAX; ++j) {
            if (j < ppl) {
                const int k = j * LPP + li;
                const bool vk = k < S2;
                const int kk = vk ? k : 0;
                const int ky = kk / s, kx = kk - ky * s;
                // clamped tap positions, in raw-tile coordinates (tile origin = support origin - 1)
                const int cx0 = clampi(ibx + kx, 0, Wl - 1), cx1 = clampi(ibx + kx + 1, 0, Wl - 1);
                const int cy0 = clampi(iby + ky, 0, Hl - 1), cy1 = clampi(iby + ky + 1, 0, Hl - 1);
                const int tx0 = cx0 - ibx + 1, tx1 = cx1 - ibx + 1, ty0 = cy0 - iby + 1, ty1 = cy1 - iby + 1;
                const int lx0 = clampi(cx0 - 1, 0, Wl - 1) - ibx + 1, rx0 = clampi(cx0 + 1, 0, Wl - 1) - ibx + 1;
                const int lx1 = clampi(cx1 - 1, 0, Wl - 1) - ibx + 1, rx1 = clampi(cx1 + 1, 0, Wl - 1) - ibx + 1;
                const int uy0 = clampi(cy0 - 1, 0, Hl - 1) - iby + 1, dy0 = clampi(cy0 + 1, 0, Hl - 1) - iby + 1;
                const int uy1 = clampi(cy1 - 1, 0, Hl - 1) - iby + 1, dy1 = clampi(cy1 + 1, 0, Hl - 1) - iby + 1;
                const float v00 = tile[ty0 * RW + tx0], v10 = tile[ty0 * RW + tx1];
                const float v01 = tile[ty1 * RW + tx0], v11 = tile[ty1 * RW + tx1];
                const float gx00 = 0.5f * (tile[ty0 * RW + rx0] - tile[ty0 * RW + lx0]);
                const float gx10 = 0.5f * (tile[ty0 * RW + rx1] - tile[ty0 * RW + lx1]);
                const float gx01 = 0.5f * (tile[ty1 * RW + rx0] - tile[ty1 * RW + lx0]);
                const float gx11 = 0.5f * (tile[ty1 * RW + rx1] - tile[ty1 * RW + lx1]);
                const float gy00 = 0.5f * (tile[dy0 * RW + tx0] - tile[uy0 * RW + tx0]);
                const float gy10 = 0.5f * (tile[dy0 * RW + tx1] - tile[uy0 * RW + tx1]);
                const float gy01 = 0.5f * (tile[dy1 * RW + tx0] - tile[uy1 * RW + tx0]);
                const float gy11 = 0.5f * (tile[dy1 * RW + tx1] - tile[uy1 * RW + tx1]);
                const float tv = w00 * v00 + w10 * v10 + w01 * v01 + w11 * v11;
                const float gxv = w00 * gx00 + w10 * gx10 + w01 * gx01 + w11 * gx11;
                const float gyv = w00 * gy00 + w10 * gy10 + w01 * gy01 + w11 * gy11;
                T[j] = vk ? tv : 0.f;
                GX[j] = vk ? gxv : 0.f;
                GY[j] = vk ? gyv : 0.f;
                off[j] = vk ? ky * TW + kx : 0;
                a = fmaf(GX[j], GX[j], a);
                b = fmaf(GX[j], GY[j], b);
                c = fmaf(GY[j], GY[j], c);
            }
        }
        a = group_sum<LPP>(a);
        b = group_sum<LPP>(b);
        c = group_sum<LPP>(c);
        const float lam = 0.5f * (a + c) - sqrtf(0.25f * (a - c) * (a - c) + b * b);
        if (active && !(lam >= P.min_eig_s2)) {
            status = DGF_ST_ILL_CONDITIONED;
            ux = __builtin_ldexpf(gX, l);
            uy = __builtin_ldexpf(gY, l);
            active = false;
        }
        const float det0 = a * c - b * b;
        const float eps2 = (l > 0) ? P.eps2c : P.eps2f;

        // ---- iterations
        dX = 0.f;
        dY = 0.f;
        bool lvl_active = active, lvl_conv = false;
        int ox1 = 0, oy1 = 0; // origin of the staged I1 tile
        for (int it = 0; it < P.iters; ++it) {
            if (!wave_any(lvl_active)) break;
            const float tx = pfx + (gX + dX), ty = pfy + (gY + dY);
            float flx = floorf(tx), fly = floorf(ty);
            const float fx = tx - flx, fy = ty - fly;
            flx = fminf(fmaxf(flx, -1048576.f), 1048576.f);
            fly = fminf(fmaxf(fly, -1048576.f), 1048576.f);
            const int bx = (int)pbx + (int)flx - r, by = (int)pby + (int)fly - r;
            int dxo = bx - ox1, dyo = by - oy1;
            const bool inr = dxo >= 0 && dxo <= 2 * M && dyo >= 0 && dyo <= 2 * M;
            if (wave_any((it == 0) || (lvl_active && !inr))) { // every point re-stages at its position
                wave_sync();
                ox1 = bx - M;
                oy1 = by - M;
                for (int cc = li; cc < TW * TW; cc += LPP) {
                    const int yy = (int)(((float)cc + 0.5f) * P.invTW);
                    const int xx = cc - yy * TW;
                    tile[cc] = load_px<PixT>(LV.p1, LV.pitch1, clampi(ox1 + xx, 0, Wl - 1), clampi(oy1 + yy, 0, Hl - 1));
                }
                wave_sync();
                dxo = M;
                dyo = M;
            } else if (!inr) { // a stopped point that drifted off its tile reads a harmless in-range spot
                dxo = 0;
                dyo = 0;
            }
            const float *tb = tile + dyo * TW + dxo;
            const float q00 = (1.f - fx) * (1.f - fy), q10 = fx * (1.f - fy), q01 = (1.f - fx) * fy, q11 = fx * fy;
            float G11 = 0.f, G12 = 0.f, G22 = 0.f, B1 = 0.f, B2 = 0.f;
#pragma unroll
            for (int j = 0; j < PPLMAX; ++j) {
                if (j < ppl) {
                    const float *tp = tb + off[j];
                    const float J = q00 * tp[0] + q10 * tp[1] + q01 * tp[TW] + q11 * tp[TW + 1];
                    const float res = J - T[j];
                    const float ar = fabsf(res);
                    const float wmid = P.cmid * (P.s2 - ar) * __builtin_amdgcn_rcpf(ar);
                    const float w = (ar <= P.s1) ? 1.f : ((ar < P.s2) ? wmid : 0.f);
                    const float ps = w * res;
                    const float wgx = w * GX[j], wgy = w * GY[j];
                    G11 = fmaf(wgx, GX[j], G11);
                    G12 = fmaf(wgx, GY[j], G12);
                    G22 = fmaf(wgy, GY[j], G22);
                    B1 = fmaf(ps, GX[j], B1);
                    B2 = fmaf(ps, GY[j], B2);
                }
            }
            G11 = group_sum<LPP>(G11);
            G12 = group_sum<LPP>(G12);
            G22 = group_sum<LPP>(G22);
            B1 = group_sum<LPP>(B1);
            B2 = group_sum<LPP>(B2);
            float det = G11 * G22 - G12 * G12;
            const bool fb = lvl_active && !(det > 1e-6f * det0);
            if (wave_any(fb)) { // too many down-weighted pixels: least-squares step for those points
                float C1 = 0.f, C2 = 0.f;
#pragma unroll
                for (int j = 0; j < PPLMAX; ++j) {
                    if (j < ppl) {
                        const float *tp = tb + off[j];
                        const float J = q00 * tp[0] + q10 * tp[1] + q01 * tp[TW] + q11 * tp[TW + 1];
                        const float res = J - T[j];
                        C1 = fmaf(res, GX[j], C1);
                        C2 = fmaf(res, GY[j], C2);
                    }
                }
                C1 = group_sum<LPP>(C1);
                C2 = group_sum<LPP>(C2);
                if (fb) {
                    G11 = a;
                    G12 = b;
                    G22 = c;
                    B1 = C1;
                    B2 = C2;
                    det = det0;
                }
            }
            const float sx = (G12 * B2 - G22 * B1) / det;
            const float sy = (G12 * B1 - G11 * B2) / det;
            if (lvl_active) {
                ++it_total;
                if (!(isfinite(sx) && isfinite(sy))) {
                    status = DGF_ST_NOT_CONVERGED;
                    ux = __builtin_nanf("");
                    uy = __builtin_nanf("");
                    active = false;
                    lvl_active = false;
                } else {
                    dX += sx;
                    dY += sy;
                    if (sx * sx + sy * sy < eps2) {
                        lvl_conv = true;
                        lvl_active = false;
                    }
                }
            }
        }
        if (l > 0) {
            if (active) {
                gX = 2.f * (gX + dX);
                gY = 2.f * (gY + dY);
            }
        } else {
            conv0 = lvl_conv;
        }
    }

    if (valid && li == 0) {
        if (status < 0) {
            ux = gX + dX;
            uy = gY + dY;
            if (!conv0) {
                status = DGF_ST_NOT_CONVERGED;
            } else {
                const float qx = px + ux, qy = py + uy;
                status = (qx >= 0.f && qy >= 0.f && qx <= (float)(W0 - 1) && qy <= (float)(H0 - 1)) ? DGF_ST_CONVERGED
                                                                                                 : DGF_ST_OUT_OF_BOUNDS;
            }
        }
        reinterpret_cast<float2 *>(P.flow)[pidx] = make_float2(ux, uy);
        P.status[pidx] = (uint8_t)status;
        if (P.iters_out) P.iters_out[pidx] = it_total;
    }
}

// ------------------------------------------------------------------------------------------
// host side
// ------------------------------------------------------------------------------------------

static const int kPplSteps[] = {2, 4, 8, 16};

int pick_ppl_max(int s, int lpp)
{
    const int need = (s * s + lpp - 1) / lpp;
    for (int v : kPplSteps)
        if (need <= v) return v;
    return -1;
}

void fill_track_geometry(TrackParams &P, int s, int margin, int lpp)
{
    P.s = s;
    P.r = s / 2;
    P.M = margin;
    P.TW = s + 1 + 2 * margin;
    P.RW = s + 3;
    P.tile_floats = (P.TW > P.RW ? P.TW * P.TW : P.RW * P.RW);
    P.invTW = 1.0f / (float)P.TW;
    P.invRW = 1.0f / (float)P.RW;
    P.ppl = (s * s + lpp - 1) / lpp;
}

size_t track_lds_bytes(int s, const TrackTuning &T)
{
    TrackParams P{};
    fill_track_geometry(P, s, T.margin, T.lpp);
    return (size_t)T.wpb * (64 / T.lpp) * P.tile_floats * sizeof(float);
}

template <int LPP, int PPLMAX, typename PixT>
static hipError_t launch_one(const TrackParams &P, int wpb, hipStream_t st)
{
    constexpr int PPW = 64 / LPP;
    const int64_t waves = (P.n + PPW - 1) / PPW;
    const int64_t blocks = (waves + wpb - 1) / wpb;
    const size_t lds = (size_t)wpb * PPW * P.tile_floats * sizeof(float);
    hipLaunchKernelGGL((k_track<LPP, PPLMAX, PixT>), dim3((unsigned)blocks), dim3(64 * wpb), lds, st, P);
    return hipGetLastError();
}

template <int LPP, typename PixT>
static hipError_t dispatch_ppl(const TrackParams &P, int pplmax, int wpb, hipStream_t st)
{
    switch (pplmax) {
    case 2: return launch_one<LPP, 2, PixT>(P, wpb, st);
    case 4: return launch_one<LPP, 4, PixT>(P, wpb, st);
    case 8: return launch_one<LPP, 8, PixT>(P, wpb, st);
    case 16: return launch_one<LPP, 16, PixT>(P, wpb, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename PixT>
static hipError_t dispatch_lpp(const TrackParams &P, const TrackTuning &T, int pplmax, hipStream_t st)
{
    switch (T.lpp) {
    case 16: return dispatch_ppl<16, PixT>(P, pplmax, T.wpb, st);
    case 32: return dispatch_ppl<32, PixT>(P, pplmax, T.wpb, st);
    case 64: return dispatch_ppl<64, PixT>(P, pplmax, T.wpb, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_track(const TrackParams &P, const TrackTuning &T, int dtype, hipStream_t st)
{
    if (P.n <= 0) return hipSuccess;
    const int pplmax = pick_ppl_max(P.s, T.lpp);
    if (pplmax < 0) return hipErrorInvalidValue;
    if (dtype == DGF_U8) return dispatch_lpp<uint8_t>(P, T, pplmax, st);
    return dispatch_lpp<float>(P, T, pplmax, st);
}

} // namespace dgf
