// track_kernel.hpp -- pyramidal robust local optical flow tracking on gfx950 (device code).
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
//   * One point per group of LPP lanes (LPP = 16, 32 or 64: 4, 2 or 1 points per wavefront).
//     Support pixel k goes to lane k mod LPP, slot k / LPP; PPL = ceil(s^2 / LPP) slots per
//     lane is a compile-time constant, so the per-slot loop is straight-line code whose LDS
//     reads the compiler can issue ahead of the arithmetic.  Each lane keeps its slots' template
//     value, gradient and gradient products in registers for the whole level.
//   * All I1 samples of one iteration share one fractional offset (the support moves rigidly),
//     so the four bilinear weights are computed once per point and iteration.  The I1
//     neighbourhood of the support is staged in LDS as a (s + 1 + 2M)^2 float tile with row pitch
//     TP (a compile-time constant, so the two rows a bilinear sample needs are one ds_read2_b32
//     pair off a single address) and a margin of M pixels; it is re-staged only when the integer
//     part of the displacement drifts more than M pixels.
//   * The template is built from a bilinearly resampled copy of the border-replicated I0 patch
//     (shared weights): the template value and its central differences at +-1 px are direct
//     reads of that copy.
//   * The sums of the normal equations are reduced across the LPP lanes with DPP row
//     butterflies and the gfx950 row-swap permutes; the 2x2 solve is done redundantly by every
//     lane of the point, so no broadcast is needed.
//   * The least-squares limit (both thresholds infinite) skips the weights: the matrix is the
//     template's own G0 and only the two right-hand-side sums are accumulated and reduced.
//   * Points that have stopped keep executing with their updates masked until every point of
//     the wavefront has stopped.  Coordinates keep integer part and fraction apart.
// No MFMA: each point's system is 2x2, not a dense contraction.
#pragma once

#include "dgf_internal.hpp"

namespace dgf {

template <int TP>
struct Log2;
template <>
struct Log2<32> { static constexpr int v = 5; };
template <>
struct Log2<64> { static constexpr int v = 6; };

template <int LPP, int PPL, int TP, typename PixT>
__global__ __launch_bounds__(256) void k_track(TrackParams P)
{
    constexpr int PPW = 64 / LPP;
    constexpr int LTP = Log2<TP>::v;
    extern __shared__ float smem[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wpb = blockDim.x >> 6;
    const int q = lane / LPP;
    const int li = lane - q * LPP;
    float *tile = smem + (size_t)(wave * PPW + q) * P.tile_floats;

    const int s = P.s, r = P.r, S2 = s * s, RW = P.RW, RP = P.RPP, TW = P.TW, M = P.M;
    const StageLanes slR = stage_lanes<LPP>(RW, li), slT = stage_lanes<LPP>(TW, li);

    // slot geometry: off = ky * TP + kx (kx, ky in [0, s)); unused slots read offset 0 and
    // carry zero gradients, so they add nothing to any sum
    int off[PPL];
    unsigned vmask = 0u;
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
        const int k = j * LPP + li;
        const bool vk = k < S2;
        const int kk = vk ? k : 0;
        const int ky = kk / s, kx = kk - ky * s;
        off[j] = ky * TP + kx;
        vmask |= (vk ? 1u : 0u) << j;
    }

    float T[PPL], GX[PPL], GY[PPL], GXX[PPL], GXY[PPL], GYY[PPL];

    // Plain launches keep the hardware's order: block b on XCD b mod 8 spreads every image band
    // over all eight XCDs, which balances the uneven per-point work.  (Giving each XCD one band
    // cut L2 fills 4.6x on the 1242x375 benchmark pair but made the launch 25% longer.)
    // Persistent launches pull from the queue of their own XCD first.
    const int home = (int)(blockIdx.x % kNumXcd);
    int visit = 0;
    int64_t item = P.persistent ? next_item(P, home, visit) : (int64_t)blockIdx.x * wpb + wave;
    for (;;) {
    const WorkItem wi = work_item<PPW>(P, item, q);
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
    const LevelPair LV0 = level_of(P, pair, 0);
    const int W0 = LV0.W, H0 = LV0.H;
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


    for (int l = P.L - 1; l >= 0; --l) {
        if (!wave_any(active)) break;
        const LevelPair LV = level_of(P, pair, l);
        const int Wl = LV.W, Hl = LV.H;
        const float sc = __builtin_ldexpf(1.0f, -l);
        const float plx = px * sc, ply = py * sc;
        const float pbx = floorf(plx), pby = floorf(ply);
        const float pfx = plx - pbx, pfy = ply - pby;
        const int ibx = (int)pbx - r, iby = (int)pby - r; // integer origin of the support

        // ---- template: stage I0_l over the support plus a one-pixel ring (RW = s + 3 square,
        //      row pitch RP), with index clamping (replicated border)
        wave_sync();
        stage_rect<LPP, PixT>(tile, RP, LV.p0, LV.pitch0, Wl, Hl, ibx - 1, iby - 1, RW, RW, slR);
        wave_sync();
        const float w00 = (1.f - pfx) * (1.f - pfy), w10 = pfx * (1.f - pfy);
        const float w01 = (1.f - pfx) * pfy, w11 = pfx * pfy;
        {
            // resampled patch B[ty][tx] = bilinear(I0_l) at (ibx - 1 + tx + pfx, iby - 1 + ty + pfy);
            // the template value and its central differences at +-1 px are direct reads of B
            float *Bt = tile + RW * RP;
            const int BW = s + 2;
            for (int c = li; c < BW * BW; c += LPP) {
                const int ty = (int)(((float)c + 0.5f) * P.invBW);
                const int tx = c - ty * BW;
                const float *rp = tile + ty * RP + tx;
                Bt[ty * RP + tx] = w00 * rp[0] + w10 * rp[1] + w01 * rp[RP] + w11 * rp[RP + 1];
            }
            wave_sync();
#pragma unroll
            for (int j = 0; j < PPL; ++j) {
                const int ky = off[j] >> LTP, kx = off[j] & (TP - 1);
                const float *bp = Bt + (ky + 1) * RP + (kx + 1);
                const bool vk = (vmask >> j) & 1u;
                T[j] = vk ? bp[0] : 0.f;
                GX[j] = vk ? 0.5f * (bp[1] - bp[-1]) : 0.f;
                GY[j] = vk ? 0.5f * (bp[RP] - bp[-RP]) : 0.f;
            }
        }
        float a = 0.f, b = 0.f, c = 0.f;
#pragma unroll
        for (int j = 0; j < PPL; ++j) {
            GXX[j] = GX[j] * GX[j];
            GXY[j] = GX[j] * GY[j];
            GYY[j] = GY[j] * GY[j];
            a += GXX[j];
            b += GXY[j];
            c += GYY[j];
        }
        if constexpr (LPP == 64) {
            float z0 = 0.f, z1 = 0.f;
            wave_sum5(a, b, c, z0, z1);
        } else {
            a = group_sum<LPP>(a);
            b = group_sum<LPP>(b);
            c = group_sum<LPP>(c);
        }
        const float lam = 0.5f * (a + c) - sqrtf(fmaf(b, b, 0.25f * (a - c) * (a - c)));
        // too flat to invert: a coarse level runs no iteration and passes the guess on; at
        // level 0 the point is ill-conditioned with u = g
        const bool flat = active && !(lam >= P.min_eig_s2);
        if (flat && l == 0) {
            status = DGF_ST_ILL_CONDITIONED;
            ux = gX;
            uy = gY;
            active = false;
        }
        const float det0 = fmaf(a, c, -b * b);
        const float eps2 = (l > 0) ? P.eps2c : P.eps2f;

        // ---- iterations
        dX = 0.f;
        dY = 0.f;
        bool lvl_active = active && !flat, lvl_conv = false;
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
                stage_rect<LPP, PixT>(tile, TP, LV.p1, LV.pitch1, Wl, Hl, ox1, oy1, TW, TW, slT);
                wave_sync();
                dxo = M;
                dyo = M;
            } else if (!inr) { // a stopped point that drifted off its tile reads a harmless in-range spot
                dxo = 0;
                dyo = 0;
            }
            const float *tb = tile + dyo * TP + dxo;
            const float q00 = (1.f - fx) * (1.f - fy), q10 = fx * (1.f - fy), q01 = (1.f - fx) * fy, q11 = fx * fy;
            float G11, G12, G22, B1 = 0.f, B2 = 0.f, det;
            if (P.mode == ROBUST_L2) {
#pragma unroll
                for (int j = 0; j < PPL; ++j) {
                    const float *tp = tb + off[j];
                    const float res = fmaf(q11, tp[TP + 1], fmaf(q01, tp[TP], fmaf(q10, tp[1], fmaf(q00, tp[0], -T[j]))));
                    B1 = fmaf(res, GX[j], B1);
                    B2 = fmaf(res, GY[j], B2);
                }
                if constexpr (LPP == 64) {
                    float z0 = 0.f, z1 = 0.f, z2 = 0.f;
                    wave_sum5(B1, B2, z0, z1, z2);
                } else {
                    B1 = group_sum<LPP>(B1);
                    B2 = group_sum<LPP>(B2);
                }
                G11 = a;
                G12 = b;
                G22 = c;
                det = det0;
            } else {
                G11 = 0.f;
                G12 = 0.f;
                G22 = 0.f;
                if (P.mode == ROBUST_HAMPEL) {
#pragma unroll
                    for (int j = 0; j < PPL; ++j) {
                        const float *tp = tb + off[j];
                        const float res = fmaf(q11, tp[TP + 1], fmaf(q01, tp[TP], fmaf(q10, tp[1], fmaf(q00, tp[0], -T[j]))));
                        const float w = hampel_weight(res, P.cs2, P.cmid);
                        const float ps = w * res;
                        G11 = fmaf(w, GXX[j], G11);
                        G12 = fmaf(w, GXY[j], G12);
                        G22 = fmaf(w, GYY[j], G22);
                        B1 = fmaf(ps, GX[j], B1);
                        B2 = fmaf(ps, GY[j], B2);
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < PPL; ++j) {
                        const float *tp = tb + off[j];
                        const float res = fmaf(q11, tp[TP + 1], fmaf(q01, tp[TP], fmaf(q10, tp[1], fmaf(q00, tp[0], -T[j]))));
                        const float w = (fabsf(res) <= P.s1) ? 1.f : 0.f;
                        const float ps = w * res;
                        G11 = fmaf(w, GXX[j], G11);
                        G12 = fmaf(w, GXY[j], G12);
                        G22 = fmaf(w, GYY[j], G22);
                        B1 = fmaf(ps, GX[j], B1);
                        B2 = fmaf(ps, GY[j], B2);
                    }
                }
                if constexpr (LPP == 64) {
                    wave_sum5(G11, G12, G22, B1, B2);
                } else {
                    G11 = group_sum<LPP>(G11);
                    G12 = group_sum<LPP>(G12);
                    G22 = group_sum<LPP>(G22);
                    B1 = group_sum<LPP>(B1);
                    B2 = group_sum<LPP>(B2);
                }
                det = fmaf(G11, G22, -G12 * G12);
                const bool fb = lvl_active && !(det > 1e-6f * det0);
                if (wave_any(fb)) { // too many down-weighted pixels: least-squares step for those points
                    float C1 = 0.f, C2 = 0.f;
#pragma unroll
                    for (int j = 0; j < PPL; ++j) {
                        const float *tp = tb + off[j];
                        const float res = fmaf(q11, tp[TP + 1], fmaf(q01, tp[TP], fmaf(q10, tp[1], fmaf(q00, tp[0], -T[j]))));
                        C1 = fmaf(res, GX[j], C1);
                        C2 = fmaf(res, GY[j], C2);
                    }
                    if constexpr (LPP == 64) {
                        float z0 = 0.f, z1 = 0.f, z2 = 0.f;
                        wave_sum5(C1, C2, z0, z1, z2);
                    } else {
                        C1 = group_sum<LPP>(C1);
                        C2 = group_sum<LPP>(C2);
                    }
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
            const float sx = fmaf(G12, B2, -G22 * B1) * inv;
            const float sy = fmaf(G12, B1, -G11 * B2) * inv;
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
                    if (fmaf(sx, sx, sy * sy) < eps2) {
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
    if (!P.persistent) break;
    item = next_item(P, home, visit);
    } // work loop
}

template <int LPP, int PPL, int TP, typename PixT>
hipError_t launch_track_t(const TrackParams &P, int wpb, hipStream_t st)
{
    constexpr int PPW = 64 / LPP;
    const int64_t waves = P.npairs ? P.grid_waves : (P.n + PPW - 1) / PPW;
    const int64_t blocks = (waves + wpb - 1) / wpb;
    const size_t lds = (size_t)wpb * PPW * P.tile_floats * sizeof(float);
    hipLaunchKernelGGL((k_track<LPP, PPL, TP, PixT>), dim3((unsigned)blocks), dim3(64 * wpb), lds, st, P);
    return hipGetLastError();
}

// The (LPP, PPL, TP) shapes compiled for each element type: PPL = ceil(s^2 / LPP) for odd
// supports s; TP = 32 for s <= 21, 64 above.
#define DGF_TRACK_SHAPES(X, PixT)                                                                                      \
    X(64, 1, 32, PixT) X(64, 2, 32, PixT) X(64, 3, 32, PixT) X(64, 4, 32, PixT) X(64, 5, 32, PixT) X(64, 6, 32, PixT) \
    X(64, 7, 32, PixT) X(64, 9, 64, PixT) X(64, 10, 64, PixT) X(64, 12, 64, PixT) X(64, 14, 64, PixT)                 \
    X(64, 16, 64, PixT) X(32, 1, 32, PixT) X(32, 2, 32, PixT) X(32, 3, 32, PixT) X(32, 4, 32, PixT)                   \
    X(32, 6, 32, PixT) X(32, 8, 32, PixT) X(32, 10, 32, PixT) X(32, 12, 32, PixT) X(32, 14, 32, PixT)                 \
    X(16, 1, 32, PixT) X(16, 2, 32, PixT) X(16, 4, 32, PixT) X(16, 6, 32, PixT) X(16, 8, 32, PixT)                    \
    X(16, 11, 32, PixT) X(16, 15, 32, PixT)

} // namespace dgf
