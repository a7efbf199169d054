// adjoint.hip -- gradient of the tracked flow w.r.t. both images on gfx950.
//
// At a converged point the level-0 flow u satisfies F(u; I0, I1) = sum_k psi(r_k) g_k = 0 with
// r_k = B(I1, p + k + u) - B(I0, p + k) and g_k the central differences at +-1 px of B(I0, .).
// Implicit differentiation gives, for an upstream gradient lambda = dL/du,
//     J = dF/du = sum_k psi'(r_k) g_k grad B(I1, p + k + u)^T,     J^T mu = lambda,
//     dL/dI1[q] = - sum_k psi'(r_k) (mu . g_k) beta_k(q)
//     dL/dI0[q] = + sum_k psi'(r_k) (mu . g_k) alpha_k(q)
//                 - sum_k psi(r_k) / 2 [mu_x (alpha_k^{+x} - alpha_k^{-x}) + mu_y (alpha_k^{+y} - alpha_k^{-y})](q)
// where alpha, beta are bilinear tap weights (taps clamped to the image, so border taps fold
// onto border pixels).  Only the level-0 images enter: the coarser levels decide which fixed
// point is reached, not its local dependence on the pixels.
//
// One point per wavefront (a one-wave workgroup).  The raw I0 patch (s+3)^2 around the template
// and the raw I1 patch (s+1)^2 under the tracked position are staged in LDS; lanes stride over the
// s x s support.  Pass 1 accumulates the four entries of J (wave reduction) and every lane solves
// the 2x2 system.  Pass 2 stores, per support pixel k, c1_k = psi'(r_k) (mu . g_k) and
// cx_k, cy_k = -psi(r_k) mu_x / 2, -psi(r_k) mu_y / 2.  The image gradients are then gathered
// rather than scattered (LDS float atomics serialise): with F(a) = c1(a) + cx(a - e_x) -
// cx(a + e_x) + cy(a - e_y) - cy(a + e_y) on the support grid,
//     dI0 cell X = sum over the 4 bilinear taps t of alpha_t F(X - (1, 1) - t),
//     dI1 cell X = - sum over the 4 taps t of beta_t c1(X - t),
// and every cell goes to the gradient map with one device float atomic at its clamped image
// position (neighbouring points overlap, so the device atomics stay).  Atomic order is not
// deterministic; sums agree up to FP32 rounding.  The batched form runs every point of a batch
// plan in one launch; a wavefront finds its pair by binary search over the plan's point offsets.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "dgf_internal.hpp"

namespace dgf {

// Value of the bilinear interpolant in the 2 x 2 cell whose top-left texel is q (row pitch w) at
// fraction (fx, fy), as nested linear interpolations: a constant cell gives exactly its value, so
// residuals between flat regions of integer frames are exact and a residual exactly on a robust
// threshold takes the same band as in any other exact evaluation.
__device__ __forceinline__ float lerp_cell(const float *q, int w, float fx, float fy)
{
    const float h0 = fmaf(fx, q[1] - q[0], q[0]);
    const float h1 = fmaf(fx, q[w + 1] - q[w], q[w]);
    return fmaf(fy, h1 - h0, h0);
}

// psi(r) and psi'(r) of the robust norm, band by band
__device__ __forceinline__ void psi_and_slope(const AdjParams &A, float r, float &ps, float &dps)
{
    const float a = fabsf(r);
    if (A.mode == ROBUST_L2 || a <= A.s1) {
        ps = r;
        dps = 1.f;
    } else if (A.mode == ROBUST_HARD || a >= A.s2) {
        ps = 0.f;
        dps = 0.f;
    } else {
        ps = copysignf(A.s1 * (A.s2 - a) / (A.s2 - A.s1), r);
        dps = A.dpsi_mid;
    }
}

__device__ __forceinline__ int adj_pair_of(const AdjParams &A, int64_t i)
{
    int lo = 0, hi = A.npairs - 1; // last pair whose first point is <= i
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (A.pt_off[mid] <= i)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

template <typename PixT>
__global__ __launch_bounds__(64) void k_track_adjoint(AdjParams A)
{
    extern __shared__ float smem[];
    const int li = threadIdx.x;
    const int64_t i = (int64_t)(((uint64_t)blockIdx.x * (uint64_t)A.perm_mul) % (uint64_t)A.n);
    if (A.dpoints && li == 0) reinterpret_cast<float2 *>(A.dpoints)[i] = make_float2(0.f, 0.f);
    if (A.status[i] != DGF_ST_CONVERGED) return;
    const AdjPair Pr = A.npairs ? A.pairs[adj_pair_of(A, i)] : A.one;
    const float2 p = reinterpret_cast<const float2 *>(A.pts)[i];
    const float2 u = reinterpret_cast<const float2 *>(A.flow)[i];
    const float2 lam = reinterpret_cast<const float2 *>(A.dflow)[i];
    const int W = Pr.W, H = Pr.H, s = A.s, r = A.r, S2 = s * s;

    // integer bases and shared fractions of the template samples (p + k) and the I1 samples
    const float pbx = floorf(p.x), pby = floorf(p.y);
    const float fx0 = p.x - pbx, fy0 = p.y - pby;
    const float tx = fx0 + u.x, ty = fy0 + u.y;
    const float qbx = floorf(tx), qby = floorf(ty);
    const float fx1 = tx - qbx, fy1 = ty - qby;
    const int ox0 = (int)pbx - r - 1, oy0 = (int)pby - r - 1; // dI0 patch origin, (s+3)^2
    const int ox1 = (int)pbx + (int)fminf(fmaxf(qbx, -1048576.f), 1048576.f) - r;
    const int oy1 = (int)pby + (int)fminf(fmaxf(qby, -1048576.f), 1048576.f) - r; // dI1 patch, (s+1)^2
    const float a00 = (1.f - fx0) * (1.f - fy0), a10 = fx0 * (1.f - fy0), a01 = (1.f - fx0) * fy0, a11 = fx0 * fy0;
    const float b00 = (1.f - fx1) * (1.f - fy1), b10 = fx1 * (1.f - fy1), b01 = (1.f - fx1) * fy1, b11 = fx1 * fy1;

    // LDS: raw I0 patch (later F on the (s+2)^2 grid), raw I1 patch, then c1, cx, cy on the support
    const int w0 = s + 3, w1 = s + 1, n0 = w0 * w0, n1 = w1 * w1;
    float *raw0 = smem, *raw1 = smem + n0, *C1 = raw1 + n1, *CX = C1 + S2, *CY = CX + S2;
    stage_rect<64, PixT>(raw0, w0, Pr.I0, Pr.pitch0, W, H, ox0, oy0, w0, w0, stage_lanes<64>(w0, li));
    stage_rect<64, PixT>(raw1, w1, Pr.I1, Pr.pitch1, W, H, ox1, oy1, w1, w1, stage_lanes<64>(w1, li));
    __syncthreads();

    // template value and central differences of the bilinear interpolant, from the raw I0 patch;
    // support offset (kx, ky) sits at local (kx + 1, ky + 1)
    auto I0s = [&](int lx, int ly) { return lerp_cell(raw0 + ly * w0 + lx, w0, fx0, fy0); };

    // gradient of the bilinear interpolant of I0 inside the cell at local (lx, ly)
    auto I0g = [&](int lx, int ly, float &gx, float &gy) {
        const float *q = raw0 + ly * w0 + lx;
        gx = (1.f - fy0) * (q[1] - q[0]) + fy0 * (q[w0 + 1] - q[w0]);
        gy = (1.f - fx0) * (q[w0] - q[0]) + fx0 * (q[w0 + 1] - q[1]);
    };

    // the norm of the equation the forward pass stopped on: where its weighted 2 x 2 system falls
    // back at the converged flow (det of sum w g g^T, w = psi(r) / r, at most 1e-6 of the
    // unweighted one's, or not a number) the fixed point solves sum r g = 0, so psi(r) = r
    bool ls = false;
    if (A.mode != ROBUST_L2) {
        float a = 0.f, b = 0.f, c = 0.f, a0 = 0.f, b0 = 0.f, c0 = 0.f;
        for (int k = li; k < S2; k += 64) {
            const int ky = k / s, kx = k - ky * s;
            const int lx = kx + 1, ly = ky + 1;
            const float g0 = 0.5f * (I0s(lx + 1, ly) - I0s(lx - 1, ly));
            const float g1 = 0.5f * (I0s(lx, ly + 1) - I0s(lx, ly - 1));
            const float res = lerp_cell(raw1 + ky * w1 + kx, w1, fx1, fy1) - I0s(lx, ly);
            float ps, dps;
            psi_and_slope(A, res, ps, dps);
            const float w = res != 0.f ? ps / res : 1.f;
            a = fmaf(w * g0, g0, a);
            b = fmaf(w * g0, g1, b);
            c = fmaf(w * g1, g1, c);
            a0 = fmaf(g0, g0, a0);
            b0 = fmaf(g0, g1, b0);
            c0 = fmaf(g1, g1, c0);
        }
        float z = 0.f;
        wave_sum5(a, b, c, a0, b0);
        wave_sum5(c0, z, z, z, z);
        ls = !(fmaf(a, c, -b * b) > 1e-6f * fmaf(a0, c0, -b0 * b0));
    }
    auto psi_at = [&](float res, float &ps, float &dps) {
        if (ls) {
            ps = res;
            dps = 1.f;
        } else {
            psi_and_slope(A, res, ps, dps);
        }
    };

    // pass 1: J = sum psi' g (grad J)^T; with dpoints also K = sum -psi' g (grad T)^T + psi dG/dx
    // (the dependence of F on the point: dF/dp = J + K)
    const bool want_dp = A.dpoints != nullptr;
    float J00 = 0.f, J01 = 0.f, J10 = 0.f, J11 = 0.f;
    float K00 = 0.f, K01 = 0.f, K10 = 0.f, K11 = 0.f;
    for (int k = li; k < S2; k += 64) {
        const int ky = k / s, kx = k - ky * s;
        const int lx = kx + 1, ly = ky + 1;
        const float T = I0s(lx, ly);
        const float g0 = 0.5f * (I0s(lx + 1, ly) - I0s(lx - 1, ly));
        const float g1 = 0.5f * (I0s(lx, ly + 1) - I0s(lx, ly - 1));
        const float *q = raw1 + ky * w1 + kx;
        const float i00 = q[0], i10 = q[1], i01 = q[w1], i11 = q[w1 + 1];
        const float J = lerp_cell(q, w1, fx1, fy1);
        const float djx = (1.f - fy1) * (i10 - i00) + fy1 * (i11 - i01);
        const float djy = (1.f - fx1) * (i01 - i00) + fx1 * (i11 - i10);
        float ps, dps;
        psi_at(J - T, ps, dps);
        J00 = fmaf(dps * g0, djx, J00);
        J01 = fmaf(dps * g0, djy, J01);
        J10 = fmaf(dps * g1, djx, J10);
        J11 = fmaf(dps * g1, djy, J11);
        if (want_dp) {
            float tgx, tgy, pxx, pxy, mxx, mxy, pyx, pyy, myx, myy;
            I0g(lx, ly, tgx, tgy);
            I0g(lx + 1, ly, pxx, pxy);
            I0g(lx - 1, ly, mxx, mxy);
            I0g(lx, ly + 1, pyx, pyy);
            I0g(lx, ly - 1, myx, myy);
            K00 += -dps * g0 * tgx + 0.5f * ps * (pxx - mxx);
            K01 += -dps * g0 * tgy + 0.5f * ps * (pxy - mxy);
            K10 += -dps * g1 * tgx + 0.5f * ps * (pyx - myx);
            K11 += -dps * g1 * tgy + 0.5f * ps * (pyy - myy);
        }
    }
    float z = 0.f;
    wave_sum5(J00, J01, J10, J11, z);
    if (want_dp) wave_sum5(K00, K01, K10, K11, z);
    const float det = J00 * J11 - J01 * J10;
    if (!(det != 0.f) || !isfinite(det)) return; // uniform across the wave
    // J^T mu = lambda, J^T = [[J00, J10], [J01, J11]]
    const float mux = (J11 * lam.x - J10 * lam.y) / det;
    const float muy = (J00 * lam.y - J01 * lam.x) / det;
    // du/dp = -J^-1 (J + K), so dL/dp = -lambda - K^T mu
    if (want_dp && li == 0)
        reinterpret_cast<float2 *>(A.dpoints)[i] =
            make_float2(-lam.x - (K00 * mux + K10 * muy), -lam.y - (K01 * mux + K11 * muy));

    // pass 2: per support pixel, c1 = psi' (mu . g) and cx, cy = -psi mu / 2
    for (int k = li; k < S2; k += 64) {
        const int ky = k / s, kx = k - ky * s;
        const int lx = kx + 1, ly = ky + 1;
        const float T = I0s(lx, ly);
        const float g0 = 0.5f * (I0s(lx + 1, ly) - I0s(lx - 1, ly));
        const float g1 = 0.5f * (I0s(lx, ly + 1) - I0s(lx, ly - 1));
        const float *q = raw1 + ky * w1 + kx;
        const float J = lerp_cell(q, w1, fx1, fy1);
        float ps, dps;
        psi_at(J - T, ps, dps);
        C1[k] = dps * (mux * g0 + muy * g1);
        CX[k] = -0.5f * ps * mux;
        CY[k] = -0.5f * ps * muy;
    }
    __syncthreads();
    auto at = [&](const float *f, int a, int b) { // field value at support (a, b), zero outside
        return (a >= 0 && a < s && b >= 0 && b < s) ? f[b * s + a] : 0.f;
    };
    // F on the support grid extended by one ring, a, b in [-1, s], stored at (a + 1, b + 1) with
    // pitch s + 2 over the raw I0 patch (no longer read)
    const int wf = s + 2;
    float *F = raw0;
    for (int c = li; c < wf * wf; c += 64) {
        const int b = c / wf - 1, a = c - (b + 1) * wf - 1;
        F[c] = at(C1, a, b) + at(CX, a - 1, b) - at(CX, a + 1, b) + at(CY, a, b - 1) - at(CY, a, b + 1);
    }
    // dI1 cells: - sum of the 4 taps of c1
    float *dI1 = A.grad1 + Pr.g1;
    for (int c = li; c < n1; c += 64) {
        const int Y = c / w1, X = c - Y * w1;
        const float v = -(b00 * at(C1, X, Y) + b10 * at(C1, X - 1, Y) + b01 * at(C1, X, Y - 1) + b11 * at(C1, X - 1, Y - 1));
        if (v != 0.f)
            unsafeAtomicAdd(dI1 + (int64_t)clampi(oy1 + Y, 0, H - 1) * Pr.gpitch1 + clampi(ox1 + X, 0, W - 1), v);
    }
    __syncthreads();
    // dI0 cells: the 4 bilinear taps of F; cell X reads F at support X - (1, 1) - t, stored at X - t
    float *dI0 = A.grad0 + Pr.g0;
    for (int c = li; c < n0; c += 64) {
        const int Y = c / w0, X = c - Y * w0;
        auto f = [&](int x, int y) { return (x >= 0 && x < wf && y >= 0 && y < wf) ? F[y * wf + x] : 0.f; };
        const float v = a00 * f(X, Y) + a10 * f(X - 1, Y) + a01 * f(X, Y - 1) + a11 * f(X - 1, Y - 1);
        if (v != 0.f)
            unsafeAtomicAdd(dI0 + (int64_t)clampi(oy0 + Y, 0, H - 1) * Pr.gpitch0 + clampi(ox0 + X, 0, W - 1), v);
    }
}

// k_track_adjoint for a support size fixed at compile time (no illumination model): the same
// quantities by the same formulas, arranged for fewer instructions.  The bilinearly resampled I0
// patch on the (S + 2)^2 grid of support offsets -r-1 .. r+1 is built once in LDS, and every
// lane computes its pixels' template gradient, I1 sample and gradient, residual and psi band once
// (NS slots of 64 pixels) and keeps them in registers for the fallback-regime test and both
// passes; the fields c1, cx, cy and F sit in LDS arrays with a zero border, so the gathers read
// them without bounds tests; divisions by the support size are by a constant.
template <typename PixT, int S>
__global__ __launch_bounds__(64) void k_track_adjoint_fixed(AdjParams A)
{
    constexpr int r = S / 2, S2 = S * S, NS = (S2 + 63) / 64;
    constexpr int w0 = S + 3, w1 = S + 1, n0 = w0 * w0, n1 = w1 * w1;
    constexpr int G = S + 2;      // resampled grid: support offsets -r-1 .. r+1
    constexpr int PC = S + 4;     // c1, cx, cy with a zero border of 2: support (a, b) at (a + 2, b + 2)
    constexpr int PF = S + 4;     // F with a zero border of 1: grid (x, y) at (x + 1, y + 1)
    extern __shared__ float smem[];
    const int li = threadIdx.x;
    const int64_t i = (int64_t)(((uint64_t)blockIdx.x * (uint64_t)A.perm_mul) % (uint64_t)A.n);
    if (A.dpoints && li == 0) reinterpret_cast<float2 *>(A.dpoints)[i] = make_float2(0.f, 0.f);
    if (A.status[i] != DGF_ST_CONVERGED) return;
    const AdjPair Pr = A.npairs ? A.pairs[adj_pair_of(A, i)] : A.one;
    const float2 p = reinterpret_cast<const float2 *>(A.pts)[i];
    const float2 u = reinterpret_cast<const float2 *>(A.flow)[i];
    const float2 lam = reinterpret_cast<const float2 *>(A.dflow)[i];
    const int W = Pr.W, H = Pr.H;

    const float pbx = floorf(p.x), pby = floorf(p.y);
    const float fx0 = p.x - pbx, fy0 = p.y - pby;
    const float tx = fx0 + u.x, ty = fy0 + u.y;
    const float qbx = floorf(tx), qby = floorf(ty);
    const float fx1 = tx - qbx, fy1 = ty - qby;
    const int ox0 = (int)pbx - r - 1, oy0 = (int)pby - r - 1;
    const int ox1 = (int)pbx + (int)fminf(fmaxf(qbx, -1048576.f), 1048576.f) - r;
    const int oy1 = (int)pby + (int)fminf(fmaxf(qby, -1048576.f), 1048576.f) - r;
    const float a00 = (1.f - fx0) * (1.f - fy0), a10 = fx0 * (1.f - fy0), a01 = (1.f - fx0) * fy0, a11 = fx0 * fy0;
    const float b00 = (1.f - fx1) * (1.f - fy1), b10 = fx1 * (1.f - fy1), b01 = (1.f - fx1) * fy1, b11 = fx1 * fy1;

    // LDS: region 0 holds the raw patches, then c1, cx, cy; region 1 the grid, then F
    float *raw0 = smem, *raw1 = smem + n0;
    float *C1 = smem, *CX = C1 + PC * PC, *CY = CX + PC * PC;
    float *grid = smem + 3 * PC * PC, *F = grid;
    stage_rect<64, PixT>(raw0, w0, Pr.I0, Pr.pitch0, W, H, ox0, oy0, w0, w0, stage_lanes<64>(w0, li));
    stage_rect<64, PixT>(raw1, w1, Pr.I1, Pr.pitch1, W, H, ox1, oy1, w1, w1, stage_lanes<64>(w1, li));
    __syncthreads();
    for (int c = li; c < G * G; c += 64) {
        const int y = c / G, x = c - y * G;
        grid[c] = lerp_cell(raw0 + y * w0 + x, w0, fx0, fy0);
    }
    __syncthreads();

    // per slot: the pixel's template central differences, I1 gradient, residual and psi band
    float g0[NS], g1[NS], djx[NS], djy[NS], res[NS], ps[NS], dps[NS];
#pragma unroll
    for (int t = 0; t < NS; ++t) {
        const int k = li + 64 * t;
        const bool in = k < S2;
        const int kk = in ? k : 0;
        const int ky = kk / S, kx = kk - ky * S;
        const float *gc = grid + (ky + 1) * G + kx + 1;
        const float T = gc[0];
        g0[t] = in ? 0.5f * (gc[1] - gc[-1]) : 0.f;
        g1[t] = in ? 0.5f * (gc[G] - gc[-G]) : 0.f;
        const float *q = raw1 + ky * w1 + kx;
        const float i00 = q[0], i10 = q[1], i01 = q[w1], i11 = q[w1 + 1];
        const float J = lerp_cell(q, w1, fx1, fy1);
        djx[t] = (1.f - fy1) * (i10 - i00) + fy1 * (i11 - i01);
        djy[t] = (1.f - fx1) * (i01 - i00) + fx1 * (i11 - i10);
        res[t] = J - T;
        psi_and_slope(A, res[t], ps[t], dps[t]);
        if (!in) {
            ps[t] = 0.f;
            dps[t] = 0.f;
        }
    }
    // the norm of the equation the forward pass stopped on (as in k_track_adjoint)
    if (A.mode != ROBUST_L2) {
        float a = 0.f, b = 0.f, c = 0.f, a0 = 0.f, b0 = 0.f, c0 = 0.f;
#pragma unroll
        for (int t = 0; t < NS; ++t) {
            const float w = res[t] != 0.f ? ps[t] / res[t] : 1.f;
            a = fmaf(w * g0[t], g0[t], a);
            b = fmaf(w * g0[t], g1[t], b);
            c = fmaf(w * g1[t], g1[t], c);
            a0 = fmaf(g0[t], g0[t], a0);
            b0 = fmaf(g0[t], g1[t], b0);
            c0 = fmaf(g1[t], g1[t], c0);
        }
        float z = 0.f;
        wave_sum5(a, b, c, a0, b0);
        wave_sum5(c0, z, z, z, z);
        if (!(fmaf(a, c, -b * b) > 1e-6f * fmaf(a0, c0, -b0 * b0))) {
#pragma unroll
            for (int t = 0; t < NS; ++t) {
                const bool in = li + 64 * t < S2;
                ps[t] = in ? res[t] : 0.f;
                dps[t] = in ? 1.f : 0.f;
            }
        }
    }

    // pass 1: J = sum psi' g (grad J)^T; with dpoints also K (see k_track_adjoint)
    const bool want_dp = A.dpoints != nullptr;
    float J00 = 0.f, J01 = 0.f, J10 = 0.f, J11 = 0.f;
    float K00 = 0.f, K01 = 0.f, K10 = 0.f, K11 = 0.f;
#pragma unroll
    for (int t = 0; t < NS; ++t) {
        J00 = fmaf(dps[t] * g0[t], djx[t], J00);
        J01 = fmaf(dps[t] * g0[t], djy[t], J01);
        J10 = fmaf(dps[t] * g1[t], djx[t], J10);
        J11 = fmaf(dps[t] * g1[t], djy[t], J11);
    }
    if (want_dp) {
        auto I0g = [&](int lx, int ly, float &gx, float &gy) {
            const float *q = raw0 + ly * w0 + lx;
            gx = (1.f - fy0) * (q[1] - q[0]) + fy0 * (q[w0 + 1] - q[w0]);
            gy = (1.f - fx0) * (q[w0] - q[0]) + fx0 * (q[w0 + 1] - q[1]);
        };
#pragma unroll
        for (int t = 0; t < NS; ++t) {
            const int k = li + 64 * t;
            if (k < S2) {
                const int ky = k / S, kx = k - ky * S, lx = kx + 1, ly = ky + 1;
                float tgx, tgy, pxx, pxy, mxx, mxy, pyx, pyy, myx, myy;
                I0g(lx, ly, tgx, tgy);
                I0g(lx + 1, ly, pxx, pxy);
                I0g(lx - 1, ly, mxx, mxy);
                I0g(lx, ly + 1, pyx, pyy);
                I0g(lx, ly - 1, myx, myy);
                K00 += -dps[t] * g0[t] * tgx + 0.5f * ps[t] * (pxx - mxx);
                K01 += -dps[t] * g0[t] * tgy + 0.5f * ps[t] * (pxy - mxy);
                K10 += -dps[t] * g1[t] * tgx + 0.5f * ps[t] * (pyx - myx);
                K11 += -dps[t] * g1[t] * tgy + 0.5f * ps[t] * (pyy - myy);
            }
        }
    }
    float z = 0.f;
    wave_sum5(J00, J01, J10, J11, z);
    if (want_dp) wave_sum5(K00, K01, K10, K11, z);
    const float det = J00 * J11 - J01 * J10;
    if (!(det != 0.f) || !isfinite(det)) return; // uniform across the wave
    const float mux = (J11 * lam.x - J10 * lam.y) / det;
    const float muy = (J00 * lam.y - J01 * lam.x) / det;
    if (want_dp && li == 0)
        reinterpret_cast<float2 *>(A.dpoints)[i] =
            make_float2(-lam.x - (K00 * mux + K10 * muy), -lam.y - (K01 * mux + K11 * muy));

    // pass 2: c1, cx, cy on the support, zero around it (the raw patches are no longer read)
    __syncthreads();
    for (int c = li; c < 3 * PC * PC; c += 64) C1[c] = 0.f;
    __syncthreads();
#pragma unroll
    for (int t = 0; t < NS; ++t) {
        const int k = li + 64 * t;
        if (k < S2) {
            const int ky = k / S, kx = k - ky * S, e = (ky + 2) * PC + kx + 2;
            C1[e] = dps[t] * (mux * g0[t] + muy * g1[t]);
            CX[e] = -0.5f * ps[t] * mux;
            CY[e] = -0.5f * ps[t] * muy;
        }
    }
    __syncthreads();
    // F on the support grid extended by one ring (a, b in [-1, S]), zero around it; the grid is no
    // longer read
    for (int c = li; c < PF * PF; c += 64) {
        const int y = c / PF, x = c - y * PF; // F index (x - 1, y - 1) = support (x - 2, y - 2)
        float v = 0.f;
        if (x >= 1 && x <= G && y >= 1 && y <= G) {
            const float *e = C1 + y * PC + x; // support (x - 2, y - 2) sits at (x, y)
            v = e[0] + CX[y * PC + x - 1] - CX[y * PC + x + 1] + CY[(y - 1) * PC + x] - CY[(y + 1) * PC + x];
        }
        F[c] = v;
    }
    // dI1 cells: - sum of the 4 taps of c1 (cell X reads support X - t at padded X - t + 2)
    float *dI1 = A.grad1 + Pr.g1;
    for (int c = li; c < n1; c += 64) {
        const int Y = c / w1, X = c - Y * w1;
        const float *e = C1 + (Y + 2) * PC + X + 2;
        const float v = -(b00 * e[0] + b10 * e[-1] + b01 * e[-PC] + b11 * e[-PC - 1]);
        if (v != 0.f)
            unsafeAtomicAdd(dI1 + (int64_t)clampi(oy1 + Y, 0, H - 1) * Pr.gpitch1 + clampi(ox1 + X, 0, W - 1), v);
    }
    __syncthreads();
    // dI0 cells: the 4 bilinear taps of F; cell X reads F index X - t, padded at X - t + 1
    float *dI0 = A.grad0 + Pr.g0;
    for (int c = li; c < n0; c += 64) {
        const int Y = c / w0, X = c - Y * w0;
        const float *f = F + (Y + 1) * PF + X + 1;
        const float v = a00 * f[0] + a10 * f[-1] + a01 * f[-PF] + a11 * f[-PF - 1];
        if (v != 0.f)
            unsafeAtomicAdd(dI0 + (int64_t)clampi(oy0 + Y, 0, H - 1) * Pr.gpitch0 + clampi(ox0 + X, 0, W - 1), v);
    }
}

// 4x4 system M^T x = v by Gaussian elimination with partial pivoting, fully unrolled (M row-major,
// both copied); x is not finite when a pivot is zero.
__device__ __forceinline__ void solve4_transposed(const float *M, const float *v, float *x)
{
    float a[4][5];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
        for (int c = 0; c < 4; ++c) a[r][c] = M[c * 4 + r];
        a[r][4] = v[r];
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        // pivot: largest |a[r][c]| for r >= c, brought to row c by selects (no dynamic indexing)
#pragma unroll
        for (int r = c + 1; r < 4; ++r) {
            const bool sw = fabsf(a[r][c]) > fabsf(a[c][c]);
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                const float t = a[c][k];
                a[c][k] = sw ? a[r][k] : t;
                a[r][k] = sw ? t : a[r][k];
            }
        }
        const float inv = 1.f / a[c][c];
#pragma unroll
        for (int r = c + 1; r < 4; ++r) {
            const float f = a[r][c] * inv;
#pragma unroll
            for (int k = c; k < 5; ++k) a[r][k] = fmaf(-f, a[c][k], a[r][k]);
        }
    }
#pragma unroll
    for (int r = 3; r >= 0; --r) {
        float acc = a[r][4];
#pragma unroll
        for (int k = r + 1; k < 4; ++k) acc = fmaf(-a[r][k], x[k], acc);
        x[r] = acc / a[r][r];
    }
}

// Adjoint of the illumination-model tracker.  At a converged point theta = (u, m, c) solves
// F = sum_k psi(r_k) phi_k = 0, r_k = J_k - (1 + m) T_k - c, phi_k = ((1 + m) g_k, -T_k, -1).
// The solve runs on the centred template T' = (T - Tm) / Ts on both sides -- a constant change of
// the equations' basis (F' = R F) and of the (m, c) parameters, which leaves dL/dI unchanged at the
// fixed point and conditions the FP32 4x4 system:
//   A = sum_k psi'(r_k) phi'_k (grad J_k, -T'_k, -1)^T with phi'_k = ((1 + m) g_k, -T'_k, -1)
//   (the psi g term of the m column is (1 + m)^-1 times the d rows of F and vanishes here),
//   A^T mu = (dL/du, 0, 0),
//   dI1 -= psi' (mu . phi') beta,
//   dI0 += [(1 + m) psi' (mu . phi') + psi mu_m / Ts] alpha - (1 + m) psi mu_d . dg/dI0.
// The image gradients are gathered as in k_track_adjoint, with the sample term A0 apart from c1.
template <typename PixT>
__global__ __launch_bounds__(64) void k_track_adjoint_illum(AdjParams A)
{
    extern __shared__ float smem[];
    const int li = threadIdx.x;
    const int64_t i = (int64_t)(((uint64_t)blockIdx.x * (uint64_t)A.perm_mul) % (uint64_t)A.n);
    if (A.dpoints && li == 0) reinterpret_cast<float2 *>(A.dpoints)[i] = make_float2(0.f, 0.f);
    if (A.status[i] != DGF_ST_CONVERGED) return;
    const AdjPair Pr = A.npairs ? A.pairs[adj_pair_of(A, i)] : A.one;
    const float2 p = reinterpret_cast<const float2 *>(A.pts)[i];
    const float2 u = reinterpret_cast<const float2 *>(A.flow)[i];
    const float2 lam = reinterpret_cast<const float2 *>(A.dflow)[i];
    const float2 mc = reinterpret_cast<const float2 *>(A.illum)[i];
    const float g1m = 1.f + mc.x;
    const int W = Pr.W, H = Pr.H, s = A.s, r = A.r, S2 = s * s;

    const float pbx = floorf(p.x), pby = floorf(p.y);
    const float fx0 = p.x - pbx, fy0 = p.y - pby;
    const float tx = fx0 + u.x, ty = fy0 + u.y;
    const float qbx = floorf(tx), qby = floorf(ty);
    const float fx1 = tx - qbx, fy1 = ty - qby;
    const int ox0 = (int)pbx - r - 1, oy0 = (int)pby - r - 1;
    const int ox1 = (int)pbx + (int)fminf(fmaxf(qbx, -1048576.f), 1048576.f) - r;
    const int oy1 = (int)pby + (int)fminf(fmaxf(qby, -1048576.f), 1048576.f) - r;
    const float a00 = (1.f - fx0) * (1.f - fy0), a10 = fx0 * (1.f - fy0), a01 = (1.f - fx0) * fy0, a11 = fx0 * fy0;
    const float b00 = (1.f - fx1) * (1.f - fy1), b10 = fx1 * (1.f - fy1), b01 = (1.f - fx1) * fy1, b11 = fx1 * fy1;

    const int w0 = s + 3, w1 = s + 1, n0 = w0 * w0, n1 = w1 * w1;
    float *raw0 = smem, *raw1 = smem + n0, *C1 = raw1 + n1, *CX = C1 + S2, *CY = CX + S2, *A0 = CY + S2;
    stage_rect<64, PixT>(raw0, w0, Pr.I0, Pr.pitch0, W, H, ox0, oy0, w0, w0, stage_lanes<64>(w0, li));
    stage_rect<64, PixT>(raw1, w1, Pr.I1, Pr.pitch1, W, H, ox1, oy1, w1, w1, stage_lanes<64>(w1, li));
    __syncthreads();
    auto I0s = [&](int lx, int ly) { return lerp_cell(raw0 + ly * w0 + lx, w0, fx0, fy0); };

    // template mean and spread over the support
    float sT = 0.f, sTT = 0.f, z0 = 0.f, z1 = 0.f, z2 = 0.f;
    for (int k = li; k < S2; k += 64) {
        const int ky = k / s, kx = k - ky * s;
        const float T = I0s(kx + 1, ky + 1);
        sT += T;
        sTT = fmaf(T, T, sTT);
    }
    wave_sum5(sT, sTT, z0, z1, z2);
    const float Tm = sT / (float)S2;
    float Ts = sqrtf(fmaxf(sTT / (float)S2 - Tm * Tm, 0.f));
    if (!(Ts > 1e-6f)) Ts = 1.f;
    const float iTs = 1.f / Ts;

    auto I0g = [&](int lx, int ly, float &gx, float &gy) {
        const float *q = raw0 + ly * w0 + lx;
        gx = (1.f - fy0) * (q[1] - q[0]) + fy0 * (q[w0 + 1] - q[w0]);
        gy = (1.f - fx0) * (q[w0] - q[0]) + fx0 * (q[w0 + 1] - q[1]);
    };

    // the norm of the equations the forward pass stopped on: where its weighted 4 x 4 system falls
    // back at the converged (u, m, c) (det of sum w phi phi^T at most 1e-6 of the unweighted one's,
    // or not a number; the ratio is the same in the centred and scaled template used here) the
    // fixed point solves the least-squares equations, so psi(r) = r
    bool ls = false;
    if (A.mode != ROBUST_L2) {
        float G[10], G0[10];
#pragma unroll
        for (int e = 0; e < 10; ++e) {
            G[e] = 0.f;
            G0[e] = 0.f;
        }
        for (int k = li; k < S2; k += 64) {
            const int ky = k / s, kx = k - ky * s;
            const int lx = kx + 1, ly = ky + 1;
            const float T = I0s(lx, ly);
            const float g0 = 0.5f * (I0s(lx + 1, ly) - I0s(lx - 1, ly));
            const float g1 = 0.5f * (I0s(lx, ly + 1) - I0s(lx, ly - 1));
            const float res = lerp_cell(raw1 + ky * w1 + kx, w1, fx1, fy1) - g1m * T - mc.y;
            float ps, dps;
            psi_and_slope(A, res, ps, dps);
            const float w = res != 0.f ? ps / res : 1.f;
            const float ph[4] = {g1m * g0, g1m * g1, -(T - Tm) * iTs, -1.f};
            int e = 0;
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = a; b < 4; ++b, ++e) {
                    G[e] = fmaf(w * ph[a], ph[b], G[e]);
                    G0[e] = fmaf(ph[a], ph[b], G0[e]);
                }
        }
        float z = 0.f;
        wave_sum5(G[0], G[1], G[2], G[3], G[4]);
        wave_sum5(G[5], G[6], G[7], G[8], G[9]);
        wave_sum5(G0[0], G0[1], G0[2], G0[3], G0[4]);
        wave_sum5(G0[5], G0[6], G0[7], G0[8], G0[9]);
        (void)z;
        ls = !(ldl4(G, nullptr, nullptr) > 1e-6f * ldl4(G0, nullptr, nullptr));
    }
    auto psi_at = [&](float res, float &ps, float &dps) {
        if (ls) {
            ps = res;
            dps = 1.f;
        } else {
            psi_and_slope(A, res, ps, dps);
        }
    };

    // pass 1: A = sum psi' phi' (grad J, -T', -1)^T; with dpoints also the point dependence
    // K = sum -(1 + m) psi' phi' (grad T)^T + psi dphi'/dp, dphi'/dp = ((1 + m) dg/dp,
    // -(grad T)^T / Ts, 0) (rows u_x, u_y, m, c; columns p_x, p_y)
    const bool want_dp = A.dpoints != nullptr;
    float Kp[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) Kp[e] = 0.f;
    float Am[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) Am[e] = 0.f;
    for (int k = li; k < S2; k += 64) {
        const int ky = k / s, kx = k - ky * s;
        const int lx = kx + 1, ly = ky + 1;
        const float T = I0s(lx, ly);
        const float g0 = 0.5f * (I0s(lx + 1, ly) - I0s(lx - 1, ly));
        const float g1 = 0.5f * (I0s(lx, ly + 1) - I0s(lx, ly - 1));
        const float *q = raw1 + ky * w1 + kx;
        const float i00 = q[0], i10 = q[1], i01 = q[w1], i11 = q[w1 + 1];
        const float J = lerp_cell(q, w1, fx1, fy1);
        const float djx = (1.f - fy1) * (i10 - i00) + fy1 * (i11 - i01);
        const float djy = (1.f - fx1) * (i01 - i00) + fx1 * (i11 - i10);
        float ps, dps;
        psi_at(J - g1m * T - mc.y, ps, dps);
        const float Tp = (T - Tm) * iTs;
        const float ph[4] = {g1m * g0, g1m * g1, -Tp, -1.f};
        const float dr[4] = {djx, djy, -Tp, -1.f};
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) Am[a * 4 + b] = fmaf(dps * ph[a], dr[b], Am[a * 4 + b]);
        if (want_dp) {
            float tgx, tgy, pxx, pxy, mxx, mxy, pyx, pyy, myx, myy;
            I0g(lx, ly, tgx, tgy);
            I0g(lx + 1, ly, pxx, pxy);
            I0g(lx - 1, ly, mxx, mxy);
            I0g(lx, ly + 1, pyx, pyy);
            I0g(lx, ly - 1, myx, myy);
            const float cg = -g1m * dps, hp = 0.5f * g1m * ps;
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                Kp[2 * a] = fmaf(cg * ph[a], tgx, Kp[2 * a]);
                Kp[2 * a + 1] = fmaf(cg * ph[a], tgy, Kp[2 * a + 1]);
            }
            Kp[0] = fmaf(hp, pxx - mxx, Kp[0]);
            Kp[1] = fmaf(hp, pxy - mxy, Kp[1]);
            Kp[2] = fmaf(hp, pyx - myx, Kp[2]);
            Kp[3] = fmaf(hp, pyy - myy, Kp[3]);
            Kp[4] = fmaf(-ps * iTs, tgx, Kp[4]);
            Kp[5] = fmaf(-ps * iTs, tgy, Kp[5]);
        }
    }
    float zz = 0.f;
    wave_sum5(Am[0], Am[1], Am[2], Am[3], Am[4]);
    wave_sum5(Am[5], Am[6], Am[7], Am[8], Am[9]);
    wave_sum5(Am[10], Am[11], Am[12], Am[13], Am[14]);
    wave_sum5(Am[15], zz, z0, z1, z2);
    if (want_dp) {
        wave_sum5(Kp[0], Kp[1], Kp[2], Kp[3], Kp[4]);
        wave_sum5(Kp[5], Kp[6], Kp[7], z0, z1);
    }
    const float v[4] = {lam.x, lam.y, 0.f, 0.f};
    float mu[4];
    solve4_transposed(Am, v, mu);
    if (!(isfinite(mu[0]) && isfinite(mu[1]) && isfinite(mu[2]) && isfinite(mu[3]))) return; // uniform
    // du/dp = -I - (A^-1 K)[u rows], so dL/dp = -lambda - K^T mu
    if (want_dp && li == 0)
        reinterpret_cast<float2 *>(A.dpoints)[i] =
            make_float2(-lam.x - (Kp[0] * mu[0] + Kp[2] * mu[1] + Kp[4] * mu[2] + Kp[6] * mu[3]),
                        -lam.y - (Kp[1] * mu[0] + Kp[3] * mu[1] + Kp[5] * mu[2] + Kp[7] * mu[3]));

    // pass 2: per support pixel c1 = psi' (mu . phi'), A0 = (1 + m) c1 + psi mu_m / Ts,
    // cx, cy = -(1 + m) psi mu_d / 2
    for (int k = li; k < S2; k += 64) {
        const int ky = k / s, kx = k - ky * s;
        const int lx = kx + 1, ly = ky + 1;
        const float T = I0s(lx, ly);
        const float g0 = 0.5f * (I0s(lx + 1, ly) - I0s(lx - 1, ly));
        const float g1 = 0.5f * (I0s(lx, ly + 1) - I0s(lx, ly - 1));
        const float *q = raw1 + ky * w1 + kx;
        const float J = lerp_cell(q, w1, fx1, fy1);
        float ps, dps;
        psi_at(J - g1m * T - mc.y, ps, dps);
        const float Tp = (T - Tm) * iTs;
        const float mphi = g1m * (mu[0] * g0 + mu[1] * g1) - mu[2] * Tp - mu[3];
        const float c1 = dps * mphi;
        C1[k] = c1;
        A0[k] = g1m * c1 + ps * mu[2] * iTs;
        CX[k] = -0.5f * g1m * ps * mu[0];
        CY[k] = -0.5f * g1m * ps * mu[1];
    }
    __syncthreads();
    auto at = [&](const float *f, int a, int b) { return (a >= 0 && a < s && b >= 0 && b < s) ? f[b * s + a] : 0.f; };
    const int wf = s + 2;
    float *F = raw0;
    for (int c = li; c < wf * wf; c += 64) {
        const int b = c / wf - 1, a = c - (b + 1) * wf - 1;
        F[c] = at(A0, a, b) + at(CX, a - 1, b) - at(CX, a + 1, b) + at(CY, a, b - 1) - at(CY, a, b + 1);
    }
    float *dI1 = A.grad1 + Pr.g1;
    for (int c = li; c < n1; c += 64) {
        const int Y = c / w1, X = c - Y * w1;
        const float val = -(b00 * at(C1, X, Y) + b10 * at(C1, X - 1, Y) + b01 * at(C1, X, Y - 1) + b11 * at(C1, X - 1, Y - 1));
        if (val != 0.f)
            unsafeAtomicAdd(dI1 + (int64_t)clampi(oy1 + Y, 0, H - 1) * Pr.gpitch1 + clampi(ox1 + X, 0, W - 1), val);
    }
    __syncthreads();
    float *dI0 = A.grad0 + Pr.g0;
    for (int c = li; c < n0; c += 64) {
        const int Y = c / w0, X = c - Y * w0;
        auto f = [&](int x, int y) { return (x >= 0 && x < wf && y >= 0 && y < wf) ? F[y * wf + x] : 0.f; };
        const float val = a00 * f(X, Y) + a10 * f(X - 1, Y) + a01 * f(X, Y - 1) + a11 * f(X - 1, Y - 1);
        if (val != 0.f)
            unsafeAtomicAdd(dI0 + (int64_t)clampi(oy0 + Y, 0, H - 1) * Pr.gpitch0 + clampi(ox0 + X, 0, W - 1), val);
    }
}

size_t adjoint_lds_bytes(int s)
{
    return sizeof(float) * (size_t)((s + 3) * (s + 3) + (s + 1) * (s + 1) + 4 * s * s);
}

// Blocks take the points in a scattered order, point (b M) mod n for M coprime to n near 0.618 n:
// the waves in flight at any time then lie spread over the frames instead of covering a band a few
// point rows high, whose windows overlap tens of times and would queue their gradient atomics on
// the same addresses.  Each point is still taken exactly once.
static int64_t scatter_multiplier(int64_t n)
{
    int64_t m = std::max<int64_t>(1, (int64_t)llround(0.6180339887498949 * (double)n));
    while (std::gcd(m, n) != 1) ++m;
    return m;
}

hipError_t launch_track_adjoint(const AdjParams &A0, int dtype, hipStream_t st)
{
    if (A0.n <= 0) return hipSuccess;
    AdjParams A = A0;
    A.perm_mul = scatter_multiplier(A.n);
    const size_t lds = adjoint_lds_bytes(A.s);
    if (A.illum) {
        if (dtype == DGF_U8)
            hipLaunchKernelGGL(k_track_adjoint_illum<uint8_t>, dim3((unsigned)A.n), dim3(64), lds, st, A);
        else
            hipLaunchKernelGGL(k_track_adjoint_illum<float>, dim3((unsigned)A.n), dim3(64), lds, st, A);
    } else if (A.s == 21 || A.s == 9) {
        // the support sizes of the benchmark workloads: the fixed-size form
        const size_t lds_fixed = sizeof(float) * 4 * (size_t)(A.s + 4) * (A.s + 4);
        if (A.s == 21) {
            if (dtype == DGF_U8)
                hipLaunchKernelGGL((k_track_adjoint_fixed<uint8_t, 21>), dim3((unsigned)A.n), dim3(64), lds_fixed, st, A);
            else
                hipLaunchKernelGGL((k_track_adjoint_fixed<float, 21>), dim3((unsigned)A.n), dim3(64), lds_fixed, st, A);
        } else {
            if (dtype == DGF_U8)
                hipLaunchKernelGGL((k_track_adjoint_fixed<uint8_t, 9>), dim3((unsigned)A.n), dim3(64), lds_fixed, st, A);
            else
                hipLaunchKernelGGL((k_track_adjoint_fixed<float, 9>), dim3((unsigned)A.n), dim3(64), lds_fixed, st, A);
        }
    } else if (dtype == DGF_U8)
        hipLaunchKernelGGL(k_track_adjoint<uint8_t>, dim3((unsigned)A.n), dim3(64), lds, st, A);
    else
        hipLaunchKernelGGL(k_track_adjoint<float>, dim3((unsigned)A.n), dim3(64), lds, st, A);
    return hipGetLastError();
}

// Gradient of the DeGraF points w.r.t. the image, the centroid ratios of Eq. (1)-(2) taken as
// functions of real pixel values: one wavefront per window; the window maximum (first maximal
// pixel in row-major order), the weight sum and the centroid of the selected kind are reduced
// across the wave, then every pixel gets dL/dp . dp/dI with a device float atomic (neighbouring
// windows overlap when the stride is below the window).
__global__ __launch_bounds__(64) void k_detect_backward(DetectGradParams G)
{
    const int li = threadIdx.x;
    const int64_t n = blockIdx.x;
    if (n >= G.n) return;
    const float2 lam = reinterpret_cast<const float2 *>(G.dpoints)[n];
    if (lam.x == 0.f && lam.y == 0.f) return; // uniform: nothing to add
    const int x0 = (int)(n % G.nx) * G.stride, y0 = (int)(n / G.nx) * G.stride, w = G.win, A2 = w * w;
    const bool neg = G.sel[n] != 0;
    // window maximum and its first position (row-major)
    int best = -1, bidx = 0x7fffffff;
    for (int q = li; q < A2; q += 64) {
        const int i = q / w, j = q - i * w;
        const int v = G.img[(int64_t)(y0 + i) * G.pitch + x0 + j];
        if (v > best) { // q increases, so a tie keeps the earlier index
            best = v;
            bidx = q;
        }
    }
    for (int off = 32; off >= 1; off >>= 1) {
        const int ob = __shfl_xor(best, off), oi = __shfl_xor(bidx, off);
        if (ob > best || (ob == best && oi < bidx)) {
            best = ob;
            bidx = oi;
        }
    }
    const float m = (float)best;
    float S = 0.f, Si = 0.f, Sj = 0.f, z0 = 0.f, z1 = 0.f;
    for (int q = li; q < A2; q += 64) {
        const int i = q / w, j = q - i * w;
        const float v = (float)G.img[(int64_t)(y0 + i) * G.pitch + x0 + j];
        const float wv = neg ? 1.f + m - v : v;
        S += wv;
        Si = fmaf((float)i, wv, Si);
        Sj = fmaf((float)j, wv, Sj);
    }
    wave_sum5(S, Si, Sj, z0, z1);
    if (!(S != 0.f)) return;
    const float iS = 1.f / S, Ci = Si * iS, Cj = Sj * iS, cmid = 0.5f * (float)(w - 1);
    for (int q = li; q < A2; q += 64) {
        const int i = q / w, j = q - i * w;
        float di, dj;
        if (!neg) {
            di = ((float)i - Ci) * iS;
            dj = ((float)j - Cj) * iS;
        } else {
            di = -((float)i - Ci) * iS;
            dj = -((float)j - Cj) * iS;
            if (q == bidx) { // the maximum raises every weight of the negative centroid
                di += (float)A2 * (cmid - Ci) * iS;
                dj += (float)A2 * (cmid - Cj) * iS;
            }
        }
        const float v = lam.x * dj + lam.y * di;
        if (v != 0.f) unsafeAtomicAdd(G.dI + (int64_t)(y0 + i) * G.dpitch + x0 + j, v);
    }
}

hipError_t launch_detect_backward(const DetectGradParams &G, hipStream_t st)
{
    if (G.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_detect_backward, dim3((unsigned)G.n), dim3(64), 0, st, G);
    return hipGetLastError();
}

void fill_adjoint_constants(AdjParams &A, const dgf_track_opts &o)
{
    A.s1 = o.sigma1;
    A.s2 = o.sigma2;
    if (std::isinf(o.sigma1)) {
        A.mode = ROBUST_L2;
        A.dpsi_mid = 0.f;
    } else if (o.sigma2 > o.sigma1) {
        A.mode = ROBUST_HAMPEL;
        A.dpsi_mid = -o.sigma1 / (o.sigma2 - o.sigma1);
    } else {
        A.mode = ROBUST_HARD;
        A.dpsi_mid = 0.f;
    }
}

} // namespace dgf

extern "C" int dgf_track_backward(const dgf_image *I0, const dgf_image *I1, const float *points, int64_t n,
                                  int32_t support, const dgf_track_opts *opts, const float *flow,
                                  const uint8_t *status, const float *dflow, float *dI0, float *dI1, float *dpoints,
                                  const float *illum, void *stream)
{
    using namespace dgf;
    auto ok = [](const dgf_image *im) {
        return im && im->data && im->width >= 1 && im->height >= 1 && im->dtype == DGF_F32 &&
               im->pitch_bytes >= (int64_t)im->width * 4 && im->pitch_bytes % 4 == 0 && (uintptr_t)im->data % 4 == 0;
    };
    if (!I0 || !I1) return DGF_ERR_INVALID_ARG;
    if ((I0->dtype != DGF_F32 || I1->dtype != DGF_F32) && I0->data && I1->data) return DGF_ERR_UNSUPPORTED;
    if (!ok(I0) || !ok(I1)) return DGF_ERR_INVALID_ARG;
    if (I0->width != I1->width || I0->height != I1->height) return DGF_ERR_INVALID_ARG;
    if (support < 1 || (support & 1) == 0 || support > DGF_MAX_SUPPORT || n < 0) return DGF_ERR_INVALID_ARG;
    if (n > 0 && (!points || !flow || !status || !dflow || !dI0 || !dI1)) return DGF_ERR_INVALID_ARG;
    if ((uintptr_t)dI0 % 4 != 0 || (uintptr_t)dI1 % 4 != 0) return DGF_ERR_INVALID_ARG;
    dgf_track_opts o;
    if (opts) {
        o = *opts;
        // the global prior only moves where the iteration starts; cross-based supports are not differentiated
        if ((o.flags & ~(DGF_TRACK_ILLUM | DGF_TRACK_GLOBAL)) != 0) return DGF_ERR_UNSUPPORTED;
    } else {
        dgf_track_opts_default(&o);
    }
    const bool im = (o.flags & DGF_TRACK_ILLUM) != 0;
    if (im && n > 0 && !illum) return DGF_ERR_INVALID_ARG;
    if (!im && illum) return DGF_ERR_INVALID_ARG;
    if (!(o.sigma1 >= 0.f) || !(o.sigma2 >= 0.f)) return DGF_ERR_INVALID_ARG;
    if (std::isinf(o.sigma2) && !std::isinf(o.sigma1)) return DGF_ERR_INVALID_ARG;
    if (n == 0) return DGF_OK;
    AdjParams A{};
    A.one = AdjPair{(const uint8_t *)I0->data, (const uint8_t *)I1->data, I0->pitch_bytes, I1->pitch_bytes, 0, 0,
                    I0->pitch_bytes / 4, I1->pitch_bytes / 4, I0->width, I0->height};
    A.grad0 = dI0;
    A.grad1 = dI1;
    A.s = support;
    A.r = support / 2;
    A.pts = points;
    A.flow = flow;
    A.dflow = dflow;
    A.status = status;
    A.dpoints = dpoints;
    A.illum = im ? illum : nullptr;
    A.n = n;
    fill_adjoint_constants(A, o);
    return launch_track_adjoint(A, DGF_F32, (hipStream_t)stream) == hipSuccess ? DGF_OK : DGF_ERR_HIP;
}

extern "C" int dgf_detect_backward(const dgf_image *I0, int32_t window, int32_t stride, const uint8_t *sel,
                                   const float *dpoints, int64_t n, float *dI0, int64_t dI0_pitch, void *stream)
{
    using namespace dgf;
    if (!I0 || !I0->data || I0->dtype != DGF_U8 || I0->width < 1 || I0->height < 1 ||
        I0->pitch_bytes < I0->width || window < 1 || window > DGF_MAX_WINDOW || stride < 1)
        return DGF_ERR_INVALID_ARG;
    if (n != dgf_detect_count(I0->width, I0->height, window, stride)) return DGF_ERR_INVALID_ARG;
    if (n == 0) return DGF_OK;
    if (!sel || !dpoints || !dI0 || dI0_pitch < I0->width || (uintptr_t)dI0 % 4 != 0) return DGF_ERR_INVALID_ARG;
    DetectGradParams G{};
    G.img = (const uint8_t *)I0->data;
    G.pitch = I0->pitch_bytes;
    G.W = I0->width;
    G.H = I0->height;
    G.win = window;
    G.stride = stride;
    G.nx = (I0->width - window) / stride + 1;
    G.sel = sel;
    G.dpoints = dpoints;
    G.dI = dI0;
    G.dpitch = dI0_pitch;
    G.n = n;
    return launch_detect_backward(G, (hipStream_t)stream) == hipSuccess ? DGF_OK : DGF_ERR_HIP;
}
