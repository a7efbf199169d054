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
// One point per wavefront: lanes stride over the s x s support; pass 1 accumulates the four
// entries of J (wave reduction), every lane solves the 2x2 system, pass 2 scatters its pixels'
// contributions with hardware float atomics into the caller's dI0 / dI1 (accumulated, so one
// buffer can collect several pairs or calls).  Atomic order is not deterministic; the sums are
// equal up to FP32 rounding.
#include <cmath>

#include "dgf_internal.hpp"

namespace dgf {

struct AdjParams {
    const uint8_t *I0, *I1;
    int64_t pitch0, pitch1; // bytes, also the row pitch of dI0 / dI1
    int32_t W, H, s, r;
    const float *pts, *flow, *dflow;
    const uint8_t *status;
    float *dI0, *dI1;
    int64_t n;
    float s1, s2, dpsi_mid; // thresholds and the middle-band slope -sigma1 / (sigma2 - sigma1)
    int32_t mode;
};

__device__ __forceinline__ float f32_at(const uint8_t *base, int64_t pitch, int x, int y)
{
    return reinterpret_cast<const float *>(base + (int64_t)y * pitch)[x];
}

__device__ __forceinline__ void add_at(float *base, int64_t pitch, int x, int y, float v)
{
    unsafeAtomicAdd(reinterpret_cast<float *>(reinterpret_cast<uint8_t *>(base) + (int64_t)y * pitch) + x, v);
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

__global__ __launch_bounds__(64) void k_track_adjoint(AdjParams A)
{
    const int li = threadIdx.x;
    const int64_t i = blockIdx.x;
    if (i >= A.n) return; // whole wave: the grid is exactly n wide
    if (A.status[i] != DGF_ST_CONVERGED) return;
    const float2 p = reinterpret_cast<const float2 *>(A.pts)[i];
    const float2 u = reinterpret_cast<const float2 *>(A.flow)[i];
    const float2 lam = reinterpret_cast<const float2 *>(A.dflow)[i];
    const int W = A.W, H = A.H, s = A.s, r = A.r, S2 = s * s;

    // integer bases and shared fractions of the template samples (p + k) and the I1 samples
    const float pbx = floorf(p.x), pby = floorf(p.y);
    const float fx0 = p.x - pbx, fy0 = p.y - pby;
    const float tx = fx0 + u.x, ty = fy0 + u.y;
    const float qbx = floorf(tx), qby = floorf(ty);
    const float fx1 = tx - qbx, fy1 = ty - qby;
    const int ibx = (int)pbx - r, iby = (int)pby - r;
    const int jbx = (int)pbx + (int)fminf(fmaxf(qbx, -1048576.f), 1048576.f) - r;
    const int jby = (int)pby + (int)fminf(fmaxf(qby, -1048576.f), 1048576.f) - r;
    const float a00 = (1.f - fx0) * (1.f - fy0), a10 = fx0 * (1.f - fy0), a01 = (1.f - fx0) * fy0, a11 = fx0 * fy0;
    const float b00 = (1.f - fx1) * (1.f - fy1), b10 = fx1 * (1.f - fy1), b01 = (1.f - fx1) * fy1, b11 = fx1 * fy1;

    auto I0s = [&](int x, int y) { // bilinear of I0 with taps at integer (x, x+1) x (y, y+1), clamped
        const int x0 = clampi(x, 0, W - 1), x1 = clampi(x + 1, 0, W - 1);
        const int y0 = clampi(y, 0, H - 1), y1 = clampi(y + 1, 0, H - 1);
        return a00 * f32_at(A.I0, A.pitch0, x0, y0) + a10 * f32_at(A.I0, A.pitch0, x1, y0) +
               a01 * f32_at(A.I0, A.pitch0, x0, y1) + a11 * f32_at(A.I0, A.pitch0, x1, y1);
    };

    // pass 1: J = sum psi' g (grad J)^T
    float J00 = 0.f, J01 = 0.f, J10 = 0.f, J11 = 0.f;
    for (int k = li; k < S2; k += 64) {
        const int ky = k / s, kx = k - ky * s;
        const int x = ibx + kx, y = iby + ky;
        const float T = I0s(x, y);
        const float g0 = 0.5f * (I0s(x + 1, y) - I0s(x - 1, y));
        const float g1 = 0.5f * (I0s(x, y + 1) - I0s(x, y - 1));
        const int x0 = clampi(jbx + kx, 0, W - 1), x1 = clampi(jbx + kx + 1, 0, W - 1);
        const int y0 = clampi(jby + ky, 0, H - 1), y1 = clampi(jby + ky + 1, 0, H - 1);
        const float i00 = f32_at(A.I1, A.pitch1, x0, y0), i10 = f32_at(A.I1, A.pitch1, x1, y0);
        const float i01 = f32_at(A.I1, A.pitch1, x0, y1), i11 = f32_at(A.I1, A.pitch1, x1, y1);
        const float J = b00 * i00 + b10 * i10 + b01 * i01 + b11 * i11;
        const float djx = (1.f - fy1) * (i10 - i00) + fy1 * (i11 - i01);
        const float djy = (1.f - fx1) * (i01 - i00) + fx1 * (i11 - i10);
        float ps, dps;
        psi_and_slope(A, J - T, ps, dps);
        J00 = fmaf(dps * g0, djx, J00);
        J01 = fmaf(dps * g0, djy, J01);
        J10 = fmaf(dps * g1, djx, J10);
        J11 = fmaf(dps * g1, djy, J11);
    }
    float z = 0.f;
    wave_sum5(J00, J01, J10, J11, z);
    const float det = J00 * J11 - J01 * J10;
    if (!(det != 0.f) || !isfinite(det)) return; // uniform across the wave
    // J^T mu = lambda, J^T = [[J00, J10], [J01, J11]]
    const float mux = (J11 * lam.x - J10 * lam.y) / det;
    const float muy = (J00 * lam.y - J01 * lam.x) / det;

    // pass 2: scatter
    for (int k = li; k < S2; k += 64) {
        const int ky = k / s, kx = k - ky * s;
        const int x = ibx + kx, y = iby + ky;
        const float T = I0s(x, y);
        const float g0 = 0.5f * (I0s(x + 1, y) - I0s(x - 1, y));
        const float g1 = 0.5f * (I0s(x, y + 1) - I0s(x, y - 1));
        const int x0 = clampi(jbx + kx, 0, W - 1), x1 = clampi(jbx + kx + 1, 0, W - 1);
        const int y0 = clampi(jby + ky, 0, H - 1), y1 = clampi(jby + ky + 1, 0, H - 1);
        const float J = b00 * f32_at(A.I1, A.pitch1, x0, y0) + b10 * f32_at(A.I1, A.pitch1, x1, y0) +
                        b01 * f32_at(A.I1, A.pitch1, x0, y1) + b11 * f32_at(A.I1, A.pitch1, x1, y1);
        float ps, dps;
        psi_and_slope(A, J - T, ps, dps);
        const float c1 = dps * (mux * g0 + muy * g1);
        // dI1: - psi' (mu . g) beta
        add_at(A.dI1, A.pitch1, x0, y0, -c1 * b00);
        add_at(A.dI1, A.pitch1, x1, y0, -c1 * b10);
        add_at(A.dI1, A.pitch1, x0, y1, -c1 * b01);
        add_at(A.dI1, A.pitch1, x1, y1, -c1 * b11);
        // dI0 on the 4 x 4 neighbourhood of the template sample: +c1 alpha at the sample, and
        // -psi mu_x / 2 (alpha^{+x} - alpha^{-x}) - psi mu_y / 2 (alpha^{+y} - alpha^{-y})
        const float cx = -0.5f * ps * mux, cy = -0.5f * ps * muy;
        const float wa[4] = {a00, a10, a01, a11};
        const int ox[4] = {0, 1, 0, 1}, oy[4] = {0, 0, 1, 1};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int xt = x + ox[t], yt = y + oy[t];
            const float w = wa[t];
            add_at(A.dI0, A.pitch0, clampi(xt, 0, W - 1), clampi(yt, 0, H - 1), c1 * w);
            add_at(A.dI0, A.pitch0, clampi(xt + 1, 0, W - 1), clampi(yt, 0, H - 1), cx * w);
            add_at(A.dI0, A.pitch0, clampi(xt - 1, 0, W - 1), clampi(yt, 0, H - 1), -cx * w);
            add_at(A.dI0, A.pitch0, clampi(xt, 0, W - 1), clampi(yt + 1, 0, H - 1), cy * w);
            add_at(A.dI0, A.pitch0, clampi(xt, 0, W - 1), clampi(yt - 1, 0, H - 1), -cy * w);
        }
    }
}

hipError_t launch_track_adjoint(const AdjParams &A, hipStream_t st)
{
    if (A.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_track_adjoint, dim3((unsigned)A.n), dim3(64), 0, st, A);
    return hipGetLastError();
}

} // namespace dgf

extern "C" int dgf_track_backward(const dgf_image *I0, const dgf_image *I1, const float *points, int64_t n,
                                  int32_t support, const dgf_track_opts *opts, const float *flow,
                                  const uint8_t *status, const float *dflow, float *dI0, float *dI1, void *stream)
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
        if (o.flags != 0) return DGF_ERR_UNSUPPORTED;
    } else {
        dgf_track_opts_default(&o);
    }
    if (!(o.sigma1 >= 0.f) || !(o.sigma2 >= 0.f)) return DGF_ERR_INVALID_ARG;
    if (std::isinf(o.sigma2) && !std::isinf(o.sigma1)) return DGF_ERR_INVALID_ARG;
    if (n == 0) return DGF_OK;
    AdjParams A{};
    A.I0 = (const uint8_t *)I0->data;
    A.I1 = (const uint8_t *)I1->data;
    A.pitch0 = I0->pitch_bytes;
    A.pitch1 = I1->pitch_bytes;
    A.W = I0->width;
    A.H = I0->height;
    A.s = support;
    A.r = support / 2;
    A.pts = points;
    A.flow = flow;
    A.dflow = dflow;
    A.status = status;
    A.dI0 = dI0;
    A.dI1 = dI1;
    A.n = n;
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
    return launch_track_adjoint(A, (hipStream_t)stream) == hipSuccess ? DGF_OK : DGF_ERR_HIP;
}
