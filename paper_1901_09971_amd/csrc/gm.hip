// gm.hip -- the global-motion prior's robust affine fit (the "GM" of RLOF(IM-GM), Section 3
// "Parameters"): one affine motion v = A (x - cx, y - cy, 1)^T per frame pair, fitted in FP64 to
// the motions of the points that the coarsest-level pass reports converged, by weighted least
// squares and then ten Tukey-biweight reweightings.
//
// One launch per weighting pass, each a grid of (nblk, npairs) workgroups.  Every workgroup first
// rebuilds the previous pass's model from the previous pass's partial sums (all workgroups of a pair
// reduce the same partials in the same order, so they agree bit for bit), then sums its slice of the
// pair's samples under the weights that model gives.  A last launch of one workgroup per pair turns
// the final partial sums into the model.  Models and partials are double-buffered by pass parity, so
// a launch only reads what the launch before it wrote: no atomics and no counters to clear, and the
// sequence can be captured into a graph.
#include <cmath>

#include "dgf_internal.hpp"

namespace dgf {

namespace {

// Weighted sums of one pass: S, Sx, Sy, Sxx, Sxy, Syy, Su, Sxu, Syu, Sv, Sxv, Syv and the number
// of samples of positive weight (x, y about the centre; u, v the sample motion).
enum { kS, kSx, kSy, kSxx, kSxy, kSyy, kSu, kSxu, kSyu, kSv, kSxv, kSyv, kNz };
static_assert(kNz + 1 == kGmSums, "sum layout");

constexpr int kThreads = 256;

// Sum of v[k] over the workgroup in a fixed order (lane butterflies, then the four wavefronts in
// turn); the result is in red[0][k] after the call.
__device__ void block_sum(double (&v)[kGmSums], double (*red)[kGmSums])
{
#pragma unroll
    for (int k = 0; k < kGmSums; ++k) {
        double x = v[k];
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
        v[k] = x;
    }
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < kGmSums; ++k) red[wave][k] = v[k];
    __syncthreads();
    if (threadIdx.x < kGmSums) {
        double x = red[0][threadIdx.x];
        for (int w = 1; w < kThreads / 64; ++w) x += red[w][threadIdx.x];
        red[0][threadIdx.x] = x;
    }
    __syncthreads();
}

// Model from one pass's sums.  `A` holds the previous model on entry and keeps it when no sample
// carries weight or the normal matrix is singular; with fewer than three samples, or positions
// whose weighted covariance C has det C <= 1e-4 (tr C)^2 (collinear), the model is the weighted
// mean motion.  Otherwise the 3 x 3 normal equations of both motion components are solved by
// Gaussian elimination with partial pivoting.
__device__ void gm_solve(const double *S, double *A)
{
    if (!(S[kNz] > 0.0)) return;
    const double is = 1.0 / S[kS];
    const double mx = S[kSx] * is, my = S[kSy] * is;
    const double cxx = S[kSxx] * is - mx * mx, cxy = S[kSxy] * is - mx * my, cyy = S[kSyy] * is - my * my;
    const double tr = cxx + cyy, det = cxx * cyy - cxy * cxy;
    if (S[kNz] < 3.0 || !(det > 1e-4 * tr * tr)) {
        A[0] = A[1] = A[3] = A[4] = 0.0;
        A[2] = S[kSu] / S[kS];
        A[5] = S[kSv] / S[kS];
        return;
    }
    // unknowns (slope in x, slope in y, offset), one right-hand side per motion component
    double N[3][5] = {{S[kSxx], S[kSxy], S[kSx], S[kSxu], S[kSxv]},
                      {S[kSxy], S[kSyy], S[kSy], S[kSyu], S[kSyv]},
                      {S[kSx], S[kSy], S[kS], S[kSu], S[kSv]}};
    for (int c = 0; c < 3; ++c) {
        int piv = c;
        for (int r = c + 1; r < 3; ++r)
            if (fabs(N[r][c]) > fabs(N[piv][c])) piv = r;
        if (!(fabs(N[piv][c]) > 0.0)) return;
        if (piv != c)
            for (int k = 0; k < 5; ++k) {
                const double t = N[c][k];
                N[c][k] = N[piv][k];
                N[piv][k] = t;
            }
        for (int r = c + 1; r < 3; ++r) {
            const double f = N[r][c] / N[c][c];
            for (int k = c; k < 5; ++k) N[r][k] -= f * N[c][k];
        }
    }
    double x[2][3];
    for (int j = 0; j < 2; ++j)
        for (int r = 2; r >= 0; --r) {
            double acc = N[r][3 + j];
            for (int k = r + 1; k < 3; ++k) acc -= N[r][k] * x[j][k];
            x[j][r] = acc / N[r][r];
        }
    for (int k = 0; k < 3; ++k) {
        A[k] = x[0][k];
        A[3 + k] = x[1][k];
    }
}

// Pass `pass` (0 .. kGmPasses - 1) sums its slice under the weights of the model of pass - 1 (pass
// 0: weight 1 on every sample); pass kGmPasses only finishes the last model.
__global__ __launch_bounds__(kThreads) void k_gm_pass(GmFit g, int pass)
{
    __shared__ double red[kThreads / 64][kGmSums];
    __shared__ double sA[6];
    const int pair = blockIdx.y;
    const int t = threadIdx.x;
    int64_t p0 = 0, p1 = g.n;
    int W = g.W, H = g.H;
    if (g.pt_off) {
        p0 = g.pt_off[pair];
        p1 = g.pt_off[pair + 1];
        W = g.blv[(size_t)pair * g.L].W;
        H = g.blv[(size_t)pair * g.L].H;
    }
    const int nb = gm_blocks(p1 - p0); // this pair's workgroups (the grid covers the largest pair)
    if ((int)blockIdx.x >= nb) return;
    if (pass > 0) {
        // the model of pass - 1 from its partial sums (kept from pass - 2 where it cannot be solved)
        const double *part = g.part + ((size_t)((pass - 1) & 1) * g.npairs + pair) * g.nblk * kGmSums;
        double v[kGmSums];
#pragma unroll
        for (int k = 0; k < kGmSums; ++k) v[k] = 0.0;
        for (int b = t; b < nb; b += kThreads)
#pragma unroll
            for (int k = 0; k < kGmSums; ++k) v[k] += part[(size_t)b * kGmSums + k];
        block_sum(v, red);
        if (t == 0) {
            double A[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            if (pass >= 2) {
                const double *prev = g.models + ((size_t)((pass - 2) & 1) * g.npairs + pair) * 6;
                for (int k = 0; k < 6; ++k) A[k] = prev[k];
            }
            gm_solve(red[0], A);
            for (int k = 0; k < 6; ++k) sA[k] = A[k];
            if (blockIdx.x == 0) {
                double *out = g.models + ((size_t)((pass - 1) & 1) * g.npairs + pair) * 6;
                for (int k = 0; k < 6; ++k) out[k] = A[k];
            }
        }
        __syncthreads();
    }
    if (pass >= kGmPasses) return;

    const double cx = 0.5 * (W - 1), cy = 0.5 * (H - 1);
    const double c2 = g.c * g.c;
    double A[6];
    for (int k = 0; k < 6; ++k) A[k] = pass > 0 ? sA[k] : 0.0;
    const int64_t chunk = (p1 - p0 + nb - 1) / nb;
    const int64_t b0 = p0 + chunk * blockIdx.x;
    const int64_t b1 = b0 + chunk < p1 ? b0 + chunk : p1;
    double v[kGmSums];
#pragma unroll
    for (int k = 0; k < kGmSums; ++k) v[k] = 0.0;
    for (int64_t i = b0 + t; i < b1; i += kThreads) {
        const float2 m = g.flow[i];
        if (g.status[i] != DGF_ST_CONVERGED || !isfinite(m.x) || !isfinite(m.y)) continue;
        const float2 p = g.pts[i];
        const double x = (double)p.x - cx, y = (double)p.y - cy, mu = m.x, mv = m.y;
        double w = 1.0;
        if (pass > 0) {
            const double ex = mu - (A[0] * x + A[1] * y + A[2]);
            const double ey = mv - (A[3] * x + A[4] * y + A[5]);
            const double e2 = ex * ex + ey * ey;
            const double q = 1.0 - e2 / c2;
            w = e2 < c2 ? q * q : 0.0;
        }
        if (!(w > 0.0)) continue;
        const double wx = w * x, wy = w * y;
        v[kS] += w;
        v[kSx] += wx;
        v[kSy] += wy;
        v[kSxx] += wx * x;
        v[kSxy] += wx * y;
        v[kSyy] += wy * y;
        v[kSu] += w * mu;
        v[kSxu] += wx * mu;
        v[kSyu] += wy * mu;
        v[kSv] += w * mv;
        v[kSxv] += wx * mv;
        v[kSyv] += wy * mv;
        v[kNz] += 1.0;
    }
    block_sum(v, red);
    if (t < kGmSums)
        g.part[(((size_t)(pass & 1) * g.npairs + pair) * g.nblk + blockIdx.x) * kGmSums + t] = red[0][t];
}

} // namespace

size_t gm_models_bytes(int npairs) { return (size_t)(2 * npairs * 6 * sizeof(double) + 255) / 256 * 256; }

size_t gm_state_bytes(int npairs, int nblk)
{
    return gm_models_bytes(npairs) + (size_t)2 * npairs * nblk * kGmSums * sizeof(double);
}

hipError_t launch_gm_fit(const GmFit &g, hipStream_t st)
{
    for (int pass = 0; pass <= kGmPasses; ++pass) {
        const dim3 grid(pass < kGmPasses ? g.nblk : 1, g.npairs);
        hipLaunchKernelGGL(k_gm_pass, grid, dim3(kThreads), 0, st, g, pass);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

} // namespace dgf

extern "C" {

size_t dgf_gm_workspace_bytes(void) { return dgf::gm_state_bytes(1, dgf::kGmMaxBlocks); }

int dgf_gm_fit(const float *points, const float *flow, const uint8_t *status, int64_t n, int32_t width, int32_t height,
               double scale, void *workspace, size_t ws_bytes, double *model, void *stream)
{
    using namespace dgf;
    if (n < 0 || width < 1 || height < 1 || !model || !(scale > 0.0) || !std::isfinite(scale)) return DGF_ERR_INVALID_ARG;
    if (n > 0 && (!points || !flow || !status)) return DGF_ERR_INVALID_ARG;
    if (!workspace || ws_bytes < dgf_gm_workspace_bytes()) return DGF_ERR_WORKSPACE;
    GmFit g{};
    g.pts = reinterpret_cast<const float2 *>(points);
    g.flow = reinterpret_cast<const float2 *>(flow);
    g.status = status;
    g.n = n;
    g.W = width;
    g.H = height;
    g.L = 1;
    g.npairs = 1;
    g.nblk = gm_blocks(n);
    g.c = kTukeyC * scale;
    g.models = reinterpret_cast<double *>(workspace);
    g.part = reinterpret_cast<double *>((uint8_t *)workspace + gm_models_bytes(1));
    hipStream_t st = (hipStream_t)stream;
    if (launch_gm_fit(g, st) != hipSuccess) return DGF_ERR_HIP;
    return hipMemcpyAsync(model, g.models, 6 * sizeof(double), hipMemcpyDeviceToDevice, st) == hipSuccess ? DGF_OK
                                                                                                       : DGF_ERR_HIP;
}

} // extern "C"
