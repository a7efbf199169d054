// pyramid.hip -- pyramid reduction steps on gfx950 (one level per launch, or up to four uint8
// levels per launch).
//
// Level l+1 = binomial [1 4 6 4 1] smoothing of level l along both axes with replicated borders,
// sampled at even pixels (size ceil(W/2) x ceil(H/2)).  uint8 levels keep the exact integer sum
// and round half up, (sum + 128) >> 8; float levels are scaled by 1/256.
//
// Each workgroup produces a 64 x 16 output tile.  It stages the (2*64+3) x (2*16+3) input
// rectangle into LDS with coalesced row loads (border rows/columns replicated by index clamping),
// runs the horizontal 5-tap pass into a second LDS buffer at the decimated column rate, then the
// vertical pass at the decimated row rate.  Every input byte is read from HBM once per tile
// (plus a 3-pixel halo), every output byte written once.  blockIdx.z selects the job (image), so
// both frames of a pair go in one launch.  (Batch plans use front_batch.hip.)
#include "dgf_internal.hpp"

namespace dgf {

constexpr int PYR_TX = 64, PYR_TY = 16;
constexpr int PYR_IW = 2 * PYR_TX + 3, PYR_IH = 2 * PYR_TY + 3;

template <typename T> struct PyrAcc;
template <> struct PyrAcc<uint8_t> { using type = int; };
template <> struct PyrAcc<float> { using type = float; };

template <typename T>
__device__ __forceinline__ void pyr_tile(const PyrJob &J, int tile_x, int tile_y)
{
    using A = typename PyrAcc<T>::type;
    __shared__ A in[PYR_IH][PYR_IW + 1];
    __shared__ A hs[PYR_IH][PYR_TX + 1];
    const int W2 = (J.W + 1) >> 1, H2 = (J.H + 1) >> 1;
    const int ox = tile_x * PYR_TX, oy = tile_y * PYR_TY; // output origin
    const int ix = 2 * ox - 2, iy = 2 * oy - 2;            // input origin of the staged rectangle
    const int tid = threadIdx.x;
    for (int i = tid; i < PYR_IW * PYR_IH; i += blockDim.x) {
        const int y = i / PYR_IW, x = i - y * PYR_IW;
        const int sx = clampi(ix + x, 0, J.W - 1), sy = clampi(iy + y, 0, J.H - 1);
        in[y][x] = (A)reinterpret_cast<const T *>(J.src + (int64_t)sy * J.src_pitch)[sx];
    }
    __syncthreads();
    for (int i = tid; i < PYR_IH * PYR_TX; i += blockDim.x) {
        const int y = i / PYR_TX, x = i - y * PYR_TX;
        const A *r = &in[y][2 * x];
        hs[y][x] = r[0] + r[4] + (A)4 * (r[1] + r[3]) + (A)6 * r[2];
    }
    __syncthreads();
    for (int i = tid; i < PYR_TY * PYR_TX; i += blockDim.x) {
        const int y = i / PYR_TX, x = i - y * PYR_TX;
        const int gx = ox + x, gy = oy + y;
        if (gx >= W2 || gy >= H2) continue;
        const A v = hs[2 * y][x] + hs[2 * y + 4][x] + (A)4 * (hs[2 * y + 1][x] + hs[2 * y + 3][x]) + (A)6 * hs[2 * y + 2][x];
        T *row = reinterpret_cast<T *>(J.dst + (int64_t)gy * J.dst_pitch);
        if constexpr (sizeof(T) == 1) {
            row[gx] = (T)((v + 128) >> 8);
        } else {
            row[gx] = v * (1.0f / 256.0f);
        }
    }
}

struct PyrJobs2 {
    PyrJob j[2];
};

template <typename T>
__global__ __launch_bounds__(256) void k_pyr_down(PyrJobs2 jobs)
{
    pyr_tile<T>(jobs.j[blockIdx.z], blockIdx.x, blockIdx.y);
}

hipError_t launch_pyr_level(const PyrJob *jobs, int njobs, int dtype, hipStream_t st)
{
    if (njobs < 1 || njobs > 2) return hipErrorInvalidValue;
    PyrJobs2 J{};
    int W2max = 0, H2max = 0;
    for (int i = 0; i < njobs; ++i) {
        J.j[i] = jobs[i];
        W2max = max(W2max, (jobs[i].W + 1) / 2);
        H2max = max(H2max, (jobs[i].H + 1) / 2);
    }
    dim3 grid((W2max + PYR_TX - 1) / PYR_TX, (H2max + PYR_TY - 1) / PYR_TY, njobs);
    if (dtype == DGF_U8)
        hipLaunchKernelGGL(k_pyr_down<uint8_t>, grid, dim3(256), 0, st, J);
    else
        hipLaunchKernelGGL(k_pyr_down<float>, grid, dim3(256), 0, st, J);
    return hipGetLastError();
}

// ---- several uint8 levels in one launch -----------------------------------------------------
//
// Levels s+1 .. s+m (m <= 4) of one or two uint8 images from level s.  A block owns a
// PC_T x PC_T tile of the coarsest level s+m and the 2^(m-k) times larger tile of every finer
// level s+k, which tile each level exactly; it computes each level over its owned tile plus the
// halo the next coarser level's taps need (the needed range [lo, hi] at level k+1 needs
// [2 lo - 2, 2 hi + 2] at level k, clamped into the level), starting from a staged rectangle of
// level s, and writes the owned pixels.  Integer sums and the (sum + 128) >> 8 rounding at every
// level, with the replicated border of every level, as in k_pyr_down, so the levels are
// identical to one launch per level.
constexpr int PC_T = 4, PC_MAXM = 4;
// Lanes per chain block: a block walks its levels one after another, each a few LDS passes with
// barriers between, and with one or two blocks per CU only its own waves hide the LDS latency;
// eight waves measured 15 % faster than four on the 1242x375 pair (sixteen: 11 %).
constexpr int kChainThreads = 512;
constexpr int pc_width(int m) { return m == 0 ? PC_T : 2 * pc_width(m - 1) + 3; } // region width m levels finer
constexpr int PC_N0 = pc_width(PC_MAXM);     // 109: staged source rectangle side
constexpr int PC_N1 = pc_width(PC_MAXM - 1); // 53: first produced level
constexpr int PC_N0P = (PC_N0 + 3) & ~3;     // 112: row pitch of the staged source rectangle

// One block of a chain launch: tile (bx, by) of the coarsest level of image f, with the LDS
// buffers the kernel provides.
__device__ __forceinline__ void pyr_chain_block(const PyrChain &A, int bx, int by, int f,
                                                uint8_t (*lvl)[PC_N0P * PC_N0], uint16_t *hs)
{
    const int m = A.m, tid = threadIdx.x;
    // needed (lo, hi) at every level, coarsest first, then clamped into the level
    int x0[PC_MAXM + 1], x1[PC_MAXM + 1], y0[PC_MAXM + 1], y1[PC_MAXM + 1];
    int lx = bx * PC_T, hx = lx + PC_T - 1, ly = by * PC_T, hy = ly + PC_T - 1;
#pragma unroll
    for (int k = PC_MAXM; k >= 0; --k) {
        if (k <= m) {
            if (k < m) {
                lx = 2 * lx - 2;
                hx = 2 * hx + 2;
                ly = 2 * ly - 2;
                hy = 2 * hy + 2;
            }
            x0[k] = lx > 0 ? lx : 0;
            x1[k] = hx < A.W[k] - 1 ? hx : A.W[k] - 1;
            y0[k] = ly > 0 ? ly : 0;
            y1[k] = hy < A.H[k] - 1 ? hy : A.H[k] - 1;
        }
    }
    // stage level s (row pitch 4 ceil(w / 4); the produced levels use their own width)
    const int w0 = x1[0] - x0[0] + 1, p0 = (w0 + 3) & ~3;
    stage_u8_block<4>(lvl[0], p0, A.src[f], A.src_pitch[f], A.W[0], x0[0], y0[0], w0, y1[0] - y0[0] + 1);
    __syncthreads();
    for (int k = 0; k < m; ++k) {
        const uint8_t *in = lvl[k & 1];
        uint8_t *out = lvl[(k + 1) & 1];
        const int wi = x1[k] - x0[k] + 1, hi = y1[k] - y0[k] + 1, pin = k == 0 ? p0 : wi;
        const int wo = x1[k + 1] - x0[k + 1] + 1, ho = y1[k + 1] - y0[k + 1] + 1;
        const float inv_wo = 1.0f / (float)wo;
        const int Wk = A.W[k], Hk = A.H[k];
        // horizontal pass: every staged row, at the output column rate
        for (int i = tid; i < hi * wo; i += kChainThreads) {
            const int r = div_small(i, inv_wo), xo = i - r * wo;
            const int c = 2 * (x0[k + 1] + xo);
            const uint8_t *row = in + r * pin;
            auto at = [&](int cc) { return (int)row[(cc < 0 ? 0 : (cc > Wk - 1 ? Wk - 1 : cc)) - x0[k]]; };
            hs[i] = (uint16_t)(at(c - 2) + at(c + 2) + 4 * (at(c - 1) + at(c + 1)) + 6 * at(c));
        }
        __syncthreads();
        // vertical pass, rounding, and the owned pixels to memory
        const int sh = m - (k + 1);
        const int ox0 = (bx * PC_T) << sh, oy0 = (by * PC_T) << sh;
        const int own = PC_T << sh;
        uint8_t *dst = A.dst[k][f];
        const int64_t dp = A.dst_pitch[k];
        for (int i = tid; i < ho * wo; i += kChainThreads) {
            const int yo = div_small(i, inv_wo), xo = i - yo * wo;
            const int gy = y0[k + 1] + yo, gx = x0[k + 1] + xo;
            const int rr = 2 * gy;
            auto at = [&](int r) { return (int)hs[((r < 0 ? 0 : (r > Hk - 1 ? Hk - 1 : r)) - y0[k]) * wo + xo]; };
            const int v = at(rr - 2) + at(rr + 2) + 4 * (at(rr - 1) + at(rr + 1)) + 6 * at(rr);
            const uint8_t q = (uint8_t)((v + 128) >> 8);
            out[i] = q;
            if (gx >= ox0 && gx < ox0 + own && gy >= oy0 && gy < oy0 + own) dst[(int64_t)gy * dp + gx] = q;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kChainThreads) void k_pyr_chain_u8(PyrChain A)
{
    __shared__ __align__(16) uint8_t lvl[2][PC_N0P * PC_N0];
    __shared__ uint16_t hs[PC_N0 * PC_N1];
    pyr_chain_block(A, (int)blockIdx.x, (int)blockIdx.y, (int)blockIdx.z, lvl, hs);
}

// The chain launch with the detection tiles of one uint8 frame beside it: blocks 0 .. nchain - 1
// build pyramid tiles (x fastest, then y, then image), the rest are 16 x 16-window detection
// tiles staged in the chain's level buffer (lanes beyond the 256 windows only help staging).  The two kinds of work are independent, so one
// launch runs both in about the time of the longer.
__global__ __launch_bounds__(kChainThreads) void k_front_u8(PyrChain A, FrontDetect D, int chain_x, int chain_y, int nchain)
{
    __shared__ __align__(16) uint8_t lvl[2][PC_N0P * PC_N0];
    __shared__ uint16_t hs[PC_N0 * PC_N1];
    const int b = (int)blockIdx.x;
    if (b < nchain) {
        const int per = chain_x * chain_y, f = b / per, t = b - f * per, by = t / chain_x;
        pyr_chain_block(A, t - by * chain_x, by, f, lvl, hs);
        return;
    }
    const int t = b - nchain, ty = t / D.tiles_x;
    detect_tile<16, 16>(&lvl[0][0], t - ty * D.tiles_x, ty, D.img, D.pitch, D.W, D.H, D.win, D.stride, D.nx, D.ny, 0,
                        D.o);
}

// Largest detection tile the fused launch can stage (the chain's two level buffers).
constexpr size_t kFrontDetectLds = 2 * (size_t)PC_N0P * PC_N0;

hipError_t launch_pyr_chain_u8(const PyrChain &A, int njobs, hipStream_t st, const FrontDetect *det)
{
    if (A.m < 1 || A.m > PC_MAXM || njobs < 1 || njobs > 2) return hipErrorInvalidValue;
    dim3 grid((A.W[A.m] + PC_T - 1) / PC_T, (A.H[A.m] + PC_T - 1) / PC_T, njobs);
    if (!det) {
        hipLaunchKernelGGL(k_pyr_chain_u8, grid, dim3(kChainThreads), 0, st, A);
        return hipGetLastError();
    }
    const int nchain = (int)(grid.x * grid.y * grid.z);
    const int blocks = nchain + det->tiles_x * det->tiles_y;
    hipLaunchKernelGGL(k_front_u8, dim3((unsigned)blocks), dim3(kChainThreads), 0, st, A, *det, (int)grid.x, (int)grid.y, nchain);
    return hipGetLastError();
}

bool front_detect_fits(int win, int stride) { return detect_tile_lds(win, stride) <= kFrontDetectLds; }

// Levels 1 .. levels-1 of one or two uint8 images (level 0 = srcs) as chains of up to four
// levels per launch; level l of image f goes to lvl[f][l], row pitch pitch[l].
hipError_t launch_pyr_chains(const uint8_t *const srcs[2], const int64_t src_pitch[2],
                             uint8_t *const lvl[2][DGF_MAX_LEVELS], const int64_t *pitch, int W, int H, int levels,
                             int njobs, hipStream_t st, const FrontDetect *det)
{
    int Wl[DGF_MAX_LEVELS], Hl[DGF_MAX_LEVELS];
    Wl[0] = W;
    Hl[0] = H;
    for (int l = 1; l < levels; ++l) {
        Wl[l] = (Wl[l - 1] + 1) / 2;
        Hl[l] = (Hl[l - 1] + 1) / 2;
    }
    for (int s = 0; s + 1 < levels; s += PC_MAXM) {
        PyrChain A{};
        A.m = levels - 1 - s < PC_MAXM ? levels - 1 - s : PC_MAXM;
        for (int f = 0; f < njobs; ++f) {
            A.src[f] = s == 0 ? srcs[f] : lvl[f][s];
            A.src_pitch[f] = s == 0 ? src_pitch[f] : pitch[s];
            for (int k = 1; k <= A.m; ++k) A.dst[k - 1][f] = lvl[f][s + k];
        }
        for (int k = 0; k <= A.m; ++k) {
            A.W[k] = Wl[s + k];
            A.H[k] = Hl[s + k];
            if (k > 0) A.dst_pitch[k - 1] = pitch[s + k];
        }
        const hipError_t e = launch_pyr_chain_u8(A, njobs, st, s == 0 ? det : nullptr);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

} // namespace dgf
