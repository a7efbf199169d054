// pyramid.hip -- one pyramid reduction step on gfx950.
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
// both frames of a pair, or a whole batch, go in one launch.
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

// Batched form: blockIdx.z selects the job in a device table; tiles beyond a job's output exit
// before staging.
template <typename T>
__global__ __launch_bounds__(256) void k_pyr_down_batched(const PyrJob *__restrict__ jobs)
{
    const PyrJob J = jobs[blockIdx.z];
    if ((int)blockIdx.x * PYR_TX >= ((J.W + 1) >> 1) || (int)blockIdx.y * PYR_TY >= ((J.H + 1) >> 1)) return;
    pyr_tile<T>(J, blockIdx.x, blockIdx.y);
}

hipError_t launch_pyr_level_batched(const PyrJob *jobs_dev, int njobs, int max_w2, int max_h2, int dtype, hipStream_t st)
{
    dim3 grid((max_w2 + PYR_TX - 1) / PYR_TX, (max_h2 + PYR_TY - 1) / PYR_TY, njobs);
    if (dtype == DGF_U8)
        hipLaunchKernelGGL(k_pyr_down_batched<uint8_t>, grid, dim3(256), 0, st, jobs_dev);
    else
        hipLaunchKernelGGL(k_pyr_down_batched<float>, grid, dim3(256), 0, st, jobs_dev);
    return hipGetLastError();
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

} // namespace dgf
