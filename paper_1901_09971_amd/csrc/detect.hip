// detect.hip -- DeGraF key-point detection on gfx950.
//
// One key-point per window of a uniform grid (DeGraF-Flow, Section 2 "Point detection"):
// positive centroid from the intensity-weighted moments (Eq. 1), negative centroid from the
// inverted weights 1 + m - I with m the window maximum (Eq. 2), and the centroid with the larger
// weight sum is kept (strictly larger for the negative one).
//
// The image is read once from HBM: a workgroup owns a TX x TY block of windows, stages the
// pixel rectangle they cover into LDS four bytes per lane (aligned dword pairs), and each lane
// then reduces its own window from LDS.  Only the positive moments are accumulated; the negative ones follow
// exactly from sum (1 + m - I) = (1 + m) w h - sum I (and likewise for the moments).
#include "dgf_internal.hpp"

namespace dgf {

// LDS of one 16 x 16-window tile: rows of (15 stride + win) bytes at a pitch rounded up to 4
size_t detect_tile_lds(int win, int stride)
{
    return (size_t)((15 * stride + win + 3) & ~3) * (size_t)(15 * stride + win);
}

template <int TX, int TY>
__global__ __launch_bounds__(TX *TY) void k_detect_tiled(const uint8_t *__restrict__ img, int64_t pitch, int W, int H,
                                                          int win, int stride, int nx, int ny, DetectOut o)
{
    extern __shared__ __align__(16) uint8_t tile[];
    detect_tile<TX, TY>(tile, (int)blockIdx.x, (int)blockIdx.y, img, pitch, W, H, win, stride, nx, ny, 0, o);
}

// Direct form for windows too large to tile: one lane per window, reads through the cache.
__global__ __launch_bounds__(256) void k_detect_direct(const uint8_t *__restrict__ img, int64_t pitch, int win,
                                                        int stride, int nx, int64_t N, DetectOut o)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const int kx = (int)(n % nx), ky = (int)(n / nx);
    const int x0 = kx * stride, y0 = ky * stride;
    int S = 0, Mi = 0, Mj = 0, m = 0;
    for (int i = 0; i < win; ++i) {
        const uint8_t *row = img + (int64_t)(y0 + i) * pitch + x0;
        int rs = 0, rj = 0;
        for (int j = 0; j < win; ++j) {
            const int v = row[j];
            rs += v;
            rj += j * v;
            m = max(m, v);
        }
        S += rs;
        Mi += i * rs;
        Mj += rj;
    }
    finish_window(S, Mi, Mj, m, win, x0, y0, n, o);
}

hipError_t launch_detect(const uint8_t *img, int64_t pitch, int W, int H, int win, int stride, float *pts,
                         uint8_t *sel, float *resp, hipStream_t st)
{
    const int nx = (W - win) / stride + 1, ny = (H - win) / stride + 1;
    DetectOut o{pts, sel, resp};
    constexpr int TX = 16, TY = 16;
    const int64_t RW = (int64_t)(TX - 1) * stride + win, RH = (int64_t)(TY - 1) * stride + win;
    const int64_t RP = (RW + 3) & ~(int64_t)3;
    if (RP * RH <= 48 * 1024) {
        dim3 grid((nx + TX - 1) / TX, (ny + TY - 1) / TY);
        hipLaunchKernelGGL((k_detect_tiled<TX, TY>), grid, dim3(TX * TY), (size_t)(RP * RH), st, img, pitch, W, H, win,
                           stride, nx, ny, o);
    } else {
        const int64_t N = (int64_t)nx * ny;
        hipLaunchKernelGGL(k_detect_direct, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, img, pitch, win,
                           stride, nx, N, o);
    }
    return hipGetLastError();
}

} // namespace dgf
