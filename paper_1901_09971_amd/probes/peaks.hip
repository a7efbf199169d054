// peaks.hip -- achievable-peak probes for the roofline fractions the benchmark reports: HBM
// stream copy and stream read, LDS read bandwidth, FP32 FMA and reciprocal issue rates.  Built
// into its own library (libdgf_peaks.so), used only by the benchmark; not part of the tracking
// library's interface.  Every kernel is a plain loop with its trip count fixed on the host.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

// one float4 in, one float4 out per element, grid-stride
__global__ __launch_bounds__(256) void k_copy(const float4 *__restrict__ src, float4 *__restrict__ dst, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// read-only: every float4 is summed; one partial sum per thread is written (so nothing is dead)
__global__ __launch_bounds__(256) void k_read(const float4 *__restrict__ src, int64_t n, float *__restrict__ out)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float a = 0.f, b = 0.f, c = 0.f, d = 0.f;
    for (int64_t i = t; i < n; i += stride) {
        const float4 v = src[i];
        a += v.x;
        b += v.y;
        c += v.z;
        d += v.w;
    }
    out[t] = (a + b) + (c + d);
}

// LDS reads: each lane reads 16 consecutive bytes per step (a wavefront covers 1 KiB without bank
// conflicts), `iters` passes over a 32 KiB buffer; four accumulators keep the reads live
__global__ __launch_bounds__(256) void k_lds(int iters, float *__restrict__ out)
{
    __shared__ float4 buf[2048];
    for (int i = threadIdx.x; i < 2048; i += blockDim.x) buf[i] = make_float4((float)i, 1.f, 2.f, 3.f);
    __syncthreads();
    float a = 0.f, b = 0.f, c = 0.f, d = 0.f;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const float4 v = buf[((wave * 8 + k + it) & 31) * 64 + lane];
            a += v.x;
            b += v.y;
            c += v.z;
            d += v.w;
        }
    }
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = (a + b) + (c + d);
}

// FP32 FMA issue rate: eight independent chains per lane, 64 FMAs per trip
__global__ __launch_bounds__(256) void k_fma(int iters, float x, float y, float *__restrict__ out)
{
    float v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = (float)(threadIdx.x + k);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int r = 0; r < 8; ++r)
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = fmaf(v[k], x, y);
    }
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += v[k];
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// FP32 reciprocal issue rate: eight independent chains per lane, 64 reciprocals per trip
__global__ __launch_bounds__(256) void k_rcp(int iters, float *__restrict__ out)
{
    float v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = 1.5f + (float)(threadIdx.x + k);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int r = 0; r < 8; ++r)
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = __builtin_amdgcn_rcpf(v[k]);
    }
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += v[k];
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

} // namespace

extern "C" {

// n float4 elements; blocks x 256 threads
int pk_copy(const void *src, void *dst, int64_t n, int blocks, void *stream)
{
    hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, (hipStream_t)stream, (const float4 *)src, (float4 *)dst, n);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// out: float[blocks * 256]
int pk_read(const void *src, int64_t n, float *out, int blocks, void *stream)
{
    hipLaunchKernelGGL(k_read, dim3(blocks), dim3(256), 0, (hipStream_t)stream, (const float4 *)src, n, out);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// bytes read from LDS = blocks * 256 * iters * 8 * 16
int pk_lds(int iters, float *out, int blocks, void *stream)
{
    hipLaunchKernelGGL(k_lds, dim3(blocks), dim3(256), 0, (hipStream_t)stream, iters, out);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// FMAs = blocks * 256 * iters * 64
int pk_fma(int iters, float *out, int blocks, void *stream)
{
    hipLaunchKernelGGL(k_fma, dim3(blocks), dim3(256), 0, (hipStream_t)stream, iters, 0.999f, 0.5f, out);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// reciprocals = blocks * 256 * iters * 64
int pk_rcp(int iters, float *out, int blocks, void *stream)
{
    hipLaunchKernelGGL(k_rcp, dim3(blocks), dim3(256), 0, (hipStream_t)stream, iters, out);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

} // extern "C"
