// track_static.hip -- dgf_track_static: robust pyramidal tracking whose pyramids live in a
// file-scope device array instead of a caller workspace, for callers that cannot allocate device
// memory (code under graph capture, allocation-free serving loops).
//
// The array is one per GPU (each device that loads this library holds its own copy until the
// process ends).  Host code never passes the array's name to a kernel: in host code that name is
// a host-side stand-in, not a device address.  The device address is looked up once per device
// with hipGetSymbolAddress, with that device current, and kept in a per-device table; every
// kernel argument derived from the array comes from that address.
#include <mutex>

#include "dgf_internal.hpp"
#include "dgf_tuning.hpp"

namespace {

constexpr size_t kScratchBytes = (size_t)DGF_TRACK_STATIC_MAX_BYTES;
static_assert(kScratchBytes % 256 == 0, "scratch size must keep 256-byte alignment");

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
void *g_scratch_dev[kMaxDevices];
std::mutex g_scratch_mu;

// Device address of this device's scratch array (looked up on the first call per device).
int scratch_address(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return DGF_ERR_HIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return DGF_ERR_HIP;
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return DGF_OK;
}

} // namespace

using namespace dgf;

extern "C" {

int dgf_track_static(const dgf_image *I0, const dgf_image *I1, const float *points, int64_t n, int32_t levels,
                     int32_t support, int32_t iters, const dgf_track_opts *opts, float *flow, uint8_t *status,
                     int32_t *iters_out, float *illum_out, void *stream)
{
    // every argument check comes before the first HIP call
    dgf_track_opts o;
    const int rc = validate_track_args(I0, I1, points, n, levels, support, iters, opts, flow, status, &o);
    if (rc != DGF_OK) return rc;
    if (illum_out && !(o.flags & DGF_TRACK_ILLUM)) return DGF_ERR_INVALID_ARG;
    if (dgf_track_workspace_bytes(I0->width, I0->height, levels, I0->dtype) > kScratchBytes) return DGF_ERR_SCRATCH;
    if (n == 0) return DGF_OK;
    void *ws = nullptr;
    const int rs = scratch_address(&ws);
    if (rs != DGF_OK) return rs;
    return dgf_track(I0, I1, points, n, levels, support, iters, opts, ws, kScratchBytes, flow, status, iters_out,
                     illum_out, stream);
}

} // extern "C"
