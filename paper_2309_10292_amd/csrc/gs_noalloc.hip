// gs_sqdiff_noalloc (include/gs.h): gs_sqdiff for callers that cannot
// allocate device memory. The per-workgroup partial sums live in a
// file-scope device array instead of a caller workspace.
#include "../../include/gs.h"
#include "gs_internal.hpp"
#include "gs_launch.hpp"

#include <hip/hip_runtime.h>

#include <mutex>

using namespace gsapi;

namespace {

constexpr int k_scratch_parts = 512;         // partial sums the array holds (4 KiB)
constexpr int k_max_devices = 64;
constexpr size_t k_max_n = (size_t)1 << 40;  // elements per call

// One copy per GPU, held until the process ends. In host code the name is
// not a device address: the kernels get the address resolved below.
static __device__ __align__(256) double scratch[k_scratch_parts];

std::mutex g_scratch_mu;
double *g_scratch[k_max_devices];

// The current device's address of `scratch`, resolved once per device.
hipError_t scratch_on_current_device(double **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= k_max_devices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[dev] = static_cast<double *>(p);
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

} // namespace

extern "C" gs_status gs_sqdiff_noalloc(const void *a, const void *b, size_t n, int32_t storage, void *hip_stream,
                                       double *out)
{
    if (!a || !b || !out) return fail(GS_ERR_INVALID_ARG, "NULL pointer");
    if (storage_bytes(storage) == 0) return fail(GS_ERR_INVALID_ARG, "unknown storage type %d", storage);
    if (n > k_max_n) return fail(GS_ERR_UNSUPPORTED, "n = %zu exceeds the maximum of 2^40 elements", n);
    if (gs::sqdiff_blocks() > k_scratch_parts)
        return fail(GS_ERR_UNSUPPORTED, "the reduction needs %d partial sums, the static scratch holds %d",
                    gs::sqdiff_blocks(), k_scratch_parts);
    double *part = nullptr;
    hipError_t e = scratch_on_current_device(&part);
    if (e != hipSuccess) return hip_fail(e, "gs_sqdiff_noalloc scratch address");
    hipStream_t st = (hipStream_t)hip_stream;
    // Every workgroup writes its own partial, so nothing needs clearing; the
    // partials are folded on the host in the order gs_sqdiff uses.
    double host[k_scratch_parts];
    const int parts = gs::sqdiff_blocks();
    e = gs::launch_sqdiff(storage, a, b, n, part, st);
    if (e == hipSuccess) e = hipMemcpyAsync(host, part, (size_t)parts * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "gs_sqdiff_noalloc");
    double sum = 0.0;
    for (int i = 0; i < parts; ++i) sum += host[i];
    *out = sum;
    return GS_OK;
}
