// sfoc_describe_noalloc: sfoc_describe with integral images for callers
// that cannot allocate device memory (code under stream capture, serving
// loops, harnesses that forbid it).  The per-tile aggregates that the
// integral images are assembled from live in a file-scope device array of
// fixed size instead of a caller workspace; the kernels are sfoc_describe's.
#include <hip/hip_runtime.h>

#include <mutex>

#include "sfoc_launch.h"

namespace sfoc {

// The aggregates' home: one copy per device, kept for the process lifetime.
// Host code never uses this symbol as an address (on the host it is only a
// stand-in); it uses the device address hipGetSymbolAddress returns for the
// current device.
static __device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and remembered.
hipError_t scratch_ptr(double** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ptr[dev] = p;
    }
    *out = (double*)g_ptr[dev];
    return hipSuccess;
}

}  // namespace
}  // namespace sfoc

using namespace sfoc;

extern "C" int sfoc_describe_noalloc(const float* img, int64_t H, int64_t W, int64_t ld, const sfoc_params* p,
                                     void* desc, double* integ1, double* integ2, void* stream) {
    int rc = check_image(img, H, W, ld);
    if (rc) return rc;
    if (!desc || !integ1 || !integ2) return SFOC_E_INVALID_ARG;
    rc = check_params(p, nullptr);
    if (rc) return rc;
    if (describe_ws_bytes(H, W) > kNoAllocScratchBytes) return SFOC_E_UNSUPPORTED;
    double* agg = nullptr;
    hipError_t e = scratch_ptr(&agg);
    if (e != hipSuccess) return hip_status(e);
    DescribeConsts c;
    build_describe_consts(p, &c);
    hipStream_t st = (hipStream_t)stream;
    // every aggregate the integral kernels read is written by this call's
    // describe launch first: nothing needs clearing
    e = launch_describe(img, (int)H, (int)W, ld, desc, integ1, integ2, agg, c, st);
    if (e == hipSuccess) e = launch_integral(integ1, integ2, (int)H, (int)W, agg, st);
    return hip_status(e);
}
