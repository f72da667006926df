// Rectification (Section 3.2.3): the sensed image resampled into the
// reference grid by bilinear interpolation, through the inverse of the
// sensed -> reference model that outlier rejection returns.
//
// HBM-bound gather: each wave covers 64 * kRun consecutive pixels of one
// output row, lane l taking pixels l, l + 64, ... so that every load and
// store instruction of the wave touches consecutive addresses.  A thread
// first computes the source positions and weights of all its pixels, then
// issues all their loads (addresses clamped into the image, so no load
// depends on a branch), then blends.  Output rows r and r + 1 read largely
// the same sensed rows,
// so the workgroups of consecutive rows should share an L2: the hardware
// deals workgroups to the eight XCDs round-robin, and the kernel renumbers
// them so that each XCD gets one contiguous band of rows.
#include <hip/hip_runtime.h>
#include <math.h>

#include "sfoc_dev.h"
#include "sfoc_launch.h"
#include "sfoc_trace.h"

namespace sfoc {
namespace rect {

constexpr int kNT = 256, kRun = 8, kXcd = 8;
constexpr int kCols = kNT * kRun;   // output columns per workgroup

__global__ __launch_bounds__(kNT) void rectify_kernel(const float* __restrict__ sen, int Hs, int Ws, int64_t lds,
                                                      const double* __restrict__ model, float* __restrict__ out,
                                                      int Ho, int Wo, int64_t ldo, float fill, int bpr) {
    // workgroup x of n runs on XCD x % 8; XCD j takes the j-th contiguous
    // share of the logical numbering (row-major over (row, column block))
    const int nb = gridDim.x, x = blockIdx.x;
    const int per = nb / kXcd, rem = nb % kXcd, xcd = x % kXcd;
    const int L = (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + x / kXcd;
    const int r = L / bpr;
    const int c0 = (L - r * bpr) * kCols + (threadIdx.x >> 6) * (64 * kRun) + (threadIdx.x & 63);
    if (r >= Ho || c0 >= Wo) return;
    // inverse model: adjugate / determinant (float64)
    double M[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) M[q] = model[q];
    double A[9];
    A[0] = M[4] * M[8] - M[5] * M[7];
    A[1] = M[2] * M[7] - M[1] * M[8];
    A[2] = M[1] * M[5] - M[2] * M[4];
    A[3] = M[5] * M[6] - M[3] * M[8];
    A[4] = M[0] * M[8] - M[2] * M[6];
    A[5] = M[2] * M[3] - M[0] * M[5];
    A[6] = M[3] * M[7] - M[4] * M[6];
    A[7] = M[1] * M[6] - M[0] * M[7];
    A[8] = M[0] * M[4] - M[1] * M[3];
    const double idet = 1.0 / (M[0] * A[0] + M[1] * A[3] + M[2] * A[6]);
    const double rr = (double)r;
    const double by = fma(A[0], rr, A[2]) * idet, bx = fma(A[3], rr, A[5]) * idet, bw = fma(A[6], rr, A[8]) * idet;
    const double ay = A[1] * idet, ax = A[4] * idet, aw = A[7] * idet;
    const double ymax = (double)(Hs - 1), xmax = (double)(Ws - 1);
    bool in[kRun];
    int o00[kRun], o01[kRun], o10[kRun], o11[kRun];
    float fy[kRun], fx[kRun];
#pragma unroll
    for (int j = 0; j < kRun; ++j) {
        const double c = (double)(c0 + 64 * j);
        const double w = fma(aw, c, bw);
        // 1 / w: hardware reciprocal refined by one Newton step (relative
        // error about the square of the estimate's)
        double iw = __builtin_amdgcn_rcp(w);
        iw = iw * fma(-w, iw, 2.0);
        const double py = fma(ay, c, by) * iw, px = fma(ax, c, bx) * iw;
        in[j] = w > 0.0 && py >= 0.0 && py <= ymax && px >= 0.0 && px <= xmax;
        const int y0 = in[j] ? min((int)py, Hs - 1) : 0, x0 = in[j] ? min((int)px, Ws - 1) : 0;
        const int y1 = min(y0 + 1, Hs - 1), x1 = min(x0 + 1, Ws - 1);
        fy[j] = in[j] ? (float)(py - (double)y0) : 0.f;
        fx[j] = in[j] ? (float)(px - (double)x0) : 0.f;
        o00[j] = y0 * (int)lds + x0;   // sides <= 2^20 and the image < 2^31 elements
        o01[j] = y0 * (int)lds + x1;
        o10[j] = y1 * (int)lds + x0;
        o11[j] = y1 * (int)lds + x1;
    }
    float v00[kRun], v01[kRun], v10[kRun], v11[kRun];
#pragma unroll
    for (int j = 0; j < kRun; ++j) {
        v00[j] = sen[o00[j]];
        v01[j] = sen[o01[j]];
        v10[j] = sen[o10[j]];
        v11[j] = sen[o11[j]];
    }
    float* o = out + (int64_t)r * ldo;
#pragma unroll
    for (int j = 0; j < kRun; ++j) {
        const float top = fmaf(fx[j], v01[j] - v00[j], v00[j]);
        const float bot = fmaf(fx[j], v11[j] - v10[j], v10[j]);
        const int c = c0 + 64 * j;
        if (c < Wo) o[c] = in[j] ? fmaf(fy[j], bot - top, top) : fill;
    }
}

}  // namespace rect
}  // namespace sfoc

using namespace sfoc;

extern "C" int sfoc_rectify(const float* sen, int64_t Hs, int64_t Ws, int64_t lds, const double* model, float* out,
                            int64_t Ho, int64_t Wo, int64_t ldo, float fill, void* stream) {
    using namespace rect;
    if (!sen || !model || !out || Hs < 1 || Ws < 1 || lds < Ws || Ho < 1 || Wo < 1 || ldo < Wo)
        return SFOC_E_INVALID_ARG;
    if (Hs > (1 << 20) || Ws > (1 << 20) || Ho > (1 << 20) || Wo > (1 << 20)) return SFOC_E_UNSUPPORTED;
    if (Hs * lds >= ((int64_t)1 << 31)) return SFOC_E_UNSUPPORTED;   // 32-bit sensed offsets
    const int64_t bpr = (Wo + kCols - 1) / kCols;
    const int64_t nb = Ho * bpr;
    if (nb > 0x7fffffff) return SFOC_E_UNSUPPORTED;
    hipStream_t st = (hipStream_t)stream;
    trace_begin(st, SFOC_K_RECTIFY);
    hipLaunchKernelGGL(rectify_kernel, dim3((unsigned)nb), dim3(kNT), 0, st, sen, (int)Hs, (int)Ws, lds, model, out,
                       (int)Ho, (int)Wo, ldo, fill, (int)bpr);
    trace_end(st, SFOC_K_RECTIFY);
    return hip_status(hipGetLastError());
}
