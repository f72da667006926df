// Block-based FAST interest-point detection (Section 3.1.1: the FAST
// operator with a partitioning strategy, so that the interest points are
// spread evenly over the sensed image).  Three launches:
//
//  1. strength + suppression, one 32 x 32 tile per workgroup: the image
//     tile with a 4-pixel halo in LDS; the FAST-9 corner strength V (the
//     largest threshold at which 9 contiguous pixels of the radius-3 circle
//     are all brighter, or all darker, than the centre) for the tile and a
//     1-pixel ring; then 3 x 3 non-maximum suppression with a raster-order
//     tie rule.  Kept corners are sparse: their strengths go to a map in
//     the workspace (other entries are never written), and a bit mask, one
//     32-bit word per row of a tile (from a wave ballot: a wave covers two
//     tile rows), marks them.
//     Per pixel the 16 arc minima and maxima of the 16 circle differences
//     come from a doubling network (pairs, fours, eights, then the ninth
//     element): 64 min and 64 max instead of 128 each.  Only float32
//     subtractions and min / max are involved, so V is exact.
//  2. selection, one workgroup per block: the threads walk the block's mask
//     words, read the strengths of the set bits, and each keeps the best
//     K >= per_block corners it sees as sorted 64-bit keys (strength
//     descending, raster index within the block ascending) in registers; a
//     bitonic sort of all threads' lists in LDS gives the block's first
//     per_block.
//  3. compaction (one workgroup): block counts prefix-summed, each block's
//     interest points copied to its place in one list.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "sfoc_dev.h"
#include "sfoc_launch.h"
#include "sfoc_plan.h"
#include "sfoc_trace.h"

namespace sfoc {
namespace fast {

constexpr int kTS = 32, kHalo = 4, kIS = kTS + 2 * kHalo, kVS = kTS + 2;   // tile, image and strength sides
constexpr int kNT = 256;
constexpr int kSelNT = 256, kMaxPer = 32, kMaxBlocks = 1 << 16;
constexpr int kCompNT = 1024;

struct Region {
    int b, H, W;           // detection region rows / columns [b, size - b)
};

struct Blocks {
    int nby, nbx, per;
};

SFOC_DEV int bound(int lo, int n, int i, int nb) { return lo + (int)(((int64_t)i * n) / nb); }

// The radius-3 circle, clockwise from the top, as (dy, dx).  Compile-time
// constants: with the reads addressed from the 7 x 7 neighbourhood's
// top-left element, every circle read is one LDS instruction with a constant
// offset and no address arithmetic.
constexpr int kCy[16] = {-3, -3, -2, -1, 0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3};
constexpr int kCx[16] = {0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3, -3, -3, -2, -1};

SFOC_DEV float strength(const float* tile, int ty, int tx) {
    const float* nb = tile + (ty - 3) * kIS + (tx - 3);
    const float c = nb[3 * kIS + 3];
    float u[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) u[i] = nb[(kCy[i] + 3) * kIS + kCx[i] + 3] - c;
    // windows of 9 starting at k (cyclic): min / max of u[k .. k+8]
    float mn2[16], mx2[16], mn4[16], mx4[16], mn8[16], mx8[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        mn2[i] = fminf(u[i], u[(i + 1) & 15]);
        mx2[i] = fmaxf(u[i], u[(i + 1) & 15]);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        mn4[i] = fminf(mn2[i], mn2[(i + 2) & 15]);
        mx4[i] = fmaxf(mx2[i], mx2[(i + 2) & 15]);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        mn8[i] = fminf(mn4[i], mn4[(i + 4) & 15]);
        mx8[i] = fmaxf(mx4[i], mx4[(i + 4) & 15]);
    }
    float v = -INFINITY;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const float lo = fminf(mn8[k], u[(k + 8) & 15]);    // min over the arc of (I_x - I_p)
        const float hi = fmaxf(mx8[k], u[(k + 8) & 15]);    // so min over the arc of (I_p - I_x) = -hi
        v = fmaxf(v, fmaxf(lo, -hi));
    }
    return v;
}

__global__ __launch_bounds__(kNT) void strength_kernel(const float* __restrict__ img, int64_t ld, Region R,
                                                       float thr, float* __restrict__ S,
                                                       uint32_t* __restrict__ mask, int mask_words, int tiles_x) {
    static_assert(kTS == 32 && kNT % 64 == 0, "a wave covers two tile rows");
    __shared__ float tile[kIS * kIS];
    __shared__ float vs[kVS * kVS];
    const int t = threadIdx.x, lane = t & 63;
    const int ty0 = (blockIdx.x / tiles_x) * kTS, tx0 = (blockIdx.x % tiles_x) * kTS;
    for (int e = t; e < kIS * kIS; e += kNT) {
        const int a = e / kIS, c = e - a * kIS;
        const int y = ty0 - kHalo + a, x = tx0 - kHalo + c;
        tile[e] = (y >= 0 && y < R.H && x >= 0 && x < R.W) ? img[(int64_t)y * ld + x] : 0.f;
    }
    __syncthreads();
    // strengths of the tile and a 1-pixel ring; -inf outside the region
    for (int e = t; e < kVS * kVS; e += kNT) {
        const int a = e / kVS, c = e - a * kVS;
        const int y = ty0 - 1 + a, x = tx0 - 1 + c;
        const bool in = y >= R.b && y < R.H - R.b && x >= R.b && x < R.W - R.b;
        vs[e] = in ? strength(tile, a + kHalo - 1, c + kHalo - 1) : -INFINITY;
    }
    __syncthreads();
    // every lane runs every pass (the ballot needs the whole wave); a pass
    // of wave w covers tile rows 2w + 8 pass and the row after it
    for (int e = t; e < kTS * kTS; e += kNT) {
        const int a = e / kTS, c = e - a * kTS;
        const int y = ty0 + a, x = tx0 + c;
        bool keep = false;
        float v = 0.f;
        if (y >= R.b && y < R.H - R.b && x >= R.b && x < R.W - R.b) {
            const float* q = vs + (a + 1) * kVS + (c + 1);
            v = q[0];
            keep = v > thr;
            // neighbours before in raster order: strictly smaller; after: not larger
            keep = keep && v > q[-kVS - 1] && v > q[-kVS] && v > q[-kVS + 1] && v > q[-1];
            keep = keep && v >= q[1] && v >= q[kVS - 1] && v >= q[kVS] && v >= q[kVS + 1];
        }
        if (keep) S[(int64_t)y * R.W + x] = v;
        const uint64_t bal = __ballot(keep);
        if ((lane & 31) == 0 && y < R.H) mask[(int64_t)y * mask_words + tx0 / kTS] = (uint32_t)(bal >> (lane & 32));
    }
}

// Keys: strength (>= 0 for kept corners) descending, then the raster index
// within the block ascending; empty = all ones.
SFOC_DEV uint64_t make_key(float v, uint32_t e) {
    const uint32_t ord = __float_as_uint(v) | 0x80000000u;   // order-preserving for v >= 0
    return ((uint64_t)(~ord) << 32) | e;
}

template <int K>
__global__ __launch_bounds__(kSelNT) void select_kernel(const float* __restrict__ S,
                                                        const uint32_t* __restrict__ mask, int mask_words, Region R,
                                                        Blocks B, int32_t* __restrict__ bips,
                                                        float* __restrict__ bsc, int32_t* __restrict__ bcnt) {
    extern __shared__ uint64_t keys[];   // kSelNT * K
    const int t = threadIdx.x;
    const int bi = blockIdx.x / B.nbx, bj = blockIdx.x - bi * B.nbx;
    const int Hd = max(0, R.H - 2 * R.b), Wd = max(0, R.W - 2 * R.b);
    const int y0 = bound(R.b, Hd, bi, B.nby), y1 = bound(R.b, Hd, bi + 1, B.nby);
    const int x0 = bound(R.b, Wd, bj, B.nbx), x1 = bound(R.b, Wd, bj + 1, B.nbx);
    const int bw = x1 - x0;
    // mask words of the block: rows y0..y1-1, words x0/32 .. (x1-1)/32
    const int w0 = x0 / 32, nw = bw > 0 ? (x1 - 1) / 32 - w0 + 1 : 0;
    const int nwords = (y1 - y0) * nw;
    uint64_t best[K];
#pragma unroll
    for (int i = 0; i < K; ++i) best[i] = ~0ull;
    constexpr int kU = 4;   // mask loads in flight per thread
    for (int q0 = t; q0 < nwords; q0 += kU * kSelNT) {
        uint32_t m[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int q = q0 + u * kSelNT;
            m[u] = 0u;
            if (q < nwords) {
                const int a = q / nw, wi = q - a * nw;
                const int xw = 32 * (w0 + wi);
                uint32_t bits = mask[(int64_t)(y0 + a) * mask_words + w0 + wi];
                if (xw < x0) bits &= ~0u << (x0 - xw);                              // columns before the block
                if (x1 - xw < 32) bits &= (1u << (x1 - xw)) - 1u;                   // columns after it
                m[u] = bits;
            }
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            uint32_t bits = m[u];
            if (!bits) continue;
            const int q = q0 + u * kSelNT;
            const int a = q / nw, xw = 32 * (w0 + q - a * nw);
            while (bits) {
                const int x = xw + __ffs(bits) - 1;
                bits &= bits - 1u;
                const float v = S[(int64_t)(y0 + a) * R.W + x];
                const uint64_t k = make_key(v, (uint32_t)a * (uint32_t)bw + (uint32_t)(x - x0));
                if (k >= best[K - 1]) continue;
                // sorted insertion with compile-time indices
#pragma unroll
                for (int i = K - 1; i > 0; --i) best[i] = k < best[i - 1] ? best[i - 1] : (k < best[i] ? k : best[i]);
                best[0] = k < best[0] ? k : best[0];
            }
        }
    }
#pragma unroll
    for (int i = 0; i < K; ++i) keys[t * K + i] = best[i];
    __syncthreads();
    // bitonic sort, ascending, of kSelNT * K keys
    constexpr int N = kSelNT * K;
    for (int size = 2; size <= N; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = t; i < N / 2; i += kSelNT) {
                const int lo = 2 * i - (i & (stride - 1));
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                const uint64_t a = keys[lo], b = keys[hi];
                if ((a > b) == up) {
                    keys[lo] = b;
                    keys[hi] = a;
                }
            }
            __syncthreads();
        }
    }
    const int base = blockIdx.x * B.per;
    if (t < B.per) {
        const uint64_t k = keys[t];
        if (k != ~0ull) {
            const uint32_t e = (uint32_t)k;
            const int a = (int)(e / (uint32_t)bw), c = (int)(e - (uint32_t)a * (uint32_t)bw);
            bips[2 * (base + t)] = y0 + a;
            bips[2 * (base + t) + 1] = x0 + c;
            bsc[base + t] = __uint_as_float(~(uint32_t)(k >> 32) & 0x7fffffffu);
        }
    }
    if (t == 0) {
        int n = 0;
        for (int i = 0; i < B.per; ++i) n += keys[i] != ~0ull;
        bcnt[blockIdx.x] = n;
    }
}

__global__ __launch_bounds__(kCompNT) void compact_kernel(const int32_t* __restrict__ bips,
                                                          const float* __restrict__ bsc,
                                                          const int32_t* __restrict__ bcnt, int nblocks, int per,
                                                          int32_t* __restrict__ ips, float* __restrict__ scores,
                                                          int32_t* __restrict__ counts, int32_t* __restrict__ n_out) {
    __shared__ int scan[kCompNT];
    const int t = threadIdx.x;
    const int chunk = (nblocks + kCompNT - 1) / kCompNT;
    const int lo = min(nblocks, t * chunk), hi = min(nblocks, lo + chunk);
    int c = 0;
    for (int b = lo; b < hi; ++b) c += bcnt[b];
    scan[t] = c;
    __syncthreads();
    for (int d = 1; d < kCompNT; d <<= 1) {
        const int v = t >= d ? scan[t - d] : 0;
        __syncthreads();
        scan[t] += v;
        __syncthreads();
    }
    int o = scan[t] - c;
    for (int b = lo; b < hi; ++b) {
        const int n = bcnt[b];
        if (counts) counts[b] = n;
        for (int i = 0; i < n; ++i) {
            ips[2 * (o + i)] = bips[2 * (b * per + i)];
            ips[2 * (o + i) + 1] = bips[2 * (b * per + i) + 1];
            if (scores) scores[o + i] = bsc[b * per + i];
        }
        o += n;
    }
    if (t == kCompNT - 1) *n_out = scan[t];
}

struct Layout {
    size_t smap, mask, bips, bsc, bcnt, total;
    int mask_words;
};
Layout layout(int64_t H, int64_t W, int nblocks, int per) {
    Layout L;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += align_up(std::max<size_t>(bytes, 1), 256);
        return at;
    };
    L.mask_words = (int)((W + kTS - 1) / kTS);
    L.smap = take(sizeof(float) * (size_t)H * (size_t)W);
    L.mask = take(sizeof(uint32_t) * (size_t)H * L.mask_words);
    L.bips = take(sizeof(int32_t) * 2 * (size_t)nblocks * per);
    L.bsc = take(sizeof(float) * (size_t)nblocks * per);
    L.bcnt = take(sizeof(int32_t) * (size_t)nblocks);
    L.total = o;
    return L;
}

int check(int64_t H, int64_t W, int nby, int nbx, int per) {
    if (H < 1 || W < 1 || nby < 1 || nbx < 1 || per < 1) return SFOC_E_INVALID_ARG;
    if (H > (1 << 20) || W > (1 << 20) || H * W > ((int64_t)1 << 32) || per > kMaxPer ||
        (int64_t)nby * nbx > kMaxBlocks)
        return SFOC_E_UNSUPPORTED;
    return SFOC_OK;
}

template <int K>
hipError_t launch_select(const float* S, const uint32_t* mask, int mask_words, Region R, Blocks B, int32_t* bips,
                         float* bsc, int32_t* bcnt, hipStream_t st) {
    const size_t lds = sizeof(uint64_t) * kSelNT * K;
    hipError_t e = ensure_dynamic_lds(reinterpret_cast<const void*>(&select_kernel<K>), lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(select_kernel<K>, dim3(B.nby * B.nbx), dim3(kSelNT), lds, st, S, mask, mask_words, R, B, bips,
                       bsc, bcnt);
    return hipGetLastError();
}

}  // namespace fast
}  // namespace sfoc

using namespace sfoc;

extern "C" int sfoc_fast_workspace(int64_t H, int64_t W, int32_t nby, int32_t nbx, int32_t per_block, size_t* bytes) {
    const int rc = fast::check(H, W, nby, nbx, per_block);
    if (rc != SFOC_OK) return rc;
    if (!bytes) return SFOC_E_INVALID_ARG;
    *bytes = fast::layout(H, W, nby * nbx, per_block).total;
    return SFOC_OK;
}

extern "C" int sfoc_detect_ips(const float* img, int64_t H, int64_t W, int64_t ld, float threshold, int32_t margin,
                               int32_t nby, int32_t nbx, int32_t per_block, int32_t* ips, float* scores,
                               int32_t* counts, int32_t* n_out, void* ws, size_t ws_bytes, void* stream) {
    using namespace fast;
    const int rc = check(H, W, nby, nbx, per_block);
    if (rc != SFOC_OK) return rc;
    if (!img || !ips || !n_out || !ws || ld < W || margin < 0 || !(threshold >= 0.f) || !isfinite(threshold))
        return SFOC_E_INVALID_ARG;
    const int nblocks = nby * nbx;
    const Layout L = layout(H, W, nblocks, per_block);
    if (ws_bytes < L.total) return SFOC_E_WORKSPACE;
    char* w = (char*)ws;
    float* S = (float*)(w + L.smap);
    uint32_t* mask = (uint32_t*)(w + L.mask);
    int32_t* bips = (int32_t*)(w + L.bips);
    float* bsc = (float*)(w + L.bsc);
    int32_t* bcnt = (int32_t*)(w + L.bcnt);
    Region R;
    R.b = std::max(3, margin);
    R.H = (int)H;
    R.W = (int)W;
    Blocks B;
    B.nby = nby;
    B.nbx = nbx;
    B.per = per_block;
    hipStream_t st = (hipStream_t)stream;
    const int tiles_x = (int)((W + kTS - 1) / kTS), tiles_y = (int)((H + kTS - 1) / kTS);
    trace_begin(st, SFOC_K_FAST);
    hipLaunchKernelGGL(strength_kernel, dim3(tiles_x * tiles_y), dim3(kNT), 0, st, img, ld, R, threshold, S, mask,
                       L.mask_words, tiles_x);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        const int K = per_block <= 1 ? 1 : per_block <= 2 ? 2 : per_block <= 4 ? 4 : per_block <= 8 ? 8
                    : per_block <= 16 ? 16 : 32;
        switch (K) {
            case 1: e = launch_select<1>(S, mask, L.mask_words, R, B, bips, bsc, bcnt, st); break;
            case 2: e = launch_select<2>(S, mask, L.mask_words, R, B, bips, bsc, bcnt, st); break;
            case 4: e = launch_select<4>(S, mask, L.mask_words, R, B, bips, bsc, bcnt, st); break;
            case 8: e = launch_select<8>(S, mask, L.mask_words, R, B, bips, bsc, bcnt, st); break;
            case 16: e = launch_select<16>(S, mask, L.mask_words, R, B, bips, bsc, bcnt, st); break;
            default: e = launch_select<32>(S, mask, L.mask_words, R, B, bips, bsc, bcnt, st); break;
        }
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(compact_kernel, dim3(1), dim3(kCompNT), 0, st, bips, bsc, bcnt, nblocks, per_block, ips,
                           scores, counts, n_out);
        e = hipGetLastError();
    }
    trace_end(st, SFOC_K_FAST);
    return hip_status(e);
}
