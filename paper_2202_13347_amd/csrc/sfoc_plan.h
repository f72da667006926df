// Plain-data structs passed by value to the kernels, and the host-side
// planning helpers that fill them.  No HIP types here so the host logic can
// be built and tested without a GPU toolchain.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include "sfoc.h"

namespace sfoc {

constexpr int kMaxSig = 2 * SFOC_MAX_SIGMAS;   // distinct sigmas over both orders
constexpr int kMaxHalfTaps = 384;              // sum over sigmas of 3 * (R + 1)
constexpr int kMaxRadius = 24;
constexpr int kMaxQ = 8;                       // K * max(dil)
constexpr int kMaxBase = 25;                   // (2K + 1)^2, K <= 2

// Constants of one SFOC evaluation (Section 2.1), synthesised on the host in
// float64 and rounded to float32.
struct DescribeConsts {
    int32_t nsig;                  // distinct sigmas
    int32_t rad[kMaxSig];          // radius ceil(trunc * sigma)
    int32_t off[kMaxSig];          // offset of this sigma's taps in taps[]
    int32_t use[kMaxSig];          // bit 0: first-order list, bit 1: second-order list
    float   cnorm[kMaxSig];        // 1 / (2 pi sigma^2), the 2-D normalisation of Eq. 1
    float   taps[kMaxHalfTaps];    // per sigma: g[0..R], d[0..R], dd[0..R] (k >= 0 half)
    int32_t N, second, z, Q, R, K, ndil;
    int32_t dil[SFOC_MAX_DIL];
    float   c1[SFOC_MAX_ORIENT], s1[SFOC_MAX_ORIENT];                       // cos, sin
    float   cc[SFOC_MAX_ORIENT], ss[SFOC_MAX_ORIENT], sc2[SFOC_MAX_ORIENT]; // cos^2, sin^2, 2 sin cos
    float   w1[kMaxBase], w2[kMaxBase];   // (2K+1)^2 smoothing base, first / second order
    float   eps;
    int32_t rectify, dtype;
};

// Validate params; fill z.  Returns SFOC_OK or SFOC_E_*.
int check_params(const sfoc_params* p, int32_t* z);
// Build the constants (params must be valid).
int build_describe_consts(const sfoc_params* p, DescribeConsts* c);

// Element size of a descriptor dtype (0 on a bad dtype).
size_t dtype_size(int32_t dtype);

// Integral-image column scan: rows per block.
constexpr int kScanRows = 64;
size_t describe_ws_bytes(int64_t H, int64_t W);

// How a match is laid out: FFT side L and the split of the (2r+1)^2 offsets
// into nb x nb blocks of at most Vb offsets per axis, each with a search
// window of at most L x L.  L = 0 means unsupported.
struct MatchPlan {
    int L, nb, Vb;
    size_t ws_bytes;   // surfaces + per-block records when nb > 1
};
MatchPlan match_plan(int32_t n, int32_t m, int32_t r);
constexpr int kMaxRadiusMatch = 511;

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace sfoc
