// Plain-data structs passed by value to the kernels, and the host-side
// planning helpers that fill them.  No HIP types here so the host logic can
// be built and tested without a GPU toolchain.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <map>
#include <string>
#include <utility>
#include <vector>
#include <tuple>

#include "sfoc.h"

// Layout helpers below are also called by device code when this header is
// compiled for the GPU.
#ifdef __HIPCC__
#define SFOC_HOST_DEVICE __host__ __device__
#else
#define SFOC_HOST_DEVICE
#endif

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

// Side of the square describe tile.
constexpr int kDescribeTile = 32;

// Integral images (Eq. 14-16) are assembled per describe tile from
// aggregates the describe kernel writes for each tile (a, b) and each of the
// two maps (sum_c g and sum_c g^2): the tile's row sums RS[b][y] (global row
// y), column sums CS[a][x] (global column x) and total TT[a][b].  Offsets in
// doubles inside the describe workspace; ntx, nty are the tile counts.
struct IntegAgg {
    int64_t ntx, nty;
    int64_t rs1, rs2, cs1, cs2, tt1, tt2, total;
};
inline SFOC_HOST_DEVICE IntegAgg integ_agg(int64_t H, int64_t W) {
    IntegAgg g;
    g.ntx = (W + kDescribeTile - 1) / kDescribeTile;
    g.nty = (H + kDescribeTile - 1) / kDescribeTile;
    g.rs1 = 0;
    g.rs2 = g.rs1 + g.ntx * H;
    g.cs1 = g.rs2 + g.ntx * H;
    g.cs2 = g.cs1 + g.nty * W;
    g.tt1 = g.cs2 + g.nty * W;
    g.tt2 = g.tt1 + g.nty * g.ntx;
    g.total = g.tt2 + g.nty * g.ntx;
    return g;
}
// Bytes of the aggregates (the describe workspace when integral images are
// asked for): 2 (ntx H + nty W + nty ntx) doubles, about 1 byte per pixel.
size_t describe_ws_bytes(int64_t H, int64_t W);
// Bytes of a one-byte-per-tile mask of an H x W image.
size_t tile_mask_bytes(int64_t H, int64_t W);
// Size of the library-owned aggregate array of sfoc_describe_noalloc.
constexpr size_t kNoAllocScratchBytes = SFOC_NOALLOC_SCRATCH_BYTES;

// Transform sides of the match kernels: L = 16 x NB with NB = 4 (L = 64,
// radices 8 x 8), 8, 10, 12.
constexpr int kNumSides = 4;
constexpr int kSides[kNumSides] = {64, 128, 160, 192};
inline int side_index(int L) {
    for (int k = 0; k < kNumSides; ++k)
        if (kSides[k] == L) return k;
    return -1;
}
// Largest template side: a search window of m + Vb - 1 rows with Vb >= 2
// offsets per block must fit the largest transform.
constexpr int kMaxTemplate = 191;

// The direct form of the match: R_ST (Eq. 10) summed in space on the
// matrix cores instead of through the FFT, for 16-bit descriptors (exact
// MFMA operands), up to 32 offsets per axis (one 32 x 32 output tile) and
// templates up to 64.  Named by the pseudo side kDirectSide wherever a
// transform side is named.
constexpr int kDirectSide = SFOC_MATCH_DIRECT;
constexpr int kDirectMaxV = 32, kDirectMaxM = 64;
inline SFOC_HOST_DEVICE bool direct_ok(int m, int r, int dtype) {
    return (dtype == SFOC_DTYPE_BF16 || dtype == SFOC_DTYPE_F16) && m >= 3 && m <= kDirectMaxM && r >= 1 &&
           2 * r + 1 <= kDirectMaxV;
}
// Launch forms of a batched plan: the transform sides, then the direct form.
constexpr int kNumForms = 5;
constexpr int kForms[kNumForms] = {64, 128, 160, 192, kDirectSide};
inline int form_index(int L) {
    for (int k = 0; k < kNumForms; ++k)
        if (kForms[k] == L) return k;
    return -1;
}

// How a match is laid out: FFT side L and the split of the (2r+1)^2 offsets
// into nb x nb blocks of at most Vb offsets per axis, each with a search
// window of at most L x L.  L = 0 means unsupported.
struct MatchPlan {
    int L, nb, Vb;
    size_t ws_bytes;   // surfaces + per-block records when nb > 1
};
// The default layout: one transform of the smallest side L >= M = m + 2r
// when M <= 192; beyond, offset blocks of the side with the least transform
// work nb^2 L^2 log2 L^2.
MatchPlan match_plan(int32_t n, int32_t m, int32_t r);
// The same for a given side L (one of kSides); L = 0 in the result if the
// template does not fit it (a block needs m + Vb - 1 <= L with Vb >= 2).
// L = kDirectSide: one block of all offsets and no scratch when the sizes
// allow the direct form (its dtype condition is checked by the caller).
MatchPlan match_plan_L(int32_t n, int32_t m, int32_t r, int L);
constexpr int kMaxRadiusMatch = 511;
// Bytes of the per-window integral images (two (M+1)^2 float64 images per
// IP) that the match builds when it is given no integral images.
size_t match_window_ws_bytes(int32_t n, int32_t m, int32_t r);

// Transform sides an autotuner may time for (m, r): the default first, then
// every other side whose plan exists with at most kMaxTuneBlocks offset
// blocks per axis, in increasing L.  Returns the count written to Ls (at
// most kNumSides).
constexpr int kMaxTuneBlocks = 8;
int match_candidates(int32_t m, int32_t r, int* Ls);
// The default form for a descriptor dtype: the direct form where direct_ok
// holds (it is the faster wherever it applies), else match_plan.  Its
// scratch never exceeds match_plan's.
MatchPlan match_plan_dt(int32_t n, int32_t m, int32_t r, int32_t dtype);
// The forms a batched plan's autotuner times for (m, r) and a descriptor
// dtype: the default of match_plan_dt first, then the other transform sides
// of match_candidates.  At most kNumForms.
int plan_candidates(int32_t m, int32_t r, int32_t dtype, int* Ls);

// Autotuner cache: one text line "device z dtype m r L" per (m, r) class
// timed before.  Reading keeps only lines that parse completely and whose
// form L is one of plan_candidates(m, r, dtype) for a positive z and a known
// dtype; anything else in the file (a corrupt or hand-edited line) is
// skipped, so a cached side is always one the match launches accept.
using TuneKey = std::tuple<std::string, int, int, int, int>;   // device, z, dtype, m, r
using TuneCache = std::map<TuneKey, int>;
TuneCache tune_cache_read(const char* path);
// Writes every entry (to path.tmp, then renamed); false on an I/O error.
bool tune_cache_write(const char* path, const TuneCache& cache);
// The cached side for the class, or 0 when there is none or it is not a
// candidate for (m, r) (the caller then times the class or takes the default).
int tune_cache_lookup(const TuneCache& cache, const std::string& dev, int z, int dtype, int m, int r);

// Template-aligned sensed tiles: the describe tiles that cover one IP's
// m x m template exactly, ceil(m / T) rows by ceil(m / T) columns of tiles
// from the template's top-left corner (tiles may run past the template).
// An IP whose template or search window leaves its image reads nothing (it
// is flagged out of bounds) and gets no tiles: template_tile_range returns
// false then, else the template's top-left corner (ty, tx).
inline SFOC_HOST_DEVICE int template_tile_rows(int m, int T) { return (m + T - 1) / T; }
inline SFOC_HOST_DEVICE int template_tile_slots(int m, int T) { return ((m + T - 1) / T) * ((m + T - 1) / T); }
inline SFOC_HOST_DEVICE bool template_tile_range(int py, int px, int pry, int prx, int m, int r, int64_t Hs,
                                                 int64_t Ws, int64_t Hr, int64_t Wr, int64_t* ty, int64_t* tx) {
    const int64_t M = (int64_t)m + 2 * r;
    const int64_t y = (int64_t)py - m / 2, x = (int64_t)px - m / 2;
    const int64_t sy = y - r + pry, sx = x - r + prx;
    if (y < 0 || x < 0 || y + m > Hs || x + m > Ws) return false;
    if (sy < 0 || sx < 0 || sy + M > Hr || sx + M > Wr) return false;
    *ty = y;
    *tx = x;
    return true;
}
// Sensed tiles of all in-bounds IPs (host arrays; prior may be null) as
// distinct (first row, first column) origins.  kCoverTemplate: each IP's
// template-aligned tiles, in IP order (what the pair call describes, but
// without its repeats); kCoverGrid: the tiles of the image's tile grid that
// the templates touch, row-major; kCoverSmaller: the shorter of the two lists
// (the template one on a tie).
constexpr int kCoverTemplate = SFOC_COVER_TEMPLATE, kCoverGrid = SFOC_COVER_GRID, kCoverSmaller = SFOC_COVER_SMALLER;
void sensed_tiles(const int32_t* ips, const int32_t* prior, int32_t n, int32_t m, int32_t r, int64_t Hs,
                  int64_t Ws, int64_t Hr, int64_t Wr, int T, int cover, std::vector<std::pair<int, int>>& out);

// Reference-image tiles (side T) that the match of in-bounds IPs reads:
// every tile holding a pixel of [sy - 1, sy + M) x [sx - 1, sx + M), the
// search window and the row and column before it (whose integral-image
// entries are the box sums' upper-left corners).  window_tile_range gives
// one IP's tile rows [a0, a1] and columns [b0, b1] (false: the IP reads
// nothing); window_tile_mask marks those of all IPs, one byte per tile of
// the Hr x Wr grid, row-major (host arrays; prior may be null).
inline SFOC_HOST_DEVICE bool window_tile_range(int py, int px, int pry, int prx, int m, int r, int64_t Hs,
                                               int64_t Ws, int64_t Hr, int64_t Wr, int T, int64_t* a0, int64_t* a1,
                                               int64_t* b0, int64_t* b1) {
    int64_t ty, tx;
    if (!template_tile_range(py, px, pry, prx, m, r, Hs, Ws, Hr, Wr, &ty, &tx)) return false;
    const int64_t M = (int64_t)m + 2 * r;
    const int64_t sy = (int64_t)py - m / 2 - r + pry, sx = (int64_t)px - m / 2 - r + prx;
    *a0 = (sy > 0 ? sy - 1 : 0) / T;
    *a1 = (sy + M - 1) / T;
    *b0 = (sx > 0 ? sx - 1 : 0) / T;
    *b1 = (sx + M - 1) / T;
    return true;
}
void window_tile_mask(const int32_t* ips, const int32_t* prior, int32_t n, int32_t m, int32_t r, int64_t Hs,
                      int64_t Ws, int64_t Hr, int64_t Wr, int T, uint8_t* mask);

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Image sides are limited so that every per-image index fits in int32 and
// every plane offset in int64; the match kernel addresses a descriptor
// plane with 32-bit element offsets, so a plane holds fewer than 2^30 pixels.
constexpr int64_t kMaxSide = 1 << 16;
constexpr int64_t kMaxPlane = (int64_t)1 << 30;

inline int check_image(const void* img, int64_t H, int64_t W, int64_t ld) {
    if (!img) return SFOC_E_INVALID_ARG;
    if (H < 1 || W < 1 || ld < W) return SFOC_E_INVALID_ARG;
    if (H > kMaxSide || W > kMaxSide) return SFOC_E_UNSUPPORTED;
    return SFOC_OK;
}

inline int check_match_shape(int32_t n, int32_t m, int32_t r) {
    if (n < 0 || m < 3 || r < 1) return SFOC_E_INVALID_ARG;
    if (match_plan(n, m, r).L == 0) return SFOC_E_UNSUPPORTED;
    return SFOC_OK;
}

}  // namespace sfoc
