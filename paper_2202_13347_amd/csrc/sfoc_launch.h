// Kernel argument records and the launch functions behind the C-ABI.  A
// launch either takes one record by value (one image or one pair) or a
// device table of records plus a table of work items (batched plans).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "sfoc_plan.h"

namespace sfoc {

// One image to describe.  A launch covers either the whole tile grid of one
// image or a table of (job, tile row origin, tile column origin) entries
// over several images.
struct DescribeJob {
    const float* img;
    void* desc;
    double* integ1;   // (H+1) x (W+1) per-pixel sum / sum of squares, or null
    double* integ2;
    double* agg;      // per-tile aggregates (layout integ_agg(H, W)) when integ1 is set
    int64_t ld;
    int H, W;
};

// The float64 integral images of one reference image and the per-tile
// aggregates its describe launch wrote (layout integ_agg(H, W)).
struct IntegJob {
    double* g1;
    double* g2;
    double* agg;
    int H, W;
};

// One pair of a match launch.
struct MatchArgs {
    const void* desc_sen;
    const void* desc_ref;
    const double* integ1;
    const double* integ2;
    const int32_t* ips;
    const int32_t* prior;
    float* ncc;
    sfoc_cp* cps;
    float* surf;      // n x V x V scratch surfaces when the offsets are split and ncc == NULL
    float4* blk;      // per (IP, offset block): best score, its index, flags
    int64_t Hs, Ws, Hr, Wr;
    int32_t z, dtype, n, m, r;
    int32_t nbu, nbv, Vb;   // offset blocks per axis and offsets per block
    // 0: integ1 / integ2 are the reference image's integral images; 1: they
    // hold one (M+1) x (M+1) pair per IP, built over its own search window
    int32_t integ_win;
    // Split form (rst set, one offset block): the transforms leave R_ST
    // (n x V x V, row-major) in rst and the template sums R_T, R_TT (2 per
    // IP) in tsum instead of the NCC; ncc_finish_kernel assembles the NCC
    // and the peaks from them and the integral images.
    float* rst = nullptr;
    double* tsum = nullptr;
};

// SFOC_OK for hipSuccess, else SFOC_E_HIP (the HIP error is kept for
// sfoc_status_string).
int hip_status(hipError_t e);

// Raises a kernel's dynamic-LDS limit on the current device to at least
// `bytes`, once per (kernel, device, size): later launches, including those
// recorded under stream capture, make no attribute call.
hipError_t ensure_dynamic_lds(const void* kern, int bytes);

// ---- one image / one pair ------------------------------------------------
// i1, i2 and agg (the aggregates, describe_ws_bytes) all null, or all set.
// tmask (one byte per tile, row-major, or null): tiles outside it are not
// described (their aggregates, when asked for, are set to zero).
hipError_t launch_describe(const float* img, int H, int W, int64_t ld, void* desc, double* i1, double* i2,
                           double* agg, const DescribeConsts& c, hipStream_t st, const uint8_t* tmask = nullptr);
// The tiles of one image that a device table lists ({0, row origin, column
// origin, 0}; entries with a negative first field are skipped), without
// integral-image inputs.
hipError_t launch_describe_tiles(const float* img, int H, int W, int64_t ld, void* desc, const int4* tiles,
                                 int ntiles, const DescribeConsts& c, hipStream_t st);
// Entries of the pair call's describe table: the reference image's grid
// tiles, then n * template_tile_slots(m, kDescribeTile) sensed slots.
int64_t pair_table_entries(int Hr, int Wr, int n, int m);
// Both images of a pair in one describe launch (n IPs, device arrays): a
// small kernel marks in mask (one byte per reference tile) the tiles each
// in-bounds IP's search window reads (window_tile_range) and writes the two
// jobs and the table (pair_table_entries entries); the describe launch then
// takes the reference tiles the mask marks (the others get zero aggregates)
// and the template-aligned sensed tiles.  Mask bytes are not cleared here:
// launch_integral, the last reader, clears every byte of the grid.
hipError_t launch_describe_pair(const float* ref, int Hr, int Wr, int64_t ldr, void* dref, double* i1, double* i2,
                                double* agg, const float* sen, int Hs, int Ws, int64_t lds, void* dsen,
                                const int32_t* ips, const int32_t* prior, int n, int m, int r, DescribeJob* jobs,
                                int4* tiles, uint8_t* mask, const DescribeConsts& c, hipStream_t st);
// Completes the integral images from what launch_describe left in i1, i2
// and agg (the same buffers).
hipError_t launch_integral(double* i1, double* i2, int H, int W, double* agg, hipStream_t st,
                           uint8_t* tmask = nullptr);
// i1 == i2 == null: per-window integral images, built into ws after the
// split-offset scratch (match_window_ws_bytes).
// consistency = false leaves out the median-displacement check (see
// launch_consistency).
hipError_t launch_match(const void* desc_sen, int64_t Hs, int64_t Ws, const void* desc_ref, int64_t Hr, int64_t Wr,
                        const double* i1, const double* i2, int z, int dtype, const int32_t* ips,
                        const int32_t* prior, int n, int m, int r, float* ncc, sfoc_cp* cps, void* ws,
                        hipStream_t st, bool consistency = true);
// The same match in two launches, so that the integral images need not
// exist before the second: launch_match_fft runs the transforms and leaves
// R_ST and the template sums in `split` (match_split_bytes(n, r) bytes);
// launch_match_finish assembles the NCC surfaces (ncc, if set) and the
// peaks into cps from them and the integral images, then (consistency) the
// median check.  Only where match_split_ok: an FFT side without offset
// blocks.  ws is launch_match's workspace.
bool match_split_ok(int n, int m, int r, int dtype);
size_t match_split_bytes(int n, int r);
hipError_t launch_match_fft(const void* desc_sen, int64_t Hs, int64_t Ws, const void* desc_ref, int64_t Hr,
                            int64_t Wr, int z, int dtype, const int32_t* ips, const int32_t* prior, int n, int m,
                            int r, float* ncc, sfoc_cp* cps, void* ws, void* split, hipStream_t st);
hipError_t launch_match_finish(const void* desc_sen, int64_t Hs, int64_t Ws, const void* desc_ref, int64_t Hr,
                               int64_t Wr, const double* i1, const double* i2, int z, int dtype, const int32_t* ips,
                               const int32_t* prior, int n, int m, int r, float* ncc, sfoc_cp* cps, void* ws,
                               void* split, hipStream_t st, bool consistency);
// The median-displacement consistency check over n records (one workgroup).
hipError_t launch_consistency(sfoc_cp* cps, const int32_t* prior, int n, hipStream_t st);
// cps[i].sen_row += dy for i < n.
hipError_t launch_cp_row_shift(sfoc_cp* cps, int n, int dy, hipStream_t st);
// Fills the offset-block fields and scratch pointers of `a` for transform
// side L (a.surf / a.blk point into ws, whose size is match_plan_L().ws_bytes).
void match_args_layout(MatchArgs& a, const MatchPlan& mp, void* ws);

// ---- tables (device pointers) --------------------------------------------
// tiles[k] = {job, tile row origin, tile column origin, 0}; var picks the
// launch configuration (0, or 1 where describe_configs() is 2): the same
// descriptors either way.
hipError_t launch_describe_batched(const DescribeJob* jobs, const int4* tiles, int ntiles, const DescribeConsts& c,
                                   hipStream_t st, int var = 0);
// Launch configurations of the describe kernel for these constants (1 or 2).
int describe_configs(const DescribeConsts& c);
// pre[k] = {job, kind, block, 0}: kind 0 a block of kScanNT rows of the
// row sums, 1 a block of kScanNT columns of the column sums, 2 the tile
// totals (integral_prefix_items lists them); tiles[k] = {job, tile row,
// tile column, 0} over every tile of every image
hipError_t launch_integral_batched(const IntegJob* jobs, const int4* pre, int npre, const int4* tiles, int ntiles,
                                   hipStream_t st);
// Threads per workgroup of the integral kernels, and the prefix work items
// of one image.
constexpr int kScanNT = 256;
void integral_prefix_items(int job, int H, int W, std::vector<int4>& out);
// Size of a direct-form launch: the largest template side and chunk count
// of the pairs it covers (direct_launch_of for one pair; componentwise
// maxima for several).
struct DirLaunch {
    int m, nkb;
};
DirLaunch direct_launch_of(int m, int r);
// items[k] = {pair, IP, offset block, 0}, all with transform side L; one
// workgroup per item, or (counter != null) a persistent grid of `grid`
// workgroups taking items from *counter (zeroed by the launch).  The direct
// form (L = kDirectSide, 16-bit dtypes) has no persistent grid and is sized
// by `dir`.
hipError_t launch_match_items(int L, int dtype, const MatchArgs* pairs, const int4* items, int nitems, int* counter,
                              int grid, DirLaunch dir, hipStream_t st);
// items[k] = {pair, first IP of a run of 256, 0, 0} over pairs with split offsets
hipError_t launch_peak_batched(const MatchArgs* pairs, const int4* items, int nitems, hipStream_t st);
// one workgroup per pair
hipError_t launch_consistency_batched(const MatchArgs* pairs, int npairs, hipStream_t st);

}  // namespace sfoc
