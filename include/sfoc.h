/*
 * sfoc.h -- C ABI of the MI355X (gfx950) SFOC / Fast-NCC_SFOC library.
 *
 * Method: Ye et al., "A Robust Multimodal Remote Sensing Image Registration
 * Method and System Using Steerable Filters with First- and Second-order
 * Gradients" (arXiv 2202.13347).  The library implements the data-parallel
 * part of the fine-registration stage (Section 3.2): dense SFOC descriptors
 * (Section 2.1, Eq. 1-7) and CP detection by template matching with
 * Fast-NCC_SFOC (Section 2.2, Eq. 8-16; Section 3.2.2).
 *
 * Conventions shared by every entry point
 *  - Images are single-band float32, row-major, origin top-left; x is the
 *    column, y the row (growing downwards).  `ld` is the row pitch in
 *    elements (ld >= W).
 *  - Descriptors are channel-planar: desc[c][y][x], row pitch W, channel
 *    pitch H*W, c in [0, z).  Channels 0..N-1 are the first-order channels at
 *    directions k*pi/N, channels N..2N-1 the second-order ones (absent when
 *    second_order == 0).  Element type: float32, bfloat16 or float16
 *    (sfoc_params.desc_dtype; bf16/f16 are rounded to nearest even).
 *  - Integral feature images (Eq. 14-16) are float64, (H+1) x (W+1),
 *    row-major with pitch W+1, zero first row and column:
 *    integ1[y][x] = sum over rows < y, columns < x, channels of g;
 *    integ2 the same for g^2.  They are built from the stored (rounded)
 *    descriptor values.
 *  - Every pointer argument except `p`, `bytes` and outputs documented as
 *    host memory is a DEVICE pointer on the current HIP device.  The caller
 *    owns all buffers, including the workspace.  No entry point allocates
 *    or frees device memory.
 *  - Work is enqueued asynchronously on `stream` (a hipStream_t; NULL is the
 *    null stream).  The caller synchronises before reading results.
 *  - Return value: SFOC_OK (0) or a negative SFOC_E_* code.  Argument errors
 *    are detected on the host before anything is enqueued.  Data-dependent
 *    conditions (flat windows, windows leaving the image, non-finite values)
 *    are never call failures: they are reported per CP in sfoc_cp.flags.
 */
#ifndef SFOC_H
#define SFOC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define SFOC_OK              0
#define SFOC_E_INVALID_ARG  (-1)  /* null pointer, bad size, z != channels, ... */
#define SFOC_E_UNSUPPORTED  (-2)  /* valid but outside what the kernels support */
#define SFOC_E_WORKSPACE    (-3)  /* workspace smaller than the *_workspace query */
#define SFOC_E_HIP          (-4)  /* a HIP launch or runtime call failed */

/* ---- descriptor element types ---------------------------------------- */
#define SFOC_DTYPE_F32   0
#define SFOC_DTYPE_BF16  1
#define SFOC_DTYPE_F16   2

/* ---- rectification of the steered responses -------------------------- */
#define SFOC_RECTIFY_ABS     0   /* |F| (default; contrast-reversal invariant) */
#define SFOC_RECTIFY_SIGNED  1
#define SFOC_RECTIFY_RELU    2

/* ---- per-CP flags ------------------------------------------------------ */
#define SFOC_CP_VALID         1u    /* usable CP: none of the bits below      */
#define SFOC_CP_OOB           2u    /* template or search window leaves image */
#define SFOC_CP_FLAT_T        4u    /* template variance <= tau               */
#define SFOC_CP_FLAT_S        8u    /* search variance <= tau at every offset */
#define SFOC_CP_EDGE_PEAK    16u    /* argmax on the border of the surface    */
#define SFOC_CP_INCONSISTENT 32u    /* > 1.5 px from the median displacement  */
#define SFOC_CP_LEARNED      64u    /* sub-pixel part from the learned head   */
#define SFOC_CP_NONFINITE   128u    /* a non-finite value reached the surface */

#define SFOC_MAX_SIGMAS   8
#define SFOC_MAX_DIL      4
#define SFOC_MAX_ORIENT  16

/*
 * SFOC parameters (Section 2.1).
 *  n_orient      N, directions k*pi/N, k = 0..N-1 (the paper uses 6); 1..16.
 *  s1[n_s1]      standard deviations of the first-order channels; the
 *                steered responses are summed over them (Table 2).
 *  s2[n_s2]      the same for the second-order channels.
 *  trunc         kernel radius = ceil(trunc * sigma), kernels point sampled.
 *  sd1, sd2      standard deviation of the (2K+1)^2 Gaussian base of the
 *                dilated smoothing for first- / second-order channels.
 *  K             half-size of that base (1 -> 3x3).
 *  dil[n_dil]    dilation rates; the dilated responses are summed ({1,2,3}).
 *  eps           added under the root of the per-order L2 normalisation.
 *  rectify       SFOC_RECTIFY_*.
 *  second_order  1: SFOC (z = 2N); 0: first-order channels only (z = N).
 *  desc_dtype    SFOC_DTYPE_* of the stored descriptor.
 * Limits: radius <= 24 (sigma*trunc), K*max(dil) <= 8, n_dil*... see
 * sfoc_params_check.
 */
typedef struct sfoc_params {
    int32_t n_orient;
    int32_t n_s1;
    double  s1[SFOC_MAX_SIGMAS];
    int32_t n_s2;
    int32_t n_dil;
    double  s2[SFOC_MAX_SIGMAS];
    double  trunc;
    double  sd1;
    double  sd2;
    double  eps;
    int32_t K;
    int32_t dil[SFOC_MAX_DIL];
    int32_t rectify;
    int32_t second_order;
    int32_t desc_dtype;
} sfoc_params;

/*
 * One control point (32 bytes).  The reference point matched to the sensed
 * point (sen_row, sen_col) is
 *   (sen_row + prior_y + dy + sub_dy, sen_col + prior_x + dx + sub_dx),
 * dy, dx in [-r, r] the integer argmax of the NCC surface (Section 3.2.2),
 * sub_* in [-0.5, 0.5] its parabola refinement, score the NCC at the
 * integer peak.  Records with OOB / FLAT_* / NONFINITE have dy = dx = 0,
 * sub_* = 0 and score = 0.
 */
typedef struct sfoc_cp {
    int32_t  sen_row, sen_col;
    int32_t  dy, dx;
    float    sub_dy, sub_dx;
    float    score;
    uint32_t flags;
} sfoc_cp;

/* Human-readable text of a status code (static storage). */
const char* sfoc_status_string(int status);

/*
 * Fill *p with a preset: 0 = the paper's (N = 6; first-order sigma 0.6,
 * 0.8, 1.0 and second-order sigma 1.5, Section 2.1 and Table 2; rates 1,2,3),
 * 1 = baseline (N = 8; sigma 1, 2, 3 for both orders).  Both use trunc 3,
 * K = 1, sd1 = 1.0, sd2 = 1.5, eps = 1e-8, |.| rectification, float32.
 * Host only.  Returns SFOC_E_INVALID_ARG for an unknown preset or p == NULL.
 */
int sfoc_params_preset(int32_t which, sfoc_params* p);

/* Validate parameters; writes the channel count z to *z (may be NULL). */
int sfoc_params_check(const sfoc_params* p, int32_t* z);

/*
 * Dense SFOC descriptor of one image (Section 2.1): steered first- and
 * second-order Gaussian-derivative responses summed over scales, rectified,
 * smoothed by the dilated Gaussians, normalised per order, stacked.  The
 * image is extended by reflect-101 and every stage is evaluated on the
 * extended domain.
 *  img      H x W float32, pitch ld.                        (input)
 *  desc     z planes of H x W, element type p->desc_dtype.  (output)
 *  integ1,  (H+1) x (W+1) float64 integral images of sum_c g and sum_c g^2
 *  integ2   of the stored values, or both NULL to skip them. (output)
 *  ws       workspace of at least sfoc_describe_workspace() bytes (may be
 *           NULL if that is 0).
 * Errors: SFOC_E_INVALID_ARG (null img/desc/p, H or W < 1, ld < W, only one
 * of integ1/integ2 NULL, bad params), SFOC_E_WORKSPACE, SFOC_E_HIP.
 */
int sfoc_describe_workspace(int64_t H, int64_t W, const sfoc_params* p, size_t* bytes);
int sfoc_describe(const float* img, int64_t H, int64_t W, int64_t ld,
                  const sfoc_params* p, void* desc, double* integ1, double* integ2,
                  void* ws, size_t ws_bytes, void* stream);

/*
 * sfoc_describe with integral images, allocating nothing: for callers that
 * cannot allocate device memory (code under HIP stream capture, serving
 * loops, harnesses that forbid allocation).  Arguments, results and errors
 * are sfoc_describe's with integ1 and integ2 required (non-NULL) and no
 * workspace: the per-tile aggregates the integral images are assembled from
 * live in a library-owned device array of SFOC_NOALLOC_SCRATCH_BYTES (one
 * per GPU, held until the process ends).  Images whose aggregates
 * (sfoc_describe_workspace) exceed it are rejected with SFOC_E_UNSUPPORTED
 * (about 8000 x 8000 pixels is the largest square image).  Every call on a
 * GPU shares that GPU's array: calls that overlap on one GPU (different
 * streams, or host threads) race and must be serialised by the caller.  The
 * results equal sfoc_describe's bit for bit.  Errors: SFOC_E_INVALID_ARG
 * (as sfoc_describe, or integ1 / integ2 NULL), SFOC_E_UNSUPPORTED, SFOC_E_HIP.
 */
#define SFOC_NOALLOC_SCRATCH_BYTES (64u << 20)
int sfoc_describe_noalloc(const float* img, int64_t H, int64_t W, int64_t ld, const sfoc_params* p,
                          void* desc, double* integ1, double* integ2, void* stream);

/*
 * Fast-NCC_SFOC CP detection for n interest points of one image pair
 * (Section 2.2, Eq. 9-16; Section 3.2.2).  For IP i at (row, col) in the
 * sensed image, the template is the m x m x z window with top-left
 * (row - m/2, col - m/2) of desc_sen; the search window is the M x M x z
 * window, M = m + 2r, with top-left (row - m/2 - r + prior_y,
 * col - m/2 - r + prior_x) of desc_ref.  NCC (Eq. 9, one mean over all
 * m*m*z entries) is evaluated at all (2r+1)^2 offsets; R_ST by FFT
 * (Eq. 13), R_S and R_SS by four lookups in the float64 integral images of
 * desc_ref (Eq. 16), the variance subtraction in float64.  Offsets whose
 * search variance is <= tau = 1e-12*m*m*z score 0.  The CP is the argmax
 * (ties: smallest row-major offset index) refined per axis by a three-point
 * parabola; then a median-displacement consistency check at 1.5 px sets
 * INCONSISTENT / VALID.
 *  desc_sen, desc_ref  descriptors (layout above), z channels, element type dtype.
 *  integ1, integ2      integral images of desc_ref ((Hr+1) x (Wr+1) float64),
 *                      or both NULL: then each IP's pair of integral images
 *                      is built over its own search window ((M+1) x (M+1)
 *                      float64, the per-pixel channel sums of the stored
 *                      values, Eq. 14-15) inside ws, which must then hold
 *                      sfoc_match_window_workspace bytes.
 *  ips                 n x 2 int32 (row, col) in the sensed image.
 *  prior               n x 2 int32 (dy, dx) search-window offsets, or NULL.
 *  ncc                 n x (2r+1) x (2r+1) float32 surfaces, or NULL.  (output)
 *  cps                 n records.                                      (output)
 * The transform side L is the smallest of 64, 128, 160 and 192 (radices
 * 8 x 8, 16 x 8, 16 x 10, 16 x 12) that holds the search window, so windows
 * up to 192 x 192 (m + 2r <= 192) are one transform.  Larger ones split the
 * offsets into blocks whose windows fit L x L, with the side of least
 * transform work, and need the workspace sfoc_match_workspace reports
 * (per-CP surfaces and block records; 0 bytes otherwise).
 * With BFLOAT16 / FLOAT16 descriptors, 2r + 1 <= 32 and m <= 64, R_ST is
 * instead summed in space on the matrix cores (the direct form,
 * SFOC_MATCH_DIRECT; exact 16-bit products, float32 sums in another order,
 * no workspace beyond the integral-mode one).
 * Limits: 3 <= m <= 191, 1 <= r <= 511, each image below 2^30 pixels
 * (SFOC_E_UNSUPPORTED beyond).
 * n == 0 is valid and enqueues nothing.
 * Errors: SFOC_E_INVALID_ARG (null descriptors, ips or cps, only one of
 * integ1 / integ2 NULL, m < 3, r < 1, z < 1, unknown dtype, sizes < 1),
 * SFOC_E_UNSUPPORTED, SFOC_E_WORKSPACE (ws smaller than the query for the
 * chosen integral mode), SFOC_E_HIP.
 */
int sfoc_match_workspace(int32_t n, int32_t m, int32_t r, int32_t z, size_t* bytes);
int sfoc_match_window_workspace(int32_t n, int32_t m, int32_t r, int32_t z, size_t* bytes);
int sfoc_fastncc_match(const void* desc_sen, int64_t Hs, int64_t Ws,
                       const void* desc_ref, int64_t Hr, int64_t Wr,
                       const double* integ1, const double* integ2,
                       int32_t z, int32_t dtype,
                       const int32_t* ips, const int32_t* prior, int32_t n,
                       int32_t m, int32_t r,
                       float* ncc, sfoc_cp* cps,
                       void* ws, size_t ws_bytes, void* stream);

/*
 * Whole fine-registration hot path for one pair: sfoc_describe of the
 * reference image's 32 x 32 tiles that the search windows read (and the row
 * and column before each window, which hold the box sums' upper-left
 * corners) and of the sensed image's tiles that the templates read (an
 * m x m template at each IP, Section 2.2), integral images of the
 * reference, then sfoc_fastncc_match.  Reference tiles no window reads are
 * not described and count as zero in the integral images, so every box sum
 * a window takes is that of the described values.  Both images' tiles go
 * into one describe launch.  Where the match runs on an FFT side without
 * offset blocks, the integral scans run on a second stream beside the
 * match's transforms (one library-owned, non-blocking, default-priority
 * stream per device and host thread, created on first use with its two
 * events); `stream` waits for it before the NCC assembly, so all later work
 * on `stream` is ordered after the call.  Arguments as above; the
 * descriptors, integral images, the describe table of both images' tiles,
 * the match's R_ST surfaces and the reference tile mask live inside ws (see
 * sfoc_register_workspace).  The CPs equal
 * those of sfoc_describe of both whole images followed by sfoc_fastncc_match
 * up to the float64 rounding of those box sums (bit for bit in every test).
 */
int sfoc_register_workspace(int64_t Hr, int64_t Wr, int64_t Hs, int64_t Ws,
                            int32_t n, int32_t m, int32_t r,
                            const sfoc_params* p, size_t* bytes);
int sfoc_register_cps(const float* ref, int64_t Hr, int64_t Wr, int64_t ldr,
                      const float* sen, int64_t Hs, int64_t Ws, int64_t lds,
                      const int32_t* ips, const int32_t* prior, int32_t n,
                      int32_t m, int32_t r, const sfoc_params* p,
                      float* ncc, sfoc_cp* cps,
                      void* ws, size_t ws_bytes, void* stream);

/*
 * The pair call streamed over bands of rows, for scenes whose descriptors
 * and integral images should not be resident whole (Section 2.2 as in
 * sfoc_register_cps; the same kernels).  IPs must be sorted by row
 * (non-decreasing; SFOC_E_INVALID_ARG otherwise) and every row prior must
 * satisfy |dy| <= max_prior.  A band holds the IPs whose rows lie in
 * [y0, y0 + band_rows), y0 the first remaining IP's row; for each band the
 * pair call runs on the reference and sensed rows its search windows and
 * templates read, widened by the descriptor's filter reach (so every row
 * read has the whole image's descriptors) and clipped to the images, with
 * the band's IP rows and priors taken relative to those rows.  The records
 * are then put back in whole-image rows, and one median-displacement check
 * runs over all n CPs.  The workspace (sfoc_register_streamed_workspace)
 * holds one band: band_rows + m + 2r + 2 max_prior rows of the reference
 * (plus the reach) instead of all Hr.  Integer CPs, flags and records equal
 * the pair call's on the whole images up to the float64 rounding of box
 * sums taken from band-relative integral images.
 * The call reads the IPs (and priors) to the host and synchronises `stream`
 * twice before its launches (the band plan is made on the host); the rest
 * is asynchronous on `stream`.
 * Errors: those of sfoc_register_cps; SFOC_E_INVALID_ARG for band_rows < 1,
 * max_prior < 0, unsorted IPs or a prior beyond max_prior.
 */
int sfoc_register_streamed_workspace(int64_t Hr, int64_t Wr, int64_t Hs, int64_t Ws,
                                     int32_t n, int32_t m, int32_t r, int32_t band_rows,
                                     int32_t max_prior, const sfoc_params* p, size_t* bytes);
int sfoc_register_cps_streamed(const float* ref, int64_t Hr, int64_t Wr, int64_t ldr,
                               const float* sen, int64_t Hs, int64_t Ws, int64_t lds,
                               const int32_t* ips, const int32_t* prior, int32_t n,
                               int32_t m, int32_t r, int32_t band_rows, int32_t max_prior,
                               const sfoc_params* p, float* ncc, sfoc_cp* cps,
                               void* ws, size_t ws_bytes, void* stream);

/*
 * Batched registration of many image pairs (uneven sizes, templates and
 * radii) as one plan.  Each pair is what sfoc_register_cps takes for one
 * pair; every pair is computed exactly as sfoc_register_cps computes it
 * with the same transform side (Section 2.2, Eq. 9-16 and the peak and
 * consistency decisions per pair), so with the default sides the results
 * are bit-identical to per-pair calls.
 *
 * sfoc_plan_create validates every pair, allocates the plan's device memory
 * (descriptors, integral images, scratch and the launch tables; it is the
 * only call of this library that allocates) and builds the work lists:
 *  - describe: one launch over (image, 32 x 32 tile) entries of all images;
 *    a reference image gets the tiles its search windows read, as in
 *    sfoc_register_cps (the others only zero integral-image aggregates);
 *    a sensed image gets only the tiles over its templates, the shorter of
 *    the two lists of sfoc_sensed_tiles (SFOC_COVER_SMALLER); with
 *    SFOC_PLAN_DENSE_SEN both images are described whole;
 *  - integral images: three launches over the read tiles of all reference
 *    images;
 *  - match: one launch per transform side over (pair, IP, offset block)
 *    items, side 64 on a second graph branch beside the larger sides; a
 *    peak launch over pairs
 *    whose offsets are split; one consistency launch, a workgroup per pair.
 * The transform side of a pair is pair.fft_side when that is 64, 128, 160
 * or 192 (SFOC_E_UNSUPPORTED if the template does not fit it), else the default of
 * sfoc_match_workspace, or with SFOC_PLAN_AUTOTUNE the faster of the
 * candidates sfoc_match_candidates lists, timed on the plan's own work at
 * creation (the images should hold data by then) and remembered per
 * (device, z, dtype, m, r) in the text file tune_cache when that is not
 * NULL (read at creation, rewritten when a new entry was timed).
 * With SFOC_PLAN_GRAPH the first sfoc_register_cps_batched captures the
 * whole sequence on its stream into a hipGraph and every call replays it.
 * Match launches are one workgroup per item, or persistent grids (about two
 * workgroups per CU taking items from a counter) with SFOC_PLAN_PERSISTENT;
 * with SFOC_PLAN_AUTOTUNE each transform side's launch form is also timed
 * at creation and the faster kept.
 * The describe launch has two configurations of its 32 x 32 tile where the
 * parameters allow (K = 1, dilation rates 1, 2, 3, both orders, z <= 16):
 * 0, three workgroups per CU; 1, four workgroups per CU with half-width
 * row-pass maps and one steered channel map at a time.  Both give the same
 * descriptors bit for bit.  SFOC_PLAN_DESCRIBE_ALT selects configuration 1;
 * with SFOC_PLAN_AUTOTUNE both are timed on the plan's tiles at creation
 * and the faster kept (not remembered in tune_cache).
 *
 * Ownership and lifetime: the caller owns every pair buffer (device
 * pointers) and keeps them allocated for the plan's lifetime; the plan
 * reads the image contents at each execution.  The IP and prior values are
 * read once at creation (host copies) when the sensed images are described
 * sparsely (both images) or the plan is autotuned; they must not change afterwards unless
 * SFOC_PLAN_DENSE_SEN is set and autotuning is off.  create synchronises
 * `stream`; execute is asynchronous on `stream`.  A plan is used by one
 * host thread at a time and on the device that was current at creation.
 * Errors: SFOC_E_INVALID_ARG (null plan or pairs, n_pairs < 1, a pair
 * failing the sfoc_register_cps checks), SFOC_E_UNSUPPORTED, SFOC_E_HIP
 * (including out of device memory).
 */
typedef struct sfoc_pair {
    const float* ref;           /* Hr x Wr float32, pitch ldr (elements) */
    int64_t Hr, Wr, ldr;
    const float* sen;           /* Hs x Ws float32, pitch lds */
    int64_t Hs, Ws, lds;
    const int32_t* ips;         /* n x 2 (row, col) in the sensed image */
    const int32_t* prior;       /* n x 2 (dy, dx) or NULL */
    int32_t n, m, r;
    int32_t fft_side;           /* 0: default / autotuned; 64, 128, 160, 192: forced;
                                   SFOC_MATCH_DIRECT: the direct form, forced */
    float* ncc;                 /* n x (2r+1)^2 float32 surfaces or NULL (output) */
    sfoc_cp* cps;               /* n records (output) */
} sfoc_pair;

typedef struct sfoc_plan sfoc_plan;

/* Pseudo transform side naming the direct form of the match: R_ST (Eq. 10)
 * summed in space on the matrix cores rather than through the FFT.  For
 * BFLOAT16 / FLOAT16 descriptors (exact operands, float32 accumulation),
 * 2r + 1 <= 32 and m <= 64; SFOC_E_UNSUPPORTED otherwise. */
#define SFOC_MATCH_DIRECT 1

#define SFOC_PLAN_GRAPH       1
#define SFOC_PLAN_AUTOTUNE    2
#define SFOC_PLAN_DENSE_SEN   4
#define SFOC_PLAN_PERSISTENT  8
#define SFOC_PLAN_DESCRIBE_ALT 16

int sfoc_plan_create(const sfoc_pair* pairs, int32_t n_pairs, const sfoc_params* p, int32_t flags,
                     const char* tune_cache, void* stream, sfoc_plan** plan);
int sfoc_register_cps_batched(sfoc_plan* plan, void* stream);
int sfoc_plan_destroy(sfoc_plan* plan);

/*
 * What a plan chose and holds.  fft_side[i] / blocks[i] (per axis) for the
 * first min(n_pairs, cap) pairs; the totals of work items and device bytes.
 */
typedef struct sfoc_plan_info {
    int32_t n_pairs;
    int32_t describe_tiles;     /* entries of the describe launch */
    int32_t match_items[4];     /* items of the L = 64, 128, 160, 192 launches */
    int32_t peak_items;
    int32_t tuned_classes;      /* (m, r) classes timed at creation */
    int32_t cached_classes;     /* (m, r) classes taken from tune_cache */
    int32_t graph;              /* 1 once a graph is captured */
    int32_t persistent[4];      /* those launches persistent (1) or one workgroup per item */
    int32_t describe_config;    /* describe launch configuration: 0, or 1 (four workgroups per CU) */
    int32_t direct_items;       /* items of the direct-form launch (SFOC_MATCH_DIRECT) */
    int64_t device_bytes;
} sfoc_plan_info;
int sfoc_plan_get_info(const sfoc_plan* plan, sfoc_plan_info* info, int32_t* fft_side, int32_t* blocks,
                       int32_t cap);

/*
 * Planning queries (host only, no device work).
 * sfoc_match_candidates: the transform sides (64 / 128 / 160 / 192) usable
 * for template m and radius r with at most 8 offset blocks per axis, the
 * default first and the others by increasing side, and the offset blocks per
 * axis of each; returns the count (0: none; at most 4).  With 16-bit
 * descriptors a plan's autotuner also times the direct form where it
 * applies, and takes it as the default there.
 * sfoc_sensed_tiles: 32 x 32 sensed-image tiles that cover the m x m
 * templates of the in-bounds IPs (template and search window inside their
 * images; host arrays, no device work).  Tiles may run past a template;
 * they are clipped to the image.
 *   SFOC_COVER_TEMPLATE: per IP, ceil(m/32) x ceil(m/32) tiles from the
 *     template's top-left corner, in IP order (what sfoc_register_cps
 *     describes, which also describes twice what tiles of two IPs share);
 *   SFOC_COVER_GRID: the tiles of the image's 32-grid that templates touch,
 *     row-major;
 *   SFOC_COVER_SMALLER: the shorter of the two (the template list on a
 *     tie), what a sparse plan describes.
 * The distinct tiles go to origins as (row, column) pairs, at most cap of
 * them (origins may be null when cap is 0); returns the number of distinct
 * tiles, or a negative status (SFOC_E_INVALID_ARG for an unknown cover).
 */
#define SFOC_COVER_TEMPLATE 0
#define SFOC_COVER_GRID     1
#define SFOC_COVER_SMALLER  2
int sfoc_match_candidates(int32_t m, int32_t r, int32_t* fft_side, int32_t* blocks, int32_t cap);
int64_t sfoc_sensed_tiles(const int32_t* ips, const int32_t* prior, int32_t n, int32_t m, int32_t r,
                          int64_t Hs, int64_t Ws, int64_t Hr, int64_t Wr, int32_t cover, int32_t* origins,
                          int64_t cap);

/*
 * Learned CP-validity and sub-pixel head (not part of the paper).  It reads
 * what the paper's matching produces, the NCC surface of Eq. 9 around the
 * argmax CP (Section 3.2.2), and is trained against the 1.5 px correctness
 * threshold of Section 4.1; the plain peak fit and consistency check stay the
 * fallback for every CP it does not take.
 *
 * Features (sfoc_head_features), per CP with an interior peak (flags VALID
 * or INCONSISTENT; every other CP gets zeros):
 *   crops  n x 33 x 33 float32: the surface around the integer peak
 *          (u*, v*) = (dy + r, dx + r), crop[a][b] = S[u*-16+a][v*-16+b],
 *          -1 outside the (2r+1)^2 surface;
 *   stats  n x 8 float32: peak; the largest value outside the 3 x 3 block
 *          around the peak (-1 if none); surface mean; surface standard
 *          deviation; template standard deviation sqrt(max(varT,0)/mnz)
 *          (Eq. 11-12, mnz = m*m*z); search-window standard deviation at the
 *          peak from the integral images (Eq. 16); template mean R_T/mnz;
 *          the mean of the two second differences at the peak.
 *   Arguments as for sfoc_fastncc_match, plus ncc (n x (2r+1)^2 surfaces it
 *   wrote) and cps (its records).
 *
 * Network (parameters: SFOC_HEAD_PARAMS float32 in this order): conv1 3x3
 * 1->32 stride 1; conv2..conv4 3x3 32->32 stride 2 (33 -> 33 -> 17 -> 9 ->
 * 5, zero padding 1, ReLU after each); fc1 (800 channel-major values + the 8
 * stats) -> 32, ReLU; fc2 32 -> 3 = (validity logit, oy, ox).  Conv
 * weights are [out][in][3][3] then the bias [out]; fc weights [out][in]
 * then the bias.  Weights (not biases) enter every product rounded to
 * bfloat16 (round to nearest even); all sums are float32.
 *
 * sfoc_head_forward: out (n x 3) for n samples.
 * sfoc_head_train_step: one step on a batch of n samples: forward, the
 *   loss mean_b[ BCE(logit, label) + 4 label (SmoothL1(oy - ty) +
 *   SmoothL1(ox - tx)) ] with SmoothL1 of width 0.1, its gradient w.r.t. the
 *   rounded weights applied to the float32 master params (straight
 *   through), written to grad (SFOC_HEAD_PARAMS floats, may be NULL) and
 *   loss (one float, may be NULL), then an Adam update (beta1 0.9, beta2
 *   0.999, eps 1e-8, bias-corrected with step t >= 1, learning rate lr; lr =
 *   0 leaves params unchanged) of params, adam_m and adam_v in place.
 *   label: n floats in {0, 1}; target: n x 2 (ty, tx).
 * sfoc_head_infer: forward, then on every CP with an interior peak:
 *   sigmoid(logit) >= threshold sets VALID (else INCONSISTENT), LEARNED is
 *   set, sub_dy / sub_dx become oy / ox clipped to [-1.5, 1.5]; other CPs
 *   are left as they are.  out (n x 3) may be NULL.
 * All device pointers; ws of sfoc_head_workspace(n, train) bytes.
 * Every reduction runs in a fixed order: results are bit-reproducible.
 * Limits: 1 <= n <= 65536 per call (SFOC_E_UNSUPPORTED beyond).
 * Errors: SFOC_E_INVALID_ARG (null pointers, n < 0, t < 1), SFOC_E_WORKSPACE,
 * SFOC_E_HIP.  n == 0 is valid and enqueues nothing.
 */
#define SFOC_HEAD_PARAMS  54051
#define SFOC_HEAD_CROP    33
#define SFOC_HEAD_NSTAT   8
int sfoc_head_features(const void* desc_sen, int64_t Hs, int64_t Ws,
                       const double* integ1, const double* integ2, int64_t Hr, int64_t Wr,
                       int32_t z, int32_t dtype,
                       const int32_t* ips, const int32_t* prior, int32_t n, int32_t m, int32_t r,
                       const float* ncc, const sfoc_cp* cps,
                       float* crops, float* stats, void* stream);
int sfoc_head_workspace(int32_t n, int32_t train, size_t* bytes);
int sfoc_head_forward(const float* params, const float* crops, const float* stats, int32_t n,
                      float* out, void* ws, size_t ws_bytes, void* stream);
int sfoc_head_train_step(float* params, float* adam_m, float* adam_v, int32_t t, float lr,
                         const float* crops, const float* stats, const float* label,
                         const float* target, int32_t n, float* grad, float* loss,
                         void* ws, size_t ws_bytes, void* stream);
int sfoc_head_infer(const float* params, const float* crops, const float* stats, int32_t n,
                    float threshold, sfoc_cp* cps, float* out, void* ws, size_t ws_bytes,
                    void* stream);

/*
 * RANSAC outlier rejection over the CPs of one pair (Section 3.2.3: after
 * matching, random sample consensus removes the mismatched CPs, under a
 * projective model in general and an affine compensation model in the
 * RPC-based variant, which needs RPC metadata and is not provided here).
 * A drop-in alternative to the median-displacement consistency check for
 * pairs related by more than a translation.
 *
 * Candidates are the CPs with an interior peak (none of OOB, FLAT_T,
 * FLAT_S, EDGE_PEAK, NONFINITE), in CP order; each maps the sensed point
 * (sen_row, sen_col) to the reference point of sfoc_cp's definition.  Both
 * point sets are normalised per image, v_n = (v - (size-1)/2) / (max(H,W)/2),
 * and every step runs in float64:
 *  - hypothesis h draws its k sample indices (k = 3 affine, 4 projective)
 *    from words[h*k .. h*k+k-1]: index = floor(word * n_cand / 2^32).  The
 *    words are the caller's uniform 32-bit random numbers; the library
 *    draws none.  A sample with a repeated index, or three points whose
 *    cross product is <= 1e-9 (normalised units) in either image, is
 *    degenerate (count -1);
 *  - the minimal model is the unique affine map through 3 correspondences,
 *    or the unique homography (h22 = 1) through 4;
 *  - a candidate is an inlier when its reprojection distance is <=
 *    threshold reference pixels (a projective denominator <= 0 is an
 *    outlier); counts[h] is the number of inliers;
 *  - the best hypothesis has the most inliers (lowest index on ties); then
 *    n_refine times: least squares over the current inliers (for the
 *    projective model the linear one with h22 = 1) and a new inlier set.
 *    Fewer than k inliers, or a normal matrix whose squared Cholesky pivot
 *    falls to 1e-12 of its largest diagonal entry, stops the refinement
 *    with the current model.
 * Result: the VALID / INCONSISTENT bits of every candidate are cleared and
 * VALID (inlier) or INCONSISTENT (outlier) set; other CPs are unchanged.
 * With fewer than k candidates or no non-degenerate hypothesis, every
 * candidate is INCONSISTENT and info[3] = 1.
 *  cps        n records, updated in place.                    (in/out)
 *  prior      n x 2 int32 or NULL, as given to the matching.
 *  words      n_hyp * k uint32.
 *  model      9 float64: the model in pixels, row-major 3x3, mapping the
 *             sensed (row, col, 1) to the reference, entry (2,2) = 1
 *             (zeros without a model).                          (output)
 *  info       4 int32: candidates, final inliers, best hypothesis (-1
 *             without a model), status (0 model, 1 none).       (output)
 *  counts     n_hyp int32 inlier counts, or NULL.               (output)
 *  hyp_models n_hyp x 9 float64 minimal models in normalised
 *             coordinates (written for non-degenerate hypotheses), or NULL.
 * All device pointers; ws of sfoc_ransac_workspace bytes.  The result is
 * bit-reproducible (fixed-order reductions).
 * Limits: n <= 2^22, n_hyp <= 2^20 (SFOC_E_UNSUPPORTED beyond).
 * Errors: SFOC_E_INVALID_ARG (null pointers, n < 0, unknown model, n_hyp <
 * 1, n_refine outside 0..16, threshold <= 0, sizes < 1), SFOC_E_WORKSPACE,
 * SFOC_E_HIP.  n == 0 is valid (no model, info = {0, 0, -1, 1}).
 */
#define SFOC_MODEL_AFFINE      6
#define SFOC_MODEL_PROJECTIVE  8
typedef struct sfoc_ransac_params {
    int32_t model;       /* SFOC_MODEL_* */
    int32_t n_hyp;       /* hypotheses */
    int32_t n_refine;    /* least-squares refits, 0..16 */
    int32_t reserved;
    double  threshold;   /* inlier distance, reference pixels (1.5) */
    int32_t Hs, Ws;      /* sensed image size (normalisation) */
    int32_t Hr, Wr;      /* reference image size */
} sfoc_ransac_params;
int sfoc_ransac_workspace(int32_t n, const sfoc_ransac_params* p, size_t* bytes);
int sfoc_ransac_cps(sfoc_cp* cps, const int32_t* prior, int32_t n, const uint32_t* words,
                    const sfoc_ransac_params* p, void* ws, size_t ws_bytes, double* model,
                    int32_t* info, int32_t* counts, double* hyp_models, void* stream);

/*
 * Rectification (Section 3.2.3: after outlier removal the sensed image is
 * resampled into the reference image's coordinate system by bilinear
 * interpolation).  model is the sensed -> reference map of
 * sfoc_ransac_cps (9 float64, device memory, row-major 3x3 on (row, col,
 * 1)); output pixel (r, c) of the Ho x Wo reference grid takes the sensed
 * image at p = model^-1 (r, c, 1) (inverse in float64, dehomogenised):
 * bilinear between the four pixels around p when p lies in [0, Hs-1] x
 * [0, Ws-1] (a neighbour past the last row or column only ever has weight
 * 0), else fill; a point whose homogeneous coordinate is <= 0, or a
 * singular model, also gives fill.  Coordinates in float64, the
 * interpolation in float32.
 *  sen   Hs x Ws float32, pitch lds (elements).             (input)
 *  out   Ho x Wo float32, pitch ldo.                        (output)
 * Limits: every side <= 2^20 and Hs * lds < 2^31.  Errors:
 * SFOC_E_INVALID_ARG (null pointers,
 * sizes < 1, pitches below the widths), SFOC_E_UNSUPPORTED, SFOC_E_HIP.
 */
int sfoc_rectify(const float* sen, int64_t Hs, int64_t Ws, int64_t lds, const double* model,
                 float* out, int64_t Ho, int64_t Wo, int64_t ldo, float fill, void* stream);

/*
 * Block-based FAST interest-point detection (Section 3.1.1: the FAST
 * operator applied with a partitioning strategy, so that the interest
 * points are spread evenly over the image).
 *  - Corner strength V(p), float32: the largest threshold at which 9
 *    cyclically contiguous pixels of the 16-pixel circle of radius 3 are all
 *    brighter than I_p + threshold or all darker than I_p - threshold, i.e.
 *    the maximum over the 16 arcs of max(min (I_x - I_p), min (I_p - I_x));
 *    p is a corner when V(p) > threshold.
 *  - Only pixels at least b = max(3, margin) from every border are
 *    considered (the region); a corner is kept when its V exceeds that of
 *    every 3 x 3 neighbour in the region before it in raster order and is
 *    not below that of every neighbour after it.
 *  - The region is split into nby x nbx blocks at rows
 *    b + floor(i * (H - 2b) / nby) (columns likewise); from each block the
 *    per_block kept corners of largest V, ties to the smaller raster index.
 *  img      H x W float32, pitch ld, finite values.               (input)
 *  ips      (row, col) int32 pairs, capacity nby * nbx * per_block; the
 *           first *n_out are written, in block order (row-major), within
 *           a block by decreasing V.                               (output)
 *  scores   their V (float32), same capacity, or NULL.            (output)
 *  counts   nby * nbx int32 per-block counts, or NULL.            (output)
 *  n_out    one int32: the number of interest points.             (output)
 * All device pointers; ws of sfoc_fast_workspace bytes (the strength map).
 * The result is exact and deterministic (no floating-point sums).
 * Limits: sides <= 2^20, H * W <= 2^32, per_block <= 32, nby * nbx <=
 * 65536 (SFOC_E_UNSUPPORTED beyond).  Errors: SFOC_E_INVALID_ARG (null
 * img / ips / n_out / ws, sizes < 1, ld < W, margin < 0, threshold < 0 or
 * not finite), SFOC_E_WORKSPACE, SFOC_E_HIP.
 */
int sfoc_fast_workspace(int64_t H, int64_t W, int32_t nby, int32_t nbx, int32_t per_block, size_t* bytes);
int sfoc_detect_ips(const float* img, int64_t H, int64_t W, int64_t ld, float threshold, int32_t margin,
                    int32_t nby, int32_t nbx, int32_t per_block, int32_t* ips, float* scores,
                    int32_t* counts, int32_t* n_out, void* ws, size_t ws_bytes, void* stream);

/*
 * Kernel timing (tracing).  While enabled, the library records a pair of
 * HIP events on the launch stream around every kernel it enqueues.
 * sfoc_trace_collect waits for those events, writes per-kernel totals into
 * ms[k] (milliseconds) and counts[k] for k in [0, n) with the kernel ids
 * below, clears the record, and returns the number of kernel ids written.
 * At most SFOC_TRACE_MAX launches are recorded between two collections;
 * later ones are not timed.  Not thread-safe; host only.
 */
#define SFOC_K_DESCRIBE     0
#define SFOC_K_INTEGRAL     1
#define SFOC_K_MATCH        2
#define SFOC_K_CONSISTENCY  3
#define SFOC_K_PEAK         4
#define SFOC_K_HEAD_FEAT    5
#define SFOC_K_HEAD_FWD     6
#define SFOC_K_HEAD_BWD     7
#define SFOC_K_HEAD_ADAM    8
#define SFOC_K_RANSAC       9
#define SFOC_K_RECTIFY     10
#define SFOC_K_FAST        11
#define SFOC_K_COUNT       12
#define SFOC_TRACE_MAX   4096
int sfoc_trace_enable(int on);
int sfoc_trace_collect(double* ms, int64_t* counts, int n);

#ifdef __cplusplus
}
#endif
#endif /* SFOC_H */
