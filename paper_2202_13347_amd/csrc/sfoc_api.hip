// extern "C" entry points: argument checks on the host, then launches on
// the caller's stream.  Nothing here allocates device memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "sfoc_launch.h"

namespace sfoc {

static thread_local hipError_t g_last_hip = hipSuccess;

int hip_status(hipError_t e) {
    if (e == hipSuccess) return SFOC_OK;
    g_last_hip = e;
    return SFOC_E_HIP;
}

hipError_t ensure_dynamic_lds(const void* kern, int bytes) {
    static std::mutex mu;
    static std::map<std::pair<const void*, int>, int> done;   // (kernel, device) -> bytes allowed
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(mu);
    auto it = done.find({kern, dev});
    if (it != done.end() && it->second >= bytes) return hipSuccess;
    e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess) done[{kern, dev}] = bytes;
    return e;
}

// A second stream (and a fork / join event pair) per device and host
// thread, for work that overlaps the caller's stream inside one call.  Kept
// for the life of the process; default priority, non-blocking.
struct SideStream {
    hipStream_t s = nullptr;
    hipEvent_t start = nullptr, join = nullptr;
};

static hipError_t side_stream(SideStream** out) {
    thread_local std::map<int, SideStream> per_device;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    SideStream& ss = per_device[dev];
    if (!ss.s) {
        SideStream t;
        e = hipStreamCreateWithFlags(&t.s, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&t.start, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&t.join, hipEventDisableTiming);
        if (e != hipSuccess) return e;
        ss = t;
    }
    *out = &ss;
    return hipSuccess;
}

struct RegisterLayout {
    size_t desc_ref, desc_sen, integ1, integ2, scan, jobs, tiles, rmask, split, match, total;
};

static RegisterLayout register_layout(int64_t Hr, int64_t Wr, int64_t Hs, int64_t Ws, int32_t n, int32_t m,
                                      int32_t r, int32_t z, size_t es, size_t match_ws) {
    RegisterLayout L;
    size_t off = 0;
    L.desc_ref = off;
    off = align_up(off + (size_t)z * Hr * Wr * es, 256);
    L.desc_sen = off;
    off = align_up(off + (size_t)z * Hs * Ws * es, 256);
    L.integ1 = off;
    off = align_up(off + (size_t)(Hr + 1) * (Wr + 1) * sizeof(double), 256);
    L.integ2 = off;
    off = align_up(off + (size_t)(Hr + 1) * (Wr + 1) * sizeof(double), 256);
    L.scan = off;
    off = align_up(off + describe_ws_bytes(Hr, Wr), 256);
    L.jobs = off;
    off = align_up(off + 2 * sizeof(DescribeJob), 256);
    L.tiles = off;
    off = align_up(off + (size_t)pair_table_entries((int)Hr, (int)Wr, n, m) * 16, 256);
    L.rmask = off;
    off = align_up(off + tile_mask_bytes(Hr, Wr), 256);
    L.split = off;
    off = align_up(off + match_split_bytes(n, r), 256);
    L.match = off;
    off = align_up(off + match_ws, 256);
    L.total = off;
    return L;
}

// The pair call's launches for sizes already checked and a workspace laid
// out by register_layout (consistency = false leaves out the median check).
static hipError_t register_core(const float* ref, int64_t Hr, int64_t Wr, int64_t ldr, const float* sen, int64_t Hs,
                                int64_t Ws, int64_t lds, const int32_t* ips, const int32_t* prior, int32_t n,
                                int32_t m, int32_t r, const DescribeConsts& c, int32_t z, int32_t dtype, float* ncc,
                                sfoc_cp* cps, const RegisterLayout& L, void* ws, hipStream_t st, bool consistency) {
    char* base = (char*)ws;
    void* dref = base + L.desc_ref;
    void* dsen = base + L.desc_sen;
    double* i1 = (double*)(base + L.integ1);
    double* i2 = (double*)(base + L.integ2);
    // Of the reference image only the tiles the search windows read are
    // described (the others get zero integral-image aggregates), and of the
    // sensed image only the tiles under the templates of in-bounds IPs, one
    // table entry per template tile.  Both images go into one describe
    // launch, so that they share the GPU to the end of the launch.  The
    // match's transforms do not read the integral images: where the match
    // splits (an FFT side without offset blocks), the integral scans run on
    // a second stream beside the transforms, and the NCC and peaks follow
    // once both are done.  Otherwise the scans precede the match.
    double* agg = (double*)(base + L.scan);
    DescribeJob* jobs = (DescribeJob*)(base + L.jobs);
    int4* tiles = (int4*)(base + L.tiles);
    uint8_t* rmask = (uint8_t*)(base + L.rmask);
    hipError_t e = launch_describe_pair(ref, (int)Hr, (int)Wr, ldr, dref, i1, i2, agg, sen, (int)Hs, (int)Ws, lds, dsen,
                                        ips, prior, n, m, r, jobs, tiles, rmask, c, st);
    if (e != hipSuccess) return e;
    if (!match_split_ok(n, m, r, dtype)) {
        e = launch_integral(i1, i2, (int)Hr, (int)Wr, agg, st, rmask);
        if (e != hipSuccess || n == 0) return e;
        return launch_match(dsen, Hs, Ws, dref, Hr, Wr, i1, i2, z, dtype, ips, prior, n, m, r, ncc, cps,
                            base + L.match, st, consistency);
    }
    SideStream* side = nullptr;
    void* split = base + L.split;
    e = side_stream(&side);
    if (e == hipSuccess) e = hipEventRecord(side->start, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(side->s, side->start, 0);
    if (e == hipSuccess) e = launch_integral(i1, i2, (int)Hr, (int)Wr, agg, side->s, rmask);
    if (e == hipSuccess) e = hipEventRecord(side->join, side->s);
    if (e == hipSuccess)
        e = launch_match_fft(dsen, Hs, Ws, dref, Hr, Wr, z, dtype, ips, prior, n, m, r, ncc, cps, base + L.match,
                             split, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, side->join, 0);
    if (e != hipSuccess) return e;
    return launch_match_finish(dsen, Hs, Ws, dref, Hr, Wr, i1, i2, z, dtype, ips, prior, n, m, r, ncc, cps,
                               base + L.match, split, st, consistency);
}

// ---- band-streamed registration ---------------------------------------------
// IPs sorted by row are taken in bands: a band starts at the next IP's row y0
// and holds the IPs with row < y0 + band_rows.  Its sub-images are the rows
// its templates and search windows read, widened by the filter reach Q + R
// (so every row read has the descriptors of the whole image) and clipped to
// the images; IP rows and priors are taken relative to them.
struct Band {
    int i0, i1;       // IPs [i0, i1)
    int64_t s0, s1;   // sensed rows [s0, s1)
    int64_t r0, r1;   // reference rows [r0, r1)
};

static void clip_rows(int64_t lo, int64_t hi, int64_t H, int64_t* a, int64_t* b) {
    *a = std::min(std::max(lo, (int64_t)0), H);
    *b = std::min(std::max(hi, (int64_t)0), H);
    if (*b <= *a) {   // nothing of the image is read (every IP of the band is out of bounds): any one row
        *a = std::min(*a, H - 1);
        *b = *a + 1;
    }
}

static void plan_bands(const int32_t* ips, const int32_t* prior, int32_t n, int32_t m, int32_t r, int64_t Hs,
                       int64_t Hr, int32_t band_rows, int halo, std::vector<Band>& out) {
    out.clear();
    const int64_t M = (int64_t)m + 2 * r;
    for (int i0 = 0; i0 < n;) {
        const int64_t y0 = ips[2 * i0];
        int64_t smin = INT64_MAX, smax = INT64_MIN, rmin = INT64_MAX, rmax = INT64_MIN;
        int i1 = i0;
        for (; i1 < n && (int64_t)ips[2 * i1] < y0 + band_rows; ++i1) {
            const int64_t ty = (int64_t)ips[2 * i1] - m / 2;
            const int64_t sy = ty - r + (prior ? prior[2 * i1] : 0);
            smin = std::min(smin, ty);
            smax = std::max(smax, ty + m);
            rmin = std::min(rmin, sy);
            rmax = std::max(rmax, sy + M);
        }
        Band b;
        b.i0 = i0;
        b.i1 = i1;
        clip_rows(smin - halo, smax + halo, Hs, &b.s0, &b.s1);
        clip_rows(rmin - halo, rmax + halo, Hr, &b.r0, &b.r1);
        out.push_back(b);
        i0 = i1;
    }
}

// Largest band sub-images for band_rows and priors with |dy| <= max_prior.
static void band_bounds(int64_t Hr, int64_t Hs, int32_t m, int32_t r, int32_t band_rows, int32_t max_prior, int halo,
                        int64_t* hs, int64_t* hr) {
    *hs = std::min<int64_t>(Hs, (int64_t)band_rows - 1 + m + 2 * halo);
    *hr = std::min<int64_t>(Hr, (int64_t)band_rows - 1 + 2 * (int64_t)max_prior + m + 2 * r + 2 * halo);
}

struct StreamLayout {
    RegisterLayout band;   // one band's register workspace
    size_t ips, prior, total;
};

static StreamLayout stream_layout(int64_t Hr, int64_t Wr, int64_t Hs, int64_t Ws, int32_t n, int32_t m, int32_t r,
                                  int32_t band_rows, int32_t max_prior, int32_t z, size_t es, int halo) {
    StreamLayout S;
    int64_t hs = 0, hr = 0;
    band_bounds(Hr, Hs, m, r, band_rows, max_prior, halo, &hs, &hr);
    S.band = register_layout(hr, Wr, hs, Ws, n, m, r, z, es, match_plan(n, m, r).ws_bytes);
    S.ips = S.band.total;
    S.prior = align_up(S.ips + (size_t)n * 2 * sizeof(int32_t), 256);
    S.total = align_up(S.prior + (size_t)n * 2 * sizeof(int32_t), 256);
    return S;
}

}  // namespace sfoc

using namespace sfoc;

extern "C" {

const char* sfoc_status_string(int status) {
    switch (status) {
        case SFOC_OK: return "SFOC_OK";
        case SFOC_E_INVALID_ARG: return "SFOC_E_INVALID_ARG: invalid argument";
        case SFOC_E_UNSUPPORTED: return "SFOC_E_UNSUPPORTED: outside the supported sizes or parameters";
        case SFOC_E_WORKSPACE: return "SFOC_E_WORKSPACE: workspace too small";
        case SFOC_E_HIP: return g_last_hip == hipSuccess ? "SFOC_E_HIP" : hipGetErrorString(g_last_hip);
        default: return "unknown status";
    }
}

int sfoc_params_preset(int32_t which, sfoc_params* p) {
    if (!p || (which != 0 && which != 1)) return SFOC_E_INVALID_ARG;
    sfoc_params q = {};
    q.trunc = 3.0;
    q.K = 1;
    q.n_dil = 3;
    q.dil[0] = 1;
    q.dil[1] = 2;
    q.dil[2] = 3;
    q.sd1 = 1.0;
    q.sd2 = 1.5;
    q.eps = 1e-8;
    q.rectify = SFOC_RECTIFY_ABS;
    q.second_order = 1;
    q.desc_dtype = SFOC_DTYPE_F32;
    if (which == 0) {
        q.n_orient = 6;
        q.n_s1 = 3;
        q.s1[0] = 0.6;
        q.s1[1] = 0.8;
        q.s1[2] = 1.0;
        q.n_s2 = 1;
        q.s2[0] = 1.5;
    } else {
        q.n_orient = 8;
        q.n_s1 = 3;
        q.n_s2 = 3;
        for (int i = 0; i < 3; ++i) q.s1[i] = q.s2[i] = (double)(i + 1);
    }
    *p = q;
    return SFOC_OK;
}

int sfoc_params_check(const sfoc_params* p, int32_t* z) { return check_params(p, z); }

int sfoc_describe_workspace(int64_t H, int64_t W, const sfoc_params* p, size_t* bytes) {
    if (!bytes || H < 1 || W < 1) return SFOC_E_INVALID_ARG;
    int rc = check_params(p, nullptr);
    if (rc) return rc;
    *bytes = describe_ws_bytes(H, W);
    return SFOC_OK;
}

int sfoc_describe(const float* img, int64_t H, int64_t W, int64_t ld, const sfoc_params* p, void* desc,
                  double* integ1, double* integ2, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_image(img, H, W, ld);
    if (rc) return rc;
    if (!desc || ((integ1 == nullptr) != (integ2 == nullptr))) return SFOC_E_INVALID_ARG;
    rc = check_params(p, nullptr);
    if (rc) return rc;
    if (integ1 && (!ws || ws_bytes < describe_ws_bytes(H, W))) return SFOC_E_WORKSPACE;
    DescribeConsts c;
    build_describe_consts(p, &c);
    hipStream_t st = (hipStream_t)stream;
    double* agg = integ1 ? (double*)ws : nullptr;
    hipError_t e = launch_describe(img, (int)H, (int)W, ld, desc, integ1, integ2, agg, c, st);
    if (e != hipSuccess) return hip_status(e);
    if (integ1) {
        e = launch_integral(integ1, integ2, (int)H, (int)W, agg, st);
        if (e != hipSuccess) return hip_status(e);
    }
    return SFOC_OK;
}

int sfoc_match_workspace(int32_t n, int32_t m, int32_t r, int32_t z, size_t* bytes) {
    if (!bytes || z < 1) return SFOC_E_INVALID_ARG;
    int rc = check_match_shape(n, m, r);
    if (rc) return rc;
    *bytes = match_plan(n, m, r).ws_bytes;
    return SFOC_OK;
}

int sfoc_match_window_workspace(int32_t n, int32_t m, int32_t r, int32_t z, size_t* bytes) {
    if (!bytes || z < 1) return SFOC_E_INVALID_ARG;
    int rc = check_match_shape(n, m, r);
    if (rc) return rc;
    *bytes = match_plan(n, m, r).ws_bytes + match_window_ws_bytes(n, m, r);
    return SFOC_OK;
}

int sfoc_fastncc_match(const void* desc_sen, int64_t Hs, int64_t Ws, const void* desc_ref, int64_t Hr, int64_t Wr,
                       const double* integ1, const double* integ2, int32_t z, int32_t dtype, const int32_t* ips,
                       const int32_t* prior, int32_t n, int32_t m, int32_t r, float* ncc, sfoc_cp* cps, void* ws,
                       size_t ws_bytes, void* stream) {
    int rc = check_match_shape(n, m, r);
    if (rc) return rc;
    if (z < 1 || dtype_size(dtype) == 0) return SFOC_E_INVALID_ARG;
    if (Hs < 1 || Ws < 1 || Hr < 1 || Wr < 1) return SFOC_E_INVALID_ARG;
    if (Hs > kMaxSide || Ws > kMaxSide || Hr > kMaxSide || Wr > kMaxSide) return SFOC_E_UNSUPPORTED;
    if (Hs * Ws >= kMaxPlane || Hr * Wr >= kMaxPlane) return SFOC_E_UNSUPPORTED;
    if (n == 0) return SFOC_OK;
    if (!desc_sen || !desc_ref || !ips || !cps || ((integ1 == nullptr) != (integ2 == nullptr)))
        return SFOC_E_INVALID_ARG;
    const size_t need = match_plan(n, m, r).ws_bytes + (integ1 ? 0 : match_window_ws_bytes(n, m, r));
    if (need > 0 && (!ws || ws_bytes < need)) return SFOC_E_WORKSPACE;
    hipError_t e = launch_match(desc_sen, Hs, Ws, desc_ref, Hr, Wr, integ1, integ2, z, dtype, ips, prior, n, m, r,
                                ncc, cps, ws, (hipStream_t)stream);
    return hip_status(e);
}

int sfoc_register_workspace(int64_t Hr, int64_t Wr, int64_t Hs, int64_t Ws, int32_t n, int32_t m, int32_t r,
                            const sfoc_params* p, size_t* bytes) {
    if (!bytes || Hr < 1 || Wr < 1 || Hs < 1 || Ws < 1) return SFOC_E_INVALID_ARG;
    int32_t z = 0;
    int rc = check_params(p, &z);
    if (rc) return rc;
    rc = check_match_shape(n, m, r);
    if (rc) return rc;
    *bytes = register_layout(Hr, Wr, Hs, Ws, n, m, r, z, dtype_size(p->desc_dtype), match_plan(n, m, r).ws_bytes).total;
    return SFOC_OK;
}

int sfoc_register_cps(const float* ref, int64_t Hr, int64_t Wr, int64_t ldr, const float* sen, int64_t Hs,
                      int64_t Ws, int64_t lds, const int32_t* ips, const int32_t* prior, int32_t n, int32_t m,
                      int32_t r, const sfoc_params* p, float* ncc, sfoc_cp* cps, void* ws, size_t ws_bytes,
                      void* stream) {
    int rc = check_image(ref, Hr, Wr, ldr);
    if (rc) return rc;
    rc = check_image(sen, Hs, Ws, lds);
    if (rc) return rc;
    int32_t z = 0;
    rc = check_params(p, &z);
    if (rc) return rc;
    rc = check_match_shape(n, m, r);
    if (rc) return rc;
    if (Hs * Ws >= kMaxPlane || Hr * Wr >= kMaxPlane) return SFOC_E_UNSUPPORTED;
    if (n > 0 && (!ips || !cps)) return SFOC_E_INVALID_ARG;
    const int64_t ntiles = (int64_t)n * template_tile_slots(m, kDescribeTile);
    if (ntiles > INT32_MAX) return SFOC_E_UNSUPPORTED;
    const RegisterLayout L =
        register_layout(Hr, Wr, Hs, Ws, n, m, r, z, dtype_size(p->desc_dtype), match_plan(n, m, r).ws_bytes);
    if (!ws || ws_bytes < L.total) return SFOC_E_WORKSPACE;
    DescribeConsts c;
    build_describe_consts(p, &c);
    return hip_status(register_core(ref, Hr, Wr, ldr, sen, Hs, Ws, lds, ips, prior, n, m, r, c, z, p->desc_dtype, ncc,
                                    cps, L, ws, (hipStream_t)stream, true));
}

int sfoc_register_streamed_workspace(int64_t Hr, int64_t Wr, int64_t Hs, int64_t Ws, int32_t n, int32_t m,
                                     int32_t r, int32_t band_rows, int32_t max_prior, const sfoc_params* p,
                                     size_t* bytes) {
    if (!bytes || Hr < 1 || Wr < 1 || Hs < 1 || Ws < 1 || band_rows < 1 || max_prior < 0) return SFOC_E_INVALID_ARG;
    int32_t z = 0;
    int rc = check_params(p, &z);
    if (rc) return rc;
    rc = check_match_shape(n, m, r);
    if (rc) return rc;
    DescribeConsts c;
    build_describe_consts(p, &c);
    *bytes = stream_layout(Hr, Wr, Hs, Ws, n, m, r, band_rows, max_prior, z, dtype_size(p->desc_dtype), c.Q + c.R)
                 .total;
    return SFOC_OK;
}

int sfoc_register_cps_streamed(const float* ref, int64_t Hr, int64_t Wr, int64_t ldr, const float* sen, int64_t Hs,
                               int64_t Ws, int64_t lds, const int32_t* ips, const int32_t* prior, int32_t n,
                               int32_t m, int32_t r, int32_t band_rows, int32_t max_prior, const sfoc_params* p,
                               float* ncc, sfoc_cp* cps, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_image(ref, Hr, Wr, ldr);
    if (rc) return rc;
    rc = check_image(sen, Hs, Ws, lds);
    if (rc) return rc;
    int32_t z = 0;
    rc = check_params(p, &z);
    if (rc) return rc;
    rc = check_match_shape(n, m, r);
    if (rc) return rc;
    if (band_rows < 1 || max_prior < 0) return SFOC_E_INVALID_ARG;
    if (Hs * Ws >= kMaxPlane || Hr * Wr >= kMaxPlane) return SFOC_E_UNSUPPORTED;
    if (n > 0 && (!ips || !cps)) return SFOC_E_INVALID_ARG;
    if ((int64_t)n * template_tile_slots(m, kDescribeTile) > INT32_MAX) return SFOC_E_UNSUPPORTED;
    DescribeConsts c;
    build_describe_consts(p, &c);
    const int halo = c.Q + c.R;
    const StreamLayout S =
        stream_layout(Hr, Wr, Hs, Ws, n, m, r, band_rows, max_prior, z, dtype_size(p->desc_dtype), halo);
    if (!ws || ws_bytes < S.total) return SFOC_E_WORKSPACE;
    if (n == 0) return SFOC_OK;
    hipStream_t st = (hipStream_t)stream;
    // the IPs (and priors) on the host: bands, sorted-order and prior checks
    std::vector<int32_t> h_ips((size_t)n * 2), h_prior(prior ? (size_t)n * 2 : 0);
    hipError_t e = hipMemcpyAsync(h_ips.data(), ips, (size_t)n * 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && prior)
        e = hipMemcpyAsync(h_prior.data(), prior, (size_t)n * 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_status(e);
    for (int32_t i = 0; i < n; ++i) {
        if (i > 0 && h_ips[2 * i] < h_ips[2 * i - 2]) return SFOC_E_INVALID_ARG;   // not sorted by row
        if (prior && std::abs((int64_t)h_prior[2 * i]) > max_prior) return SFOC_E_INVALID_ARG;
    }
    std::vector<Band> bands;
    plan_bands(h_ips.data(), prior ? h_prior.data() : nullptr, n, m, r, Hs, Hr, band_rows, halo, bands);
    // band-relative IP rows and row priors; far-outside values are clamped
    // (such IPs are out of bounds either way)
    const int64_t kFar = (int64_t)1 << 30;
    std::vector<int32_t> b_ips((size_t)n * 2), b_prior((size_t)n * 2);
    for (const Band& b : bands)
        for (int i = b.i0; i < b.i1; ++i) {
            const int64_t y = (int64_t)h_ips[2 * i] - b.s0;
            const int64_t py = (prior ? (int64_t)h_prior[2 * i] : 0) + b.s0 - b.r0;
            b_ips[2 * i] = (int32_t)std::min(std::max(y, -kFar), kFar);
            b_ips[2 * i + 1] = h_ips[2 * i + 1];
            b_prior[2 * i] = (int32_t)std::min(std::max(py, -kFar), kFar);
            b_prior[2 * i + 1] = prior ? h_prior[2 * i + 1] : 0;
        }
    char* base = (char*)ws;
    int32_t* d_ips = (int32_t*)(base + S.ips);
    int32_t* d_prior = (int32_t*)(base + S.prior);
    e = hipMemcpyAsync(d_ips, b_ips.data(), b_ips.size() * sizeof(int32_t), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_prior, b_prior.data(), b_prior.size() * sizeof(int32_t), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);   // the host arrays go out of scope before the bands finish
    const int64_t V = 2 * (int64_t)r + 1;
    for (size_t k = 0; k < bands.size() && e == hipSuccess; ++k) {
        const Band& b = bands[k];
        const int nb = b.i1 - b.i0;
        e = register_core(ref + b.r0 * ldr, b.r1 - b.r0, Wr, ldr, sen + b.s0 * lds, b.s1 - b.s0, Ws, lds,
                          d_ips + 2 * b.i0, d_prior + 2 * b.i0, nb, m, r, c, z, p->desc_dtype,
                          ncc ? ncc + b.i0 * V * V : nullptr, cps + b.i0, S.band, ws, st, false);
        if (e == hipSuccess) e = launch_cp_row_shift(cps + b.i0, nb, (int)b.s0, st);
    }
    if (e == hipSuccess) e = launch_consistency(cps, prior, n, st);
    return hip_status(e);
}

int sfoc_match_candidates(int32_t m, int32_t r, int32_t* fft_side, int32_t* blocks, int32_t cap) {
    if (cap < 0 || (cap > 0 && !fft_side)) return SFOC_E_INVALID_ARG;
    int Ls[kNumSides];
    const int n = match_candidates(m, r, Ls);
    for (int k = 0; k < n && k < cap; ++k) {
        fft_side[k] = Ls[k];
        if (blocks) blocks[k] = match_plan_L(1, m, r, Ls[k]).nb;
    }
    return n;
}

int64_t sfoc_sensed_tiles(const int32_t* ips, const int32_t* prior, int32_t n, int32_t m, int32_t r, int64_t Hs,
                          int64_t Ws, int64_t Hr, int64_t Wr, int32_t cover, int32_t* origins, int64_t cap) {
    if (n < 0 || m < 3 || r < 1 || Hs < 1 || Ws < 1 || Hr < 1 || Wr < 1 || cap < 0 || (cap > 0 && !origins) ||
        (n > 0 && !ips) || cover < kCoverTemplate || cover > kCoverSmaller)
        return SFOC_E_INVALID_ARG;
    if (Hs > kMaxSide || Ws > kMaxSide) return SFOC_E_UNSUPPORTED;
    std::vector<std::pair<int, int>> t;
    sensed_tiles(ips, prior, n, m, r, Hs, Ws, Hr, Wr, kDescribeTile, cover, t);
    for (size_t k = 0; k < t.size() && (int64_t)k < cap; ++k) {
        origins[2 * k] = t[k].first;
        origins[2 * k + 1] = t[k].second;
    }
    return (int64_t)t.size();
}

}  // extern "C"
