// Dense SFOC descriptor (Section 2.1, Eq. 1-7) as one fused gfx950 kernel
// per 32x32 output tile, plus the float64 integral-image scans (Eq. 14-16).
//
// Per tile, everything stays in LDS:
//   1. the input tile plus a halo of R (largest kernel radius) + Q (dilated
//      smoothing reach), read once from HBM with reflect-101 indices;
//   2. for each distinct sigma, a separable row pass (1-D Gaussian g, first
//      derivative d, second derivative dd) and a column pass that adds the
//      five basis responses Gx, Gy, Gxx, Gyy, Gxy * I into per-pixel sums
//      over sigma (sum over scales commutes with steering: both linear);
//   3. per group of channels: steer (Eq. 4/6 and the directional reading of
//      Eq. 7), rectify, write to LDS, then the dilated Gaussian smoothing
//      (rates dil[], summed) into registers;
//   4. per-order L2 normalisation, rounding to the storage type, one
//      coalesced store per channel plane, and the per-pixel channel sums
//      sum_c g and sum_c g^2 (float64, from the stored values) for the
//      integral images.
#include "sfoc_dev.h"
#include "sfoc_launch.h"
#include "sfoc_trace.h"

namespace sfoc {

constexpr int kTS = kDescribeTile;   // output tile side
constexpr int kNT = 256;      // threads per tile
constexpr int kRun = 4;       // outputs per thread along a run
constexpr int kPXT = kTS * kTS / kNT;   // output pixels per thread (one run of 4)
static_assert(kPXT == kRun, "one horizontal run of outputs per thread");

// LDS geometry of one tile.  Every side is padded to a multiple of kRun so
// runs never straddle a row; padded rows and columns hold harmless values
// that no output reads.
struct DescribeGeom {
    int BSP;    // basis / channel side incl. the smoothing halo Q, padded
    int ISX;    // image-region side (BSP + 2R)
    int nrun;   // runs per basis row (BSP / kRun)
    int BPP;    // LDS row pitch of the basis / channel / row-pass maps (odd)
    int IPP;    // LDS row pitch of the image region (odd)
    size_t bytes;
};

// Pitch of the half-width row-pass maps of the four-workgroup configuration
// (20 columns, odd).
constexpr int kHalfPitch = 21;

static DescribeGeom describe_geom(const DescribeConsts& c, int CG, bool halves) {
    DescribeGeom g;
    g.BSP = (kTS + 2 * c.Q + kRun - 1) / kRun * kRun;
    g.ISX = g.BSP + 2 * c.R;
    g.nrun = g.BSP / kRun;
    // Odd pitches spread the rows of a wave's accesses over all LDS banks.
    g.BPP = g.BSP | 1;
    g.IPP = g.ISX | 1;
    // Phase 2 holds the image region and the row-pass maps; phase 3 the five
    // basis maps (over the same memory) and CG steered channels.
    const size_t img = (size_t)g.ISX * g.IPP;
    const size_t row = 3 * (size_t)g.ISX * (halves ? kHalfPitch : g.BPP);
    const size_t bb = (size_t)g.BSP * g.BPP;
    const size_t p2 = img + row, p3 = (5 + (size_t)CG) * bb;
    g.bytes = (p2 > p3 ? p2 : p3) * sizeof(float);
    return g;
}

// Dilated Gaussian smoothing of one channel for a horizontal run of kRun
// outputs, base 3x3 (K = 1) at rates 1, 2, 3.  With weights wc (centre), we
// (edge) and wk (corner) shared by the three rates,
//   out = 3 wc I(p) + we sum_r E_r(p) + wk sum_r C_r(p),
// where E_r / C_r sum the 4 edge / 4 corner neighbours at distance r.  Per
// rate, the vertical pair sums S_r(x) = I(y - r, x) + I(y + r, x) over the
// run's columns widened by r give both: E_r = S_r(x) + I(y, x - r) +
// I(y, x + r) and C_r = S_r(x - r) + S_r(x + r).
// The run's first output is element i0 of map s (pitch P).  Reads are
// addressed from the neighbourhood's top-left element, whose index is kept
// opaque to the compiler: the address then stays in one register and each
// read's constant offset (at most 6 P + kRun + 5 elements) fits the LDS
// instruction's offset field instead of costing an address add.
SFOC_DEV void smooth_run_k1_123(const float* s, int i0, int P, float wc, float we, float wk, float out[kRun]) {
    int b = i0 - 3 * P - 3;
    asm volatile("" : "+v"(b));
    const float* n = s + b;
    float c[kRun + 6];
#pragma unroll
    for (int q = 0; q < kRun + 6; ++q) c[q] = n[3 * P + q];
    float e[kRun], k[kRun];
#pragma unroll
    for (int r = 1; r <= 3; ++r) {
        // one rate's reads in flight at a time keeps registers for the
        // 4 x z accumulators the caller holds
        __builtin_amdgcn_sched_barrier(0);
        float S[kRun + 6];
#pragma unroll
        for (int q = 0; q < kRun + 2 * r; ++q) S[q] = n[(3 - r) * P + 3 - r + q] + n[(3 + r) * P + 3 - r + q];
#pragma unroll
        for (int j = 0; j < kRun; ++j) {
            const float ej = S[j + r] + (c[j + 3 - r] + c[j + 3 + r]);
            const float kj = S[j] + S[j + 2 * r];
            e[j] = r == 1 ? ej : e[j] + ej;
            k[j] = r == 1 ? kj : k[j] + kj;
        }
    }
    const float wc3 = 3.f * wc;
#pragma unroll
    for (int j = 0; j < kRun; ++j) out[j] = fmaf(we, e[j], fmaf(wk, k[j], wc3 * c[j + 3]));
}

// Row pass for a horizontal run of kRun outputs with radius RHO: g, d, dd
// taps paired symmetrically, so odd responses of constant input are exactly
// zero.  p points at the first output's centre.  Correlation form of the
// convolution: out(x) = sum_k t(-k) I(x + k) -> odd taps act on
// I(x - k) - I(x + k).
template <int RHO>
SFOC_DEV void row_run(const float* p, const float* tg, const float* td, const float* tdd, float og[kRun],
                      float od[kRun], float odd[kRun]) {
    float x[2 * RHO + kRun];
#pragma unroll
    for (int q = 0; q < 2 * RHO + kRun; ++q) x[q] = p[q - RHO];
#pragma unroll
    for (int j = 0; j < kRun; ++j) {
        const float c = x[j + RHO];
        float g = tg[0] * c, dd = tdd[0] * c, d = 0.f;
#pragma unroll
        for (int k = 1; k <= RHO; ++k) {
            const float l = x[j + RHO - k], r = x[j + RHO + k];
            const float sm = l + r, df = l - r;
            g = fmaf(tg[k], sm, g);
            dd = fmaf(tdd[k], sm, dd);
            d = fmaf(td[k], df, d);
        }
        og[j] = g;
        od[j] = d;
        odd[j] = dd;
    }
}

// Even (te) and odd (to) column taps on one map for a vertical run; the
// first output's centre is element i0 of map s (pitch P).  The top element's
// index is kept opaque to the compiler, so the reads share one base register
// and fold their row offsets into the LDS instructions where those fit.
template <int RHO>
SFOC_DEV void col_run(const float* s, int i0, int P, const float* te, const float* to, float ev[kRun],
                      float od[kRun]) {
    int b = i0 - RHO * P;
    asm volatile("" : "+v"(b));
    const float* n = s + b;
    float x[2 * RHO + kRun];
#pragma unroll
    for (int q = 0; q < 2 * RHO + kRun; ++q) x[q] = n[q * P];
#pragma unroll
    for (int j = 0; j < kRun; ++j) {
        const float c = x[j + RHO];
        float e = te ? te[0] * c : 0.f, d = 0.f;
#pragma unroll
        for (int k = 1; k <= RHO; ++k) {
            const float l = x[j + RHO - k], r = x[j + RHO + k];
            if (te) e = fmaf(te[k], l + r, e);
            if (to) d = fmaf(to[k], l - r, d);
        }
        ev[j] = e;
        od[j] = d;
    }
}

// Any radius: the same sums with taps read pairwise from LDS.
SFOC_DEV void row_run_any(const float* p, int rho, const float* tg, const float* td, const float* tdd,
                          float og[kRun], float od[kRun], float odd[kRun]) {
#pragma unroll
    for (int j = 0; j < kRun; ++j) {
        const float c = p[j];
        float g = tg[0] * c, dd = tdd[0] * c, d = 0.f;
        for (int k = 1; k <= rho; ++k) {
            const float l = p[j - k], r = p[j + k];
            g = fmaf(tg[k], l + r, g);
            dd = fmaf(tdd[k], l + r, dd);
            d = fmaf(td[k], l - r, d);
        }
        og[j] = g;
        od[j] = d;
        odd[j] = dd;
    }
}
SFOC_DEV void col_run_any(const float* p, int P, int rho, const float* te, const float* to, float ev[kRun],
                          float od[kRun]) {
#pragma unroll
    for (int j = 0; j < kRun; ++j) {
        const float c = p[j * P];
        float e = te ? te[0] * c : 0.f, d = 0.f;
        for (int k = 1; k <= rho; ++k) {
            const float l = p[(j - k) * P], r = p[(j + k) * P];
            if (te) e = fmaf(te[k], l + r, e);
            if (to) d = fmaf(to[k], l - r, d);
        }
        ev[j] = e;
        od[j] = d;
    }
}

#define SFOC_RADIUS_SWITCH(rho, CALL_T, CALL_ANY) \
    switch (rho) {                                \
        case 1: CALL_T(1); break;                 \
        case 2: CALL_T(2); break;                 \
        case 3: CALL_T(3); break;                 \
        case 4: CALL_T(4); break;                 \
        case 5: CALL_T(5); break;                 \
        case 6: CALL_T(6); break;                 \
        case 7: CALL_T(7); break;                 \
        case 8: CALL_T(8); break;                 \
        case 9: CALL_T(9); break;                 \
        case 10: CALL_T(10); break;               \
        case 11: CALL_T(11); break;               \
        case 12: CALL_T(12); break;               \
        default: CALL_ANY; break;                 \
    }

// Two launch configurations of the 32 x 32 tile.  Configuration 0: three
// workgroups per CU, two steered channel maps per group.  Configuration 1
// (K = 1, rates 1-3, up to 16 channels): four workgroups per CU in at most
// 40 KB of LDS and 128 VGPRs each: the basis columns in two halves (half-width
// row-pass maps), one steered channel map per group, and the accumulators of
// one order at a time.  Both give the same descriptors bit for bit.
template <int Z, bool FAST, int VAR>
constexpr int describe_wpc() { return VAR ? 4 : (Z >= 32 ? 2 : 3); }
template <int Z, bool FAST, int VAR>
constexpr int describe_cg() { return VAR ? 1 : (FAST ? 2 : (Z >= 4 ? 4 : Z)); }

// The row sums, column sums and total of a tile that is not described, set
// to zero (the layout of the describe kernel's aggregate output).
SFOC_DEV void zero_tile_aggregates(const DescribeJob& J, int ty0, int tx0) {
    const IntegAgg ag = integ_agg(J.H, J.W);
    const int t = threadIdx.x, ta = ty0 / kTS, tb = tx0 / kTS;
    if (t < 2 * kTS) {
        const int q = t / kTS, i = t % kTS;
        if (ty0 + i < J.H) J.agg[(q ? ag.rs2 : ag.rs1) + tb * (int64_t)J.H + ty0 + i] = 0.0;
        if (tx0 + i < J.W) J.agg[(q ? ag.cs2 : ag.cs1) + ta * (int64_t)J.W + tx0 + i] = 0.0;
        if (i == 0) J.agg[(q ? ag.tt2 : ag.tt1) + ta * ag.ntx + tb] = 0.0;
    }
}

template <int Z, int CG, bool FAST, int VAR>
__global__ __launch_bounds__(kNT, (describe_wpc<Z, FAST, VAR>())) void describe_kernel(const DescribeJob single,
                                                          const DescribeJob* __restrict__ jobs,
                                                          const int4* __restrict__ tiles,
                                                          const uint8_t* __restrict__ tmask, const DescribeConsts C,
                                                          int BSP_, int ISX, int BPP_, int IPP) {
    extern __shared__ float lds[];
    const int t = threadIdx.x;
    DescribeJob J;
    int ty0, tx0;
    // Workgroups are dealt to the eight XCDs in turn; renumbered so that each
    // XCD takes a contiguous run of tiles, whose overlapping input halos then
    // meet in one L2.
    const int nblk = (int)(gridDim.x * gridDim.y), q8 = nblk / 8 * 8;
    const int id = (int)(blockIdx.y * gridDim.x + blockIdx.x);
    const int k = id < q8 ? (id % 8) * (q8 / 8) + id / 8 : id;
    if (tiles) {
        // entries: {job, tile row origin, tile column origin, what}; without
        // a job table every entry is of `single`, and a negative job is an
        // empty slot that the whole workgroup skips.  what = 1: a grid tile
        // that nothing reads, whose integral-image aggregates are set to
        // zero (the box sums over the tiles that are described stay exact);
        // what = 2: a grid tile that is described if the mask marks it
        const int4 e = tiles[k];
        if (e.x < 0) return;
        J = jobs ? load_table(jobs, e.x) : single;
        ty0 = e.y;
        tx0 = e.z;
        if (e.w == 1 || (e.w == 2 && !tmask[(ty0 / kTS) * ((J.W + kTS - 1) / kTS) + tx0 / kTS])) {
            if (J.agg) zero_tile_aggregates(J, ty0, tx0);
            return;
        }
    } else {
        J = single;
        ty0 = (k / gridDim.x) * kTS;
        tx0 = (k % gridDim.x) * kTS;
        // a grid tile outside the mask is not described; with integral
        // inputs its aggregates are set to zero
        if (tmask && !tmask[(ty0 / kTS) * gridDim.x + tx0 / kTS]) {
            if (J.agg) zero_tile_aggregates(J, ty0, tx0);
            return;
        }
    }
    const float* __restrict__ img = J.img;
    void* __restrict__ desc = J.desc;
    double* __restrict__ integ1 = J.integ1;
    double* __restrict__ integ2 = J.integ2;
    const int H = J.H, W = J.W;
    const int64_t ld = J.ld;
    // The K = 1, rates 1..3 path has Q = 3: its tile geometry is compile-time,
    // so the index arithmetic below divides by constants.
    constexpr int kFastQ = 3, kFastBSP = (kTS + 2 * kFastQ + kRun - 1) / kRun * kRun;
    const int Q = FAST ? kFastQ : C.Q;
    const int BSP = FAST ? kFastBSP : BSP_;
    const int BPP = FAST ? (kFastBSP | 1) : BPP_;
    const int R = C.R;
    const int nrun = BSP / kRun;
    float* simg = lds;
    float* srow = simg + ISX * IPP;
    float* sbas = lds;   // written once the image and row-pass maps are dead
    const int BB = BSP * BPP;   // one basis / channel map

    // 1. input region (top-left at tile origin - Q - R), reflect-101 borders;
    //    four rows' loads are issued before any of their LDS stores.
    {
        const int y0 = ty0 - Q - R, x0 = tx0 - Q - R;
        const bool inside = y0 >= 0 && x0 >= 0 && y0 + ISX <= H && x0 + ISX <= W;
        constexpr int kRows = kNT / 64, kU = 4;
        for (int b = t % 64; b < ISX; b += 64) {
            const int gx = inside ? x0 + b : reflect101(x0 + b, W);
            for (int a0 = t / 64; a0 < ISX; a0 += kRows * kU) {
                float v[kU];
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const int a = a0 + u * kRows;
                    v[u] = 0.f;
                    if (a < ISX) {
                        const int gy = inside ? y0 + a : reflect101(y0 + a, H);
                        v[u] = img[(int64_t)gy * ld + gx];
                    }
                }
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const int a = a0 + u * kRows;
                    if (a < ISX) simg[a * IPP + b] = v[u];
                }
            }
        }
    }
    __syncthreads();

    // 2. basis responses Gx, Gy, Gxx, Gyy, Gxy * I summed over sigma, held in
    //    registers by the thread that owns each vertical run of kRun pixels.
    // runs: (BSP / kRun) vertical runs in each of the BSr = kTS + 2Q columns
    // that steering reads (the padding columns up to BSP are skipped); BSP =
    // 40 and BSr = 38 when Q = 3 (the K = 1, rates 1-3 path), BSP at most 48
    // otherwise.
    constexpr int kMaxOwn = FAST ? 2 : 3;
    float bas[kMaxOwn][5][kRun];
#pragma unroll
    for (int o = 0; o < kMaxOwn; ++o)
#pragma unroll
        for (int m = 0; m < 5; ++m)
#pragma unroll
            for (int j = 0; j < kRun; ++j) bas[o][m][j] = 0.f;
    const int BSr = kTS + 2 * Q;      // rows / columns of the basis maps that steering reads
    const int ncolrun = nrun * BSr;   // (row-run, column) pairs
    if constexpr (VAR == 1) {
        // The basis columns in two halves, [0, 20) and [20, 38): per sigma
        // and half, a row pass over the half's 20 columns (five runs per
        // row) into half-width maps, then the column pass of that half.
        // Thread t owns run t of each half (10 row runs x the half's
        // columns), so bas[h] holds its half-h run for the whole sigma sum.
        constexpr int kHW = kFastBSP / 2, kHR = kHW / kRun;
        static_assert(kMaxOwn == 2 && kFastBSP == 40 && kNT >= kHW * (kFastBSP / kRun), "two halves of 40 columns");
        for (int s = 0; s < C.nsig; ++s) {
            const int rho = C.rad[s];
            const float* tg = C.taps + C.off[s];
            const float* td = tg + (rho + 1);
            const float* tdd = td + (rho + 1);
            const float cn = C.cnorm[s];
            const int use = C.use[s];
            const int rows = BSP + 2 * rho;
            const int ig = ISX * IPP, id = ig + rows * kHalfPitch, idd = ig + 2 * rows * kHalfPitch;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                for (int e = t; e < rows * kHR; e += kNT) {
                    const int a = e / kHR, b0 = (e - a * kHR) * kRun;
                    const float* p = simg + (a + R - rho) * IPP + (h * kHW + b0 + R);
                    float og[kRun], od[kRun], odd[kRun];
#define ROW_T(RR) row_run<RR>(p, tg, td, tdd, og, od, odd)
                    SFOC_RADIUS_SWITCH(rho, ROW_T, row_run_any(p, rho, tg, td, tdd, og, od, odd))
#undef ROW_T
                    float* w = srow + a * kHalfPitch + b0;
#pragma unroll
                    for (int j = 0; j < kRun; ++j) {
                        w[j] = og[j];
                        w[rows * kHalfPitch + j] = od[j];
                        w[2 * rows * kHalfPitch + j] = odd[j];
                    }
                }
                __syncthreads();
                const int wh = h ? BSr - kHW : kHW;   // basis columns of this half
                if (t < wh * nrun) {
                    const int b = t % wh, a0 = (t / wh) * kRun;
                    float bx[kRun], by[kRun], bxx[kRun], byy[kRun], bxy[kRun], dummy[kRun];
                    const int c0 = (a0 + rho) * kHalfPitch + b;
#define COL_T(RR)                                                       \
    do {                                                                \
        col_run<RR>(lds, ig + c0, kHalfPitch, tdd, td, byy, by);        \
        col_run<RR>(lds, id + c0, kHalfPitch, tg, td, bx, bxy);         \
        col_run<RR>(lds, idd + c0, kHalfPitch, tg, nullptr, bxx, dummy); \
    } while (0)
#define COL_ANY                                                         \
    do {                                                                \
        col_run_any(lds + ig + c0, kHalfPitch, rho, tdd, td, byy, by);  \
        col_run_any(lds + id + c0, kHalfPitch, rho, tg, td, bx, bxy);   \
        col_run_any(lds + idd + c0, kHalfPitch, rho, tg, nullptr, bxx, dummy); \
    } while (0)
                    SFOC_RADIUS_SWITCH(rho, COL_T, COL_ANY)
#undef COL_T
#undef COL_ANY
                    (void)dummy;
#pragma unroll
                    for (int j = 0; j < kRun; ++j) {
                        if (use & 1) {
                            bas[h][0][j] = fmaf(cn, bx[j], bas[h][0][j]);
                            bas[h][1][j] = fmaf(cn, by[j], bas[h][1][j]);
                        }
                        if (use & 2) {
                            bas[h][2][j] = fmaf(cn, bxx[j], bas[h][2][j]);
                            bas[h][3][j] = fmaf(cn, byy[j], bas[h][3][j]);
                            bas[h][4][j] = fmaf(cn, bxy[j], bas[h][4][j]);
                        }
                    }
                }
                __syncthreads();
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int wh = h ? BSr - kHW : kHW;
            if (t < wh * nrun) {
                const int b = h * kHW + t % wh, a0 = (t / wh) * kRun;
#pragma unroll
                for (int m = 0; m < 5; ++m)
#pragma unroll
                    for (int j = 0; j < kRun; ++j) sbas[m * BB + (a0 + j) * BPP + b] = bas[h][m][j];
            }
        }
    } else {
        for (int s = 0; s < C.nsig; ++s) {
            const int rho = C.rad[s];
            const float* tg = C.taps + C.off[s];
            const float* td = tg + (rho + 1);
            const float* tdd = td + (rho + 1);
            const float cn = C.cnorm[s];
            const int rows = BSP + 2 * rho;
            // row pass on rows [0, rows) x cols [0, BSP): horizontal runs.  Row a
            // of this pass is image-region row a + R - rho.
            for (int e = t; e < rows * nrun; e += kNT) {
                const int a = e / nrun, b0 = (e - a * nrun) * kRun;
                const float* p = simg + (a + R - rho) * IPP + (b0 + R);
                float og[kRun], od[kRun], odd[kRun];
#define ROW_T(RR) row_run<RR>(p, tg, td, tdd, og, od, odd)
                SFOC_RADIUS_SWITCH(rho, ROW_T, row_run_any(p, rho, tg, td, tdd, og, od, odd))
#undef ROW_T
                float* w = srow + a * BPP + b0;
#pragma unroll
                for (int j = 0; j < kRun; ++j) {
                    w[j] = og[j];
                    w[rows * BPP + j] = od[j];
                    w[2 * rows * BPP + j] = odd[j];
                }
            }
            __syncthreads();
            // column pass on vertical runs; output row a reads pass rows a + rho + k.
            const float* rg = srow;
            const float* rd = srow + rows * BPP;
            const float* rdd = srow + 2 * rows * BPP;
            const int ig = ISX * IPP, id = ig + rows * BPP, idd = ig + 2 * rows * BPP;   // the same, as lds indices
            const int use = C.use[s];
#pragma unroll
            for (int o = 0; o < kMaxOwn; ++o) {
                const int e = t + o * kNT;
                if (e < ncolrun) {
                    const int b = e % BSr, a0 = (e / BSr) * kRun;
                    float bx[kRun], by[kRun], bxx[kRun], byy[kRun], bxy[kRun], dummy[kRun];
                    const int c0 = (a0 + rho) * BPP + b;
                    // rg -> By (odd d), Byy (even dd); rd -> Bx (even g), Bxy (odd d);
                    // rdd -> Bxx (even g).
#define COL_T(RR)                                                \
        do {                                                         \
            col_run<RR>(lds, ig + c0, BPP, tdd, td, byy, by);        \
            col_run<RR>(lds, id + c0, BPP, tg, td, bx, bxy);         \
            col_run<RR>(lds, idd + c0, BPP, tg, nullptr, bxx, dummy); \
        } while (0)
#define COL_ANY                                                  \
        do {                                                         \
            col_run_any(rg + c0, BPP, rho, tdd, td, byy, by);        \
            col_run_any(rd + c0, BPP, rho, tg, td, bx, bxy);         \
            col_run_any(rdd + c0, BPP, rho, tg, nullptr, bxx, dummy); \
        } while (0)
                    SFOC_RADIUS_SWITCH(rho, COL_T, COL_ANY)
#undef COL_T
#undef COL_ANY
                    (void)dummy;
#pragma unroll
                    for (int j = 0; j < kRun; ++j) {
                        // the 2-D normalisation cn of this sigma, applied as the
                        // response joins the sum over sigma
                        if (use & 1) {
                            bas[o][0][j] = fmaf(cn, bx[j], bas[o][0][j]);
                            bas[o][1][j] = fmaf(cn, by[j], bas[o][1][j]);
                        }
                        if (use & 2) {
                            bas[o][2][j] = fmaf(cn, bxx[j], bas[o][2][j]);
                            bas[o][3][j] = fmaf(cn, byy[j], bas[o][3][j]);
                            bas[o][4][j] = fmaf(cn, bxy[j], bas[o][4][j]);
                        }
                    }
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int o = 0; o < kMaxOwn; ++o) {
            const int e = t + o * kNT;
            if (e < ncolrun) {
                const int b = e % BSr, a0 = (e / BSr) * kRun;
#pragma unroll
                for (int m = 0; m < 5; ++m)
#pragma unroll
                    for (int j = 0; j < kRun; ++j) sbas[m * BB + (a0 + j) * BPP + b] = bas[o][m][j];
            }
        }
    }
    __syncthreads();

    // 3. steer + rectify per channel group into LDS, then dilated smoothing
    //    of this thread's horizontal run of kRun outputs.
    float acc[Z][kRun];
    float* schan = sbas + 5 * BB;
    // The fast path has both orders (N = Z / 2 at compile time).
    const int N = FAST ? Z / 2 : C.N;
    const int B = 2 * C.K + 1;
    const int oy = t / (kTS / kRun), ox0 = (t % (kTS / kRun)) * kRun;

    // 4. (per order block) normalisation, rounding, store, channel sums.
    //    Each thread stores its run of kRun pixels of a channel as one
    //    vector (8 threads cover a 128-byte row segment), so every store
    //    instruction writes whole cache lines; unaligned widths, tiles whose
    //    column origin is not a multiple of kRun and the right edge fall back
    //    to scalar stores.  The channel sums for the
    //    integral images accumulate in channel order.
    const int64_t plane = (int64_t)H * W;
    const int gy = ty0 + oy, gx0 = tx0 + ox0;
    const size_t align = C.dtype == SFOC_DTYPE_F32 ? 15 : 7;
    const bool full =
        (W & (kRun - 1)) == 0 && (gx0 & (kRun - 1)) == 0 && ((uintptr_t)desc & align) == 0 && gx0 + kRun <= W;
    const int64_t off0 = (int64_t)gy * W + gx0;
    double d1[kRun], d2[kRun];
#pragma unroll
    for (int j = 0; j < kRun; ++j) d1[j] = d2[j] = 0.0;
    auto emit = [&](int lo, int hi) {   // channels [lo, hi): one order block
        float inv[kRun];
#pragma unroll
        for (int j = 0; j < kRun; ++j) {
            float s2 = 0.f;
#pragma unroll
            for (int c = 0; c < Z; ++c)
                if (c >= lo && c < hi) s2 = fmaf(acc[c][j], acc[c][j], s2);
            inv[j] = rsqrtf(s2 + C.eps);
        }
        if (gy >= H) return;
#pragma unroll
        for (int c = 0; c < Z; ++c) {
            if (c < lo || c >= hi) continue;
            float v[kRun];
#pragma unroll
            for (int j = 0; j < kRun; ++j) v[j] = acc[c][j] * inv[j];
            if (C.dtype == SFOC_DTYPE_F32) {
                float* dst = (float*)desc + c * plane + off0;
                if (full) {
                    *(float4*)dst = make_float4(v[0], v[1], v[2], v[3]);
                } else {
#pragma unroll
                    for (int j = 0; j < kRun; ++j)
                        if (gx0 + j < W) dst[j] = v[j];
                }
            } else {
                uint16_t q[kRun];
#pragma unroll
                for (int j = 0; j < kRun; ++j) {
                    q[j] = C.dtype == SFOC_DTYPE_BF16 ? f32_to_bf16_bits(v[j]) : f32_to_f16_bits(v[j]);
                    v[j] = C.dtype == SFOC_DTYPE_BF16 ? bf16_bits_to_f32(q[j]) : f16_bits_to_f32(q[j]);
                }
                uint16_t* dst = (uint16_t*)desc + c * plane + off0;
                if (full) {
                    *(ushort4*)dst = make_ushort4(q[0], q[1], q[2], q[3]);
                } else {
#pragma unroll
                    for (int j = 0; j < kRun; ++j)
                        if (gx0 + j < W) dst[j] = q[j];
                }
            }
            if (integ1) {
#pragma unroll
                for (int j = 0; j < kRun; ++j) {
                    const double dv = (double)v[j];
                    d1[j] += dv;
                    d2[j] = fma(dv, dv, d2[j]);
                }
            }
        }
    };
    // channels [lo, hi) in groups of CG: steer into LDS, then smooth
    auto steer_smooth = [&](int lo, int hi) {
#pragma unroll
    for (int c0 = lo; c0 < hi; c0 += CG) {
        // thread index laundered per group: keeps the group's LDS addresses
        // from being hoisted (and kept live) across the whole channel loop.
        int tl = t;
        asm volatile("" : "+v"(tl));
        const int obase = (tl / (kTS / kRun) + Q) * BPP + (tl % (kTS / kRun)) * kRun + Q;
        for (int e = tl; e < BSr * BSr; e += kNT) {
            const int a = e / BSr, b = e - a * BSr;
            const int idx = a * BPP + b;
#pragma unroll
            for (int cc = 0; cc < CG; ++cc) {
                const int c = c0 + cc;
                if (c < Z) {
                    float v;
                    if (c < N) {
                        v = C.c1[c] * sbas[idx] + C.s1[c] * sbas[BB + idx];
                    } else {
                        const int k = c - N;
                        v = C.cc[k] * sbas[2 * BB + idx] + C.ss[k] * sbas[3 * BB + idx] +
                            C.sc2[k] * sbas[4 * BB + idx];
                    }
                    if (C.rectify == SFOC_RECTIFY_ABS) v = fabsf(v);
                    else if (C.rectify == SFOC_RECTIFY_RELU) v = fmaxf(v, 0.f);
                    schan[cc * BB + idx] = v;
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int cc = 0; cc < CG; ++cc) {
            const int c = c0 + cc;
            if (c < Z) {
                const float* w = (c < N) ? C.w1 : C.w2;
                const float* ch = schan + cc * BB + obase;
                if (FAST) {
                    smooth_run_k1_123(lds, (5 + cc) * BB + obase, BPP, w[4], w[1], w[0], acc[c]);
                    // one channel's reads in flight at a time (the scheduler
                    // would otherwise hoist all of a group's LDS reads)
                    __builtin_amdgcn_sched_barrier(0);
                } else {
#pragma unroll
                    for (int j = 0; j < kRun; ++j) {
                        float a = 0.f;
                        for (int di = 0; di < C.ndil; ++di) {
                            const int r = C.dil[di];
                            for (int i = 0; i < B; ++i)
                                for (int jj = 0; jj < B; ++jj)
                                    a = fmaf(w[i * B + jj], ch[(i - C.K) * r * BPP + (jj - C.K) * r + j], a);
                        }
                        acc[c][j] = a;
                    }
                }
            }
        }
        __syncthreads();
    }
    };
    if constexpr (VAR == 1) {
        // one order at a time: its accumulators die at its emit
        steer_smooth(0, Z / 2);
        emit(0, Z / 2);
        steer_smooth(Z / 2, Z);
        emit(Z / 2, Z);
    } else {
        steer_smooth(0, Z);
        emit(0, N);
        emit(N, Z);
    }
    if (integ1) {
        // Per-pixel channel sums of the stored values (zero outside the
        // image) into the integral-image buffers, and this tile's aggregates
        // for the prefix pass: row sums (the 8 lanes of a row, butterfly),
        // column sums (the 8 rows of a wave, butterfly, then the 4 waves in
        // order) and the total (the 32 column sums, butterfly).  Every sum is
        // taken in a fixed order, so the integral images are reproducible.
#pragma unroll
        for (int j = 0; j < kRun; ++j)
            if (gy >= H || gx0 + j >= W) d1[j] = d2[j] = 0.0;
        if (gy < H) {
            const int64_t io = (int64_t)(gy + 1) * (W + 1) + gx0 + 1;
#pragma unroll
            for (int j = 0; j < kRun; ++j)
                if (gx0 + j < W) {
                    integ1[io + j] = d1[j];
                    integ2[io + j] = d2[j];
                }
        }
        const IntegAgg ag = integ_agg(H, W);
        double* __restrict__ agg = J.agg;
        const int tb = tx0 / kTS, ta = ty0 / kTS;
        double r1 = ((d1[0] + d1[1]) + d1[2]) + d1[3];
        double r2 = ((d2[0] + d2[1]) + d2[2]) + d2[3];
#pragma unroll
        for (int d = 1; d < kTS / kRun; d <<= 1) {
            r1 += __shfl_xor(r1, d, 64);
            r2 += __shfl_xor(r2, d, 64);
        }
        if ((t & (kTS / kRun - 1)) == 0 && gy < H) {
            agg[ag.rs1 + tb * (int64_t)H + gy] = r1;
            agg[ag.rs2 + tb * (int64_t)H + gy] = r2;
        }
#pragma unroll
        for (int j = 0; j < kRun; ++j)
#pragma unroll
            for (int d = kTS / kRun; d < 64; d <<= 1) {
                d1[j] += __shfl_xor(d1[j], d, 64);
                d2[j] += __shfl_xor(d2[j], d, 64);
            }
        double* cs = reinterpret_cast<double*>(lds);   // [map][wave][column], then [map][column]
        const int lane = t & 63, wv = t >> 6;
        if (lane < kTS / kRun) {
#pragma unroll
            for (int j = 0; j < kRun; ++j) {
                cs[(0 * (kNT / 64) + wv) * kTS + lane * kRun + j] = d1[j];
                cs[(1 * (kNT / 64) + wv) * kTS + lane * kRun + j] = d2[j];
            }
        }
        __syncthreads();
        static_assert(2 * kTS == 64, "the column sums of both maps fill one wave");
        if (t < 2 * kTS) {
            // wave 0: lane q * 32 + x sums column x of map q over the four
            // waves in order, then the 32 columns of each map are summed by
            // a butterfly within its half-wave (a fixed order)
            const int q = t / kTS, x = t % kTS;
            double c = 0.0;
#pragma unroll
            for (int w = 0; w < kNT / 64; ++w) c += cs[(q * (kNT / 64) + w) * kTS + x];
            if (tx0 + x < W) agg[(q ? ag.cs2 : ag.cs1) + ta * (int64_t)W + tx0 + x] = c;
#pragma unroll
            for (int d = 1; d < kTS; d <<= 1) c += __shfl_xor(c, d, 64);
            if (x == 0) agg[(q ? ag.tt2 : ag.tt1) + ta * ag.ntx + tb] = c;
        }
    }
}


// ---- integral images (Eq. 14-16) ------------------------------------------
// The inclusive 2-D prefix sum (Eq. 15) of a per-pixel map s, at a pixel
// (y0 + i, x0 + j) of the tile (a, b) with origin (y0, x0), splits into
//   Corner(a, b)                  the tiles above and to the left,
// + sum_{j' <= j} Above(x0 + j')  the rows above the tile, per column,
// + sum_{i' <= i} [Left(y0 + i') + sum_{j' <= j} s(y0 + i', x0 + j')]
// with Left(y) the sum of row y left of the tile and Above(x) the sum of
// column x above it.  The describe kernel wrote s into the integral buffers
// and each tile's row sums, column sums and total; integral_prefix turns
// these into Left (exclusive prefixes of the row sums over tile columns),
// Above (of the column sums over tile rows) and Corner (the 2-D exclusive
// prefix of the tile totals); integral_tiles then reads s once and writes
// the prefix sums in place.  All sums are in a fixed order.

// In place, for two sequences at once: a[0], a[step], ... and b[0],
// b[step], ... (n entries each) -> their exclusive prefix sums.  Sixteen
// loads of each are in flight before their sums, which run in order.
SFOC_DEV void exclusive_prefix2(double* __restrict__ a, double* __restrict__ b, int64_t n, int64_t step) {
    constexpr int kB = 16;
    double ra = 0.0, rb = 0.0;
    int64_t k = 0;
    for (; k + kB <= n; k += kB) {
        double x[kB], y[kB];
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            x[u] = a[(k + u) * step];
            y[u] = b[(k + u) * step];
        }
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            a[(k + u) * step] = ra;
            b[(k + u) * step] = rb;
            ra += x[u];
            rb += y[u];
        }
    }
    for (; k < n; ++k) {
        const double x = a[k * step], y = b[k * step];
        a[k * step] = ra;
        b[k * step] = rb;
        ra += x;
        rb += y;
    }
}

void integral_prefix_items(int job, int H, int W, std::vector<int4>& out) {
    for (int k = 0; k < (H + kScanNT - 1) / kScanNT; ++k) out.push_back(make_int4(job, 0, k, 0));
    for (int k = 0; k < (W + kScanNT - 1) / kScanNT; ++k) out.push_back(make_int4(job, 1, k, 0));
    out.push_back(make_int4(job, 2, 0, 0));
}

template <bool BATCH>
__global__ __launch_bounds__(kScanNT) void integral_prefix(const IntegJob single, const IntegJob* __restrict__ jobs,
                                                           const int4* __restrict__ items) {
    IntegJob J;
    int kind, blk;
    if (BATCH) {
        const int4 it = items[blockIdx.x];
        J = load_table(jobs, it.x);
        kind = it.y;
        blk = it.z;
    } else {
        J = single;
        const int nbr = (J.H + kScanNT - 1) / kScanNT, nbc = (J.W + kScanNT - 1) / kScanNT;
        const int k = blockIdx.x;
        kind = k < nbr ? 0 : (k < nbr + nbc ? 1 : 2);
        blk = kind == 0 ? k : (kind == 1 ? k - nbr : 0);
    }
    const int H = J.H, W = J.W, t = threadIdx.x;
    const IntegAgg ag = integ_agg(H, W);
    double* __restrict__ agg = J.agg;
    if (kind == 0) {          // Left: per row y, over the tile columns
        const int y = blk * kScanNT + t;
        if (y < H) exclusive_prefix2(agg + ag.rs1 + y, agg + ag.rs2 + y, ag.ntx, H);
    } else if (kind == 1) {   // Above: per column x, over the tile rows
        const int x = blk * kScanNT + t;
        if (x < W) exclusive_prefix2(agg + ag.cs1 + x, agg + ag.cs2 + x, ag.nty, W);
    } else {                  // Corner: tile totals, over tile columns, then over tile rows
        for (int64_t a = t; a < ag.nty; a += kScanNT)
            exclusive_prefix2(agg + ag.tt1 + a * ag.ntx, agg + ag.tt2 + a * ag.ntx, ag.ntx, 1);
        __syncthreads();
        for (int64_t b = t; b < ag.ntx; b += kScanNT)
            exclusive_prefix2(agg + ag.tt1 + b, agg + ag.tt2 + b, ag.nty, ag.ntx);
    }
}

// One 32 x 32 tile per workgroup, in three phases over an LDS copy of the
// tile.  Thread t first holds column t % 32 of rows 4 (t / 32) .. + 3, so a
// wave's loads and stores cover two rows of 32 consecutive pixels: it loads
// s, sums down its four rows, then adds the totals of the row groups above
// (the column prefix C).  Then thread t holds a run of 4 pixels of row t / 8
// and sums C along the row: I = Corner + prefix(Above) + prefix(Left) +
// prefix over the row of C, the decomposition above in another order.  The
// results go back through LDS to the column layout for the stores.  Row 0
// and column 0 of the integral images are set to zero by the tiles that
// border them.
template <bool BATCH>
__global__ __launch_bounds__(kScanNT) void integral_tiles(const IntegJob single, const IntegJob* __restrict__ jobs,
                                                          const int4* __restrict__ tiles,
                                                          uint8_t* __restrict__ tmask) {
    constexpr int kRows = kTS * kTS / kScanNT;   // rows per thread in the column layout
    constexpr int kGroups = kTS / kRows;         // row groups in a tile
    constexpr int kRuns = kTS / kRun;            // runs in a tile row
    static_assert(kRows == 4 && kGroups * kTS == kScanNT && kRuns * kTS == kScanNT, "tile layouts");
    IntegJob J;
    int ta, tb;
    // Workgroups are dealt to the eight XCDs in turn; renumbered so that each
    // XCD takes one contiguous run of tiles (row-major), neighbouring tiles
    // share an L2 and the cache lines on their borders (the images' row
    // pitch W + 1 is not a multiple of a line) are fetched once.
    const int nblk = BATCH ? (int)gridDim.x : (int)(gridDim.x * gridDim.y);
    const int id = BATCH ? (int)blockIdx.x : (int)(blockIdx.y * gridDim.x + blockIdx.x);
    const int q8 = nblk / 8 * 8;
    const int k = id < q8 ? (id % 8) * (q8 / 8) + id / 8 : id;
    if (BATCH) {
        const int4 e = tiles[k];
        J = load_table(jobs, e.x);
        ta = e.y;
        tb = e.z;
    } else {
        J = single;
        ta = k / gridDim.x;
        tb = k - ta * gridDim.x;
        if (tmask) {   // the mask's last reader: the byte is cleared for the next call
            const bool read = tmask[k] != 0;
            __syncthreads();
            if (threadIdx.x == 0) tmask[k] = 0;
            if (!read) return;   // a tile that nothing reads
        }
    }
    __shared__ double T[2][kTS][kTS + 1];   // the tile of both maps
    __shared__ double tot[2][kScanNT];      // row-group totals, then run totals
    __shared__ double pre_left[2][kTS];     // inclusive prefix of Left over the tile rows
    __shared__ double pre_above[2][kTS];    // Corner + inclusive prefix of Above over the tile columns
    const int H = J.H, W = J.W, t = threadIdx.x;
    const IntegAgg ag = integ_agg(H, W);
    const double* __restrict__ agg = J.agg;
    const int64_t P = W + 1;
    const int y0 = ta * kTS, x0 = tb * kTS;
    const int c = t % kTS, gr = t / kTS;    // column layout: column c, rows kRows * gr + k
    // Left (map 1 in lanes 0..31, map 2 in lanes 32..63 of waves 0 and 2)
    // and Above with Corner (waves 1 and 3), loaded before the tile and
    // without branches (waves 2 and 3 repeat 0 and 1; only those store).
    const bool is_above = (t / (2 * kTS)) & 1;
    const int qa = (t / kTS) & 1, ea = t % kTS;
    const int64_t ia = is_above ? (qa ? ag.cs2 : ag.cs1) + ta * (int64_t)W + min(x0 + ea, W - 1)
                                : (qa ? ag.rs2 : ag.rs1) + tb * (int64_t)H + min(y0 + ea, H - 1);
    const double va_in = agg[ia];
    const bool va_ok = is_above ? x0 + ea < W : y0 + ea < H;
    const double corner = agg[(qa ? ag.tt2 : ag.tt1) + ta * ag.ntx + tb];
    // The tile, at clamped addresses (every load in bounds and all of them in
    // flight at once); pixels outside the image count as zero.
    double s[2][kRows];
    bool ok[kRows];
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
        const int y = y0 + kRows * gr + k, x = x0 + c;
        ok[k] = y < H && x < W;
        const int64_t off = (int64_t)(min(y, H - 1) + 1) * P + min(x, W - 1) + 1;
        s[0][k] = J.g1[off];
        s[1][k] = J.g2[off];
    }
    // the prefixes of Left, and of Above with Corner
    double va = va_ok ? va_in : 0.0;
#pragma unroll
    for (int d = 1; d < kTS; d <<= 1) {
        const double u = __shfl_up(va, d, kTS);
        if (ea >= d) va += u;
    }
    if (t < 4 * kTS) {
        if (!is_above) pre_left[qa][ea] = va;
        else pre_above[qa][ea] = corner + va;
    }
    // column prefix: down the thread's rows, then the row groups above
#pragma unroll
    for (int q = 0; q < 2; ++q) {
#pragma unroll
        for (int k = 0; k < kRows; ++k) s[q][k] = ok[k] ? s[q][k] : 0.0;
#pragma unroll
        for (int k = 1; k < kRows; ++k) s[q][k] += s[q][k - 1];
        tot[q][gr * kTS + c] = s[q][kRows - 1];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        double e = 0.0;
        for (int g2 = 0; g2 < gr; ++g2) e += tot[q][g2 * kTS + c];
#pragma unroll
        for (int k = 0; k < kRows; ++k) T[q][kRows * gr + k][c] = s[q][k] + e;
    }
    __syncthreads();
    // row prefix of C: thread t holds the run of row i from column j0
    const int i = t / kRuns, rl = t % kRuns, j0 = rl * kRun;
    double v[2][kRun];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
#pragma unroll
        for (int k = 0; k < kRun; ++k) v[q][k] = T[q][i][j0 + k];
#pragma unroll
        for (int k = 1; k < kRun; ++k) v[q][k] += v[q][k - 1];
        tot[q][i * kRuns + rl] = v[q][kRun - 1];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        double e = pre_left[q][i];
        for (int r2 = 0; r2 < rl; ++r2) e += tot[q][i * kRuns + r2];
#pragma unroll
        for (int k = 0; k < kRun; ++k) T[q][i][j0 + k] = pre_above[q][j0 + k] + (e + v[q][k]);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        double* __restrict__ g = q ? J.g2 : J.g1;
#pragma unroll
        for (int k = 0; k < kRows; ++k) {
            const int y = y0 + kRows * gr + k, x = x0 + c;
            if (ok[k]) g[(int64_t)(y + 1) * P + x + 1] = T[q][kRows * gr + k][c];
        }
        if (ta == 0 && t < kTS && x0 + t < W) g[x0 + t + 1] = 0.0;
        if (ta == 0 && tb == 0 && t == 0) g[0] = 0.0;
        if (tb == 0 && t < kTS && y0 + t < H) g[(int64_t)(y0 + t + 1) * P] = 0.0;
    }
}

// ---- launch -------------------------------------------------------------
template <int Z, bool FAST, int VAR>
static hipError_t launch_describe_zf(const DescribeJob& job, const DescribeJob* jobs, const int4* tiles, int ntiles,
                                     const uint8_t* tmask, const DescribeConsts& c, hipStream_t st) {
    constexpr int CG = describe_cg<Z, FAST, VAR>();
    const DescribeGeom g = describe_geom(c, CG, VAR == 1);
    dim3 grid = tiles ? dim3(ntiles) : dim3((job.W + kTS - 1) / kTS, (job.H + kTS - 1) / kTS);
    if (grid.x == 0) return hipSuccess;
    auto kern = describe_kernel<Z, CG, FAST, VAR>;
    hipError_t e = ensure_dynamic_lds((const void*)kern, (int)g.bytes);
    if (e != hipSuccess) return e;
    trace_begin(st, SFOC_K_DESCRIBE);
    hipLaunchKernelGGL(kern, grid, dim3(kNT), g.bytes, st, job, jobs, tiles, tmask, c, g.BSP, g.ISX, g.BPP, g.IPP);
    trace_end(st, SFOC_K_DESCRIBE);
    return hipGetLastError();
}

// The K = 1, rates 1-3 path with both orders: compile-time geometry.
static bool describe_fast(const DescribeConsts& c) {
    return c.K == 1 && c.ndil == 3 && c.dil[0] == 1 && c.dil[1] == 2 && c.dil[2] == 3 && c.second &&
           c.N * 2 == c.z;
}

int describe_configs(const DescribeConsts& c) { return describe_fast(c) && c.z <= 16 && c.z % 2 == 0 ? 2 : 1; }

template <int Z>
static hipError_t launch_describe_z(const DescribeJob& job, const DescribeJob* jobs, const int4* tiles, int ntiles,
                                    const uint8_t* tmask, const DescribeConsts& c, hipStream_t st, int var) {
    if (!describe_fast(c)) return launch_describe_zf<Z, false, 0>(job, jobs, tiles, ntiles, tmask, c, st);
    if constexpr (Z <= 16 && Z % 2 == 0)
        if (var == 1) return launch_describe_zf<Z, true, 1>(job, jobs, tiles, ntiles, tmask, c, st);
    return launch_describe_zf<Z, true, 0>(job, jobs, tiles, ntiles, tmask, c, st);
}

static hipError_t launch_describe_any(const DescribeJob& job, const DescribeJob* jobs, const int4* tiles, int ntiles,
                                      const uint8_t* tmask, const DescribeConsts& c, hipStream_t st, int var) {
    switch (c.z) {
        case 2: return launch_describe_z<2>(job, jobs, tiles, ntiles, tmask, c, st, var);
        case 3: return launch_describe_z<3>(job, jobs, tiles, ntiles, tmask, c, st, var);
        case 4: return launch_describe_z<4>(job, jobs, tiles, ntiles, tmask, c, st, var);
        case 6: return launch_describe_z<6>(job, jobs, tiles, ntiles, tmask, c, st, var);
        case 8: return launch_describe_z<8>(job, jobs, tiles, ntiles, tmask, c, st, var);
        case 12: return launch_describe_z<12>(job, jobs, tiles, ntiles, tmask, c, st, var);
        case 16: return launch_describe_z<16>(job, jobs, tiles, ntiles, tmask, c, st, var);
        case 24: return launch_describe_z<24>(job, jobs, tiles, ntiles, tmask, c, st, var);
        case 32: return launch_describe_z<32>(job, jobs, tiles, ntiles, tmask, c, st, var);
        default: return hipErrorInvalidValue;
    }
}

// Several images in one launch: jobs and tiles are device tables.
hipError_t launch_describe_batched(const DescribeJob* jobs, const int4* tiles, int ntiles, const DescribeConsts& c,
                                   hipStream_t st, int var) {
    DescribeJob none{};
    return launch_describe_any(none, jobs, tiles, ntiles, nullptr, c, st, var);
}

hipError_t launch_describe(const float* img, int H, int W, int64_t ld, void* desc, double* i1, double* i2,
                           double* agg, const DescribeConsts& c, hipStream_t st, const uint8_t* tmask) {
    DescribeJob job{img, desc, i1, i2, agg, ld, H, W};
    return launch_describe_any(job, nullptr, nullptr, 0, tmask, c, st, 0);
}

hipError_t launch_describe_tiles(const float* img, int H, int W, int64_t ld, void* desc, const int4* tiles,
                                 int ntiles, const DescribeConsts& c, hipStream_t st) {
    if (ntiles == 0) return hipSuccess;
    DescribeJob job{img, desc, nullptr, nullptr, nullptr, ld, H, W};
    return launch_describe_any(job, nullptr, tiles, ntiles, nullptr, c, st, 0);
}

// ---- the pair call's describe table ---------------------------------------
// One launch describes both images of a pair.  Entries 0 .. NR - 1 of the
// table are the reference image's grid tiles in row-major order, {0, row
// origin, column origin, 2}: described where the window mask marks the
// tile, else given zero integral-image aggregates.  Slot (i, a, c) after
// them, i < n, a, c < ceil(m / T), is the sensed image's tile of IP i's
// template with rows from the template's row a * T and columns from its
// column c * T ({1, ...}), or an empty slot (job -1) where the IP reads
// nothing (template_tile_range).  Tiles of two IPs may overlap: both
// describe the shared pixels, with equal results (a pixel's descriptor does
// not depend on the tile that computes it).  Thread 0 writes the two jobs;
// thread i < n also marks the reference tiles of IP i's search window
// (window_tile_range, the rule batched plans apply on the host), byte
// stores of 1 in any order.  The mask is not cleared first: the integral
// pass, its last reader, clears every byte it reads, and a byte left set by
// memory that never held a mask only makes a tile be described that
// nothing reads.
__global__ __launch_bounds__(256) void pair_table_kernel(const int32_t* __restrict__ ips,
                                                         const int32_t* __restrict__ prior, int n, int m, int r,
                                                         int Hs, int Ws, int Hr, int Wr, const DescribeJob jref,
                                                         const DescribeJob jsen, DescribeJob* __restrict__ jobs,
                                                         int4* __restrict__ tiles, uint8_t* __restrict__ mask) {
    const int S = template_tile_slots(m, kTS), CT = template_tile_rows(m, kTS);
    const int ntx = (Wr + kTS - 1) / kTS, NR = ntx * ((Hr + kTS - 1) / kTS);
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e == 0) {
        jobs[0] = jref;
        jobs[1] = jsen;
    }
    if (e < n) {
        const int i = (int)e;
        int64_t a0, a1, b0, b1;
        if (window_tile_range(ips[2 * i], ips[2 * i + 1], prior ? prior[2 * i] : 0, prior ? prior[2 * i + 1] : 0, m,
                              r, Hs, Ws, Hr, Wr, kTS, &a0, &a1, &b0, &b1))
            for (int64_t a = a0; a <= a1; ++a)
                for (int64_t b = b0; b <= b1; ++b) mask[a * ntx + b] = 1;
    }
    if (e < NR) {
        const int a = (int)(e / ntx), b = (int)(e - (int64_t)a * ntx);
        tiles[e] = make_int4(0, a * kTS, b * kTS, 2);
    } else if (e < NR + (int64_t)n * S) {
        const int64_t f = e - NR;
        const int i = (int)(f / S), s = (int)(f - (int64_t)i * S), a = s / CT, c = s - a * CT;
        int64_t ty, tx;
        const bool in = template_tile_range(ips[2 * i], ips[2 * i + 1], prior ? prior[2 * i] : 0,
                                            prior ? prior[2 * i + 1] : 0, m, r, Hs, Ws, Hr, Wr, &ty, &tx);
        tiles[e] = in ? make_int4(1, (int)(ty + (int64_t)a * kTS), (int)(tx + (int64_t)c * kTS), 0)
                      : make_int4(-1, 0, 0, 0);
    }
}

int64_t pair_table_entries(int Hr, int Wr, int n, int m) {
    return (int64_t)((Wr + kTS - 1) / kTS) * ((Hr + kTS - 1) / kTS) + (int64_t)n * template_tile_slots(m, kTS);
}

hipError_t launch_describe_pair(const float* ref, int Hr, int Wr, int64_t ldr, void* dref, double* i1, double* i2,
                                double* agg, const float* sen, int Hs, int Ws, int64_t lds, void* dsen,
                                const int32_t* ips, const int32_t* prior, int n, int m, int r, DescribeJob* jobs,
                                int4* tiles, uint8_t* mask, const DescribeConsts& c, hipStream_t st) {
    const DescribeJob jref{ref, dref, i1, i2, agg, ldr, Hr, Wr};
    const DescribeJob jsen{sen, dsen, nullptr, nullptr, nullptr, lds, Hs, Ws};
    const int64_t cnt = pair_table_entries(Hr, Wr, n, m);
    const int64_t nthr = cnt > n ? cnt : n;
    hipLaunchKernelGGL(pair_table_kernel, dim3((unsigned)((nthr + 255) / 256)), dim3(256), 0, st, ips, prior, n, m, r,
                       Hs, Ws, Hr, Wr, jref, jsen, jobs, tiles, mask);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // configuration 1 (four workgroups per CU) where the parameters have it
    DescribeJob none{};
    return launch_describe_any(none, jobs, tiles, (int)cnt, mask, c, st, 1);
}

hipError_t launch_integral(double* i1, double* i2, int H, int W, double* agg, hipStream_t st, uint8_t* tmask) {
    const IntegJob J{i1, i2, agg, H, W};
    const IntegJob* none = nullptr;
    const int4* nit = nullptr;
    const int npre = (H + kScanNT - 1) / kScanNT + (W + kScanNT - 1) / kScanNT + 1;
    trace_begin(st, SFOC_K_INTEGRAL);
    hipLaunchKernelGGL(integral_prefix<false>, dim3(npre), dim3(kScanNT), 0, st, J, none, nit);
    hipLaunchKernelGGL(integral_tiles<false>, dim3((W + kTS - 1) / kTS, (H + kTS - 1) / kTS), dim3(kScanNT), 0, st,
                       J, none, nit, tmask);
    trace_end(st, SFOC_K_INTEGRAL);
    return hipGetLastError();
}

hipError_t launch_integral_batched(const IntegJob* jobs, const int4* pre, int npre, const int4* tiles, int ntiles,
                                   hipStream_t st) {
    if (npre == 0) return hipSuccess;
    const IntegJob none{};
    trace_begin(st, SFOC_K_INTEGRAL);
    hipLaunchKernelGGL(integral_prefix<true>, dim3(npre), dim3(kScanNT), 0, st, none, jobs, pre);
    hipLaunchKernelGGL(integral_tiles<true>, dim3(ntiles), dim3(kScanNT), 0, st, none, jobs, tiles,
                       (uint8_t*)nullptr);
    trace_end(st, SFOC_K_INTEGRAL);
    return hipGetLastError();
}

}  // namespace sfoc
