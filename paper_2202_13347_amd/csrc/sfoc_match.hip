// Fast-NCC_SFOC CP detection (Section 2.2, Eq. 9-16; Section 3.2.2) on gfx950.
//
// One workgroup per interest point.  For each descriptor channel h the
// template T_h (m x m, zero padded) and the search window S_h (M x M) get a
// real 2-D FFT of side L >= M, with the spectrum product F(S_h) conj(F(T_h))
// summed over channels in registers; summing in the spectrum is exact by
// linearity, so one inverse transform gives R_ST (Eq. 10, 13).
//
// Each length-L transform is a two-pass Cooley-Tukey with L = NA * NB:
//   pass A: a thread holds x[n1 + NB*n2], n2 = 0..NA-1, does an NA-point
//           DFT in registers and applies the twiddle W_L^(n1*k2);
//   pass B: a thread holds those results for two mirrored columns k2 and
//           NA - k2 and does NB-point DFTs, so it ends with the bins k and
//           L - k together.
// Rows of the window are real: two rows form one complex row, and the two
// half spectra are separated in the thread that holds k and L - k.  Of the
// column transforms, the DC and Nyquist columns (both real) are packed into
// one complex column and separated the same way.  The spectrum of T_h and
// the running sum over channels stay in registers; one LDS buffer of
// L x (L/2 + 1) complex values (padded) carries each 2-D transform.
//
// R_S and R_SS come from four lookups in the float64 integral images of the
// reference descriptor (Eq. 16); R_T and R_TT are accumulated in float64
// while the template is read.  NCC (Eq. 9) is assembled with the variance
// subtraction in float64, then the argmax, the parabola refinement and the
// per-CP flags are written.
#include "sfoc_dev.h"
#include "sfoc_launch.h"
#include "sfoc_trace.h"

namespace sfoc {

// Per-block flags of a split surface.
constexpr int kBlkNonflat = 1, kBlkNonfin = 2, kBlkFlatT = 4, kBlkBadT = 8, kBlkOOB = 16;

// Keeps the scheduler from moving work across stage boundaries (it would
// otherwise hoist the next stage's global loads and raise register pressure).
SFOC_DEV void stage_fence() { __builtin_amdgcn_sched_barrier(0); }
// The thread index laundered through an empty asm: index arithmetic derived
// from it is recomputed inside each stage instead of being hoisted out of
// the channel loop and kept live (which costs registers, then spills).
SFOC_DEV int tid_local() {
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

SFOC_DEV float2 cmul(float2 a, float2 b) { return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
SFOC_DEV float2 cmulc(float2 a, float2 b) {  // a * conj(b)
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
SFOC_DEV float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
// c ? a : b per component (a select of two array elements written this way
// stays in registers; as one conditional expression the compiler may turn
// it into a select of the arrays' addresses, which puts both in scratch).
SFOC_DEV float2 pick(bool c, float2 a, float2 b) { return make_float2(c ? a.x : b.x, c ? a.y : b.y); }
SFOC_DEV float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
SFOC_DEV float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
SFOC_DEV float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
SFOC_DEV float2 mul_mi(float2 a) { return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x); }

// Descriptor element of type DT (0 f32, 1 bf16, 2 f16) at p[i].
template <int DT>
SFOC_DEV float ldd(const void* p, int i) {
    if constexpr (DT == 0) return ((const float*)p)[i];
    else if constexpr (DT == 1) return bf16_bits_to_f32(((const uint16_t*)p)[i]);
    else return f16_bits_to_f32(((const uint16_t*)p)[i]);
}
template <int DT>
SFOC_DEV const void* elem_ptr(const void* base, int64_t idx) {
    return (const char*)base + idx * (DT == 0 ? 4 : 2);
}

// Orders one wave's LDS reads before its following writes.  Enough where
// every location a lane writes is read only by lanes of its own wave in the
// same round (the row-pair passes: a pair's tasks are consecutive lanes);
// LDS instructions of one wave execute in order.
SFOC_DEV void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Orders the reads of a row pair's tasks before their in-place writes.  A
// pair's TPP tasks are consecutive task indices; when TPP divides the wave
// size they are lanes of one wave and wave_sync suffices, otherwise a pair
// can straddle two waves and the whole workgroup synchronises (every
// thread runs the same number of rounds, so all of them reach it).
template <int TPP>
SFOC_DEV void pair_sync() {
    if constexpr (64 % TPP == 0) wave_sync();
    else __syncthreads();
}

// ---- small DFTs in registers -------------------------------------------
template <bool INV>
SFOC_DEV void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
    const float2 t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = mul_mi<INV>(csub(a1, a3));
    a0 = cadd(t0, t2);
    a2 = csub(t0, t2);
    a1 = cadd(t1, t3);
    a3 = csub(t1, t3);
}

// x[k] <- sum_n x[n] W_8^(nk), W_8 = exp(-+2 pi i / 8); 2 x 4 split.
template <bool INV>
SFOC_DEV void dft8(float2 (&x)[8]) {
    float2 a0 = x[0], a1 = x[2], a2 = x[4], a3 = x[6];
    float2 b0 = x[1], b1 = x[3], b2 = x[5], b3 = x[7];
    dft4<INV>(a0, a1, a2, a3);
    dft4<INV>(b0, b1, b2, b3);
    const float h = 0.70710678118654752f;
    const float sg = INV ? 1.f : -1.f;
    b1 = cmul(b1, make_float2(h, sg * h));
    b2 = mul_mi<INV>(b2);
    b3 = cmul(b3, make_float2(-h, sg * h));
    x[0] = cadd(a0, b0);
    x[4] = csub(a0, b0);
    x[1] = cadd(a1, b1);
    x[5] = csub(a1, b1);
    x[2] = cadd(a2, b2);
    x[6] = csub(a2, b2);
    x[3] = cadd(a3, b3);
    x[7] = csub(a3, b3);
}

// 16-point DFT, 4 x 4 split: n = n1 + 4 n2, k = 4 k1 + k2.
template <bool INV>
SFOC_DEV void dft16(float2 (&x)[16]) {
    const float sg = INV ? 1.f : -1.f;
    const float c1 = 0.92387953251128676f, s1 = 0.38268343236508977f, h = 0.70710678118654752f;
    // twiddles W_16^e for e = 0..9
    const float2 w[10] = {make_float2(1.f, 0.f),  make_float2(c1, sg * s1), make_float2(h, sg * h),
                          make_float2(s1, sg * c1), make_float2(0.f, sg * 1.f), make_float2(-s1, sg * c1),
                          make_float2(-h, sg * h), make_float2(-c1, sg * s1), make_float2(-1.f, 0.f),
                          make_float2(-c1, -sg * s1)};
    float2 y[4][4];
#pragma unroll
    for (int n1 = 0; n1 < 4; ++n1) {
        float2 a0 = x[n1], a1 = x[n1 + 4], a2 = x[n1 + 8], a3 = x[n1 + 12];
        dft4<INV>(a0, a1, a2, a3);
        y[n1][0] = a0;
        y[n1][1] = a1;
        y[n1][2] = a2;
        y[n1][3] = a3;
    }
#pragma unroll
    for (int n1 = 1; n1 < 4; ++n1)
#pragma unroll
        for (int k2 = 1; k2 < 4; ++k2) y[n1][k2] = cmul(y[n1][k2], w[n1 * k2]);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) {
        float2 a0 = y[0][k2], a1 = y[1][k2], a2 = y[2][k2], a3 = y[3][k2];
        dft4<INV>(a0, a1, a2, a3);
        x[k2] = a0;
        x[4 + k2] = a1;
        x[8 + k2] = a2;
        x[12 + k2] = a3;
    }
}

// 3-point DFT: with W = exp(-+2 pi i / 3) = -1/2 -+ i sqrt(3)/2,
// X1, X2 = a0 - (a1 + a2)/2 +- i s (a1 - a2), s = -+sqrt(3)/2.
template <bool INV>
SFOC_DEV void dft3(float2& a0, float2& a1, float2& a2) {
    const float s = (INV ? 1.f : -1.f) * 0.86602540378443865f;
    const float2 t1 = cadd(a1, a2), t2 = csub(a1, a2);
    const float2 m = make_float2(a0.x - 0.5f * t1.x, a0.y - 0.5f * t1.y);
    const float2 q = make_float2(-s * t2.y, s * t2.x);   // i s t2
    a0 = cadd(a0, t1);
    a1 = cadd(m, q);
    a2 = csub(m, q);
}

// 5-point DFT from the conjugate-symmetric pairs (a1, a4) and (a2, a3):
// with c_k = cos(2 pi k / 5), s_k = sin(2 pi k / 5) and sigma = -+1,
// X1,4 = a0 + c1 t1 + c2 t2 +- sigma i (s1 d1 + s2 d2),
// X2,3 = a0 + c2 t1 + c1 t2 +- sigma i (s2 d1 - s1 d2),
// t1 = a1 + a4, t2 = a2 + a3, d1 = a1 - a4, d2 = a2 - a3.
template <bool INV>
SFOC_DEV void dft5(float2 (&a)[5]) {
    const float sg = INV ? 1.f : -1.f;
    const float c1 = 0.30901699437494742f, c2 = -0.80901699437494742f;
    const float s1 = 0.95105651629515357f, s2 = 0.58778525229247313f;
    const float2 t1 = cadd(a[1], a[4]), t2 = cadd(a[2], a[3]);
    const float2 d1 = csub(a[1], a[4]), d2 = csub(a[2], a[3]);
    const float2 p1 = make_float2(a[0].x + c1 * t1.x + c2 * t2.x, a[0].y + c1 * t1.y + c2 * t2.y);
    const float2 p2 = make_float2(a[0].x + c2 * t1.x + c1 * t2.x, a[0].y + c2 * t1.y + c1 * t2.y);
    const float2 e1 = make_float2(s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y);
    const float2 e2 = make_float2(s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y);
    const float2 q1 = make_float2(-sg * e1.y, sg * e1.x);   // sigma i e1
    const float2 q2 = make_float2(-sg * e2.y, sg * e2.x);
    a[0] = cadd(a[0], cadd(t1, t2));
    a[1] = cadd(p1, q1);
    a[4] = csub(p1, q1);
    a[2] = cadd(p2, q2);
    a[3] = csub(p2, q2);
}

// 10-point DFT, 2 x 5: the even and odd samples each get a 5-point DFT,
// the odd ones then W_10^k, and X[k], X[k+5] = E[k] +- W_10^k O[k].
template <bool INV>
SFOC_DEV void dft10(float2 (&x)[10]) {
    const float sg = INV ? 1.f : -1.f;
    float2 e[5], o[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        e[k] = x[2 * k];
        o[k] = x[2 * k + 1];
    }
    dft5<INV>(e);
    dft5<INV>(o);
    // W_10^k = cos(pi k / 5) + sigma i sin(pi k / 5), k = 1..4
    const float ca = 0.80901699437494742f, sa = 0.58778525229247313f;   // 36 degrees
    const float cb = 0.30901699437494742f, sb = 0.95105651629515357f;   // 72 degrees
    o[1] = cmul(o[1], make_float2(ca, sg * sa));
    o[2] = cmul(o[2], make_float2(cb, sg * sb));
    o[3] = cmul(o[3], make_float2(-cb, sg * sb));
    o[4] = cmul(o[4], make_float2(-ca, sg * sa));
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        x[k] = cadd(e[k], o[k]);
        x[k + 5] = csub(e[k], o[k]);
    }
}

// 12-point DFT, 3 x 4: n = n1 + 3 n2, k = 4 k1 + k2; 4-point DFTs over n2,
// twiddles W_12^(n1 k2), 3-point DFTs over n1.
template <bool INV>
SFOC_DEV void dft12(float2 (&x)[12]) {
    const float sg = INV ? 1.f : -1.f;
    const float h = 0.86602540378443865f;   // cos 30 degrees
    float2 y[3][4];
#pragma unroll
    for (int n1 = 0; n1 < 3; ++n1) {
        float2 a0 = x[n1], a1 = x[n1 + 3], a2 = x[n1 + 6], a3 = x[n1 + 9];
        dft4<INV>(a0, a1, a2, a3);
        y[n1][0] = a0;
        y[n1][1] = a1;
        y[n1][2] = a2;
        y[n1][3] = a3;
    }
    // W_12^e, e = n1 k2 in 1..6: angles 30 e degrees
    const float2 w[7] = {make_float2(1.f, 0.f),     make_float2(h, sg * 0.5f), make_float2(0.5f, sg * h),
                         make_float2(0.f, sg * 1.f), make_float2(-0.5f, sg * h), make_float2(-h, sg * 0.5f),
                         make_float2(-1.f, 0.f)};
#pragma unroll
    for (int n1 = 1; n1 < 3; ++n1)
#pragma unroll
        for (int k2 = 1; k2 < 4; ++k2) y[n1][k2] = cmul(y[n1][k2], w[n1 * k2]);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) {
        float2 a0 = y[0][k2], a1 = y[1][k2], a2 = y[2][k2];
        dft3<INV>(a0, a1, a2);
        x[k2] = a0;
        x[4 + k2] = a1;
        x[8 + k2] = a2;
    }
}

template <int N, bool INV>
SFOC_DEV void dftn(float2 (&x)[N]) {
    if constexpr (N == 8) dft8<INV>(x);
    else if constexpr (N == 10) dft10<INV>(x);
    else if constexpr (N == 12) dft12<INV>(x);
    else dft16<INV>(x);
}

// ---- geometry ----------------------------------------------------------
// A side L = NA * NB transform: pass A are NA-point DFTs, pass B NB-point
// ones.  NT threads per workgroup and MINB workgroups per CU (the LDS
// buffer of the larger sides leaves room for one); the kernels' launch
// bounds ask for the waves per SIMD that MINB workgroups need, which caps
// their registers accordingly.
template <int L>
struct Fft;
// LDS layout of the transform buffer: row r starts at r * PITCH + (r / NB) *
// SKEW complex values.  The column passes read rows n1 + NB k (k across the
// lanes of a wave, or across the loop), whose starts would otherwise fall on
// the same LDS banks; the pitch and the per-group skew spread both kinds of
// access over all banks, and keep each row (and each row pair) contiguous.
template <>
struct Fft<128> {
    static constexpr int NA = 16, NB = 8, NT = 512, PITCH = 68, SKEW = 8, MINB = 2;
};
template <>
struct Fft<64> {
    static constexpr int NA = 8, NB = 8, NT = 128, PITCH = 40, SKEW = 8, MINB = 7;
};
template <>
struct Fft<160> {
    static constexpr int NA = 16, NB = 10, NT = 640, PITCH = 84, SKEW = 8, MINB = 1;
};
template <>
struct Fft<192> {
    static constexpr int NA = 16, NB = 12, NT = 768, PITCH = 100, SKEW = 8, MINB = 1;
};

template <int L>
struct MatchCfg {
    using F = Fft<L>;
    static constexpr int NA = F::NA, NB = F::NB, NT = F::NT, P = F::PITCH, SKEW = F::SKEW, MINB = F::MINB;
    static constexpr int WAVES_PER_SIMD = (MINB * NT + 255) / 256;   // 4 SIMDs of 64 lanes per CU
    static constexpr int HA = NA / 2;
    static constexpr int COLS = L / 2;                     // column transforms (DC+Nyquist packed)
    static constexpr int RB = COLS * HA / NT;              // pass-B tasks per thread
    static constexpr int BINS = 2 * NB;                    // bins per pass-B task
    // Two tasks' loads in flight in the search window's stages where a
    // thread has at least two tasks per stage (L / 2 row pairs or columns
    // of NB tasks each) and the registers allow it (side 64).
    static constexpr bool PIPE = L * NB / 2 >= 2 * NT && L <= 128;
    static_assert(L == NA * NB && NB % 2 == 0 && NA % 2 == 0, "even radices");
    static_assert(COLS * HA % NT == 0, "whole pass-B rounds");
    static_assert(2 * P >= L, "a row pair holds one real row of L values per row");
    static constexpr size_t buf_elems = (size_t)L * P + (size_t)(L / NB) * SKEW;   // complex
    static SFOC_DEV int row(int r) { return r * P + (r / NB) * SKEW; }
    // row n1 + NB * k with n1 < NB: its NB-row group is k
    static SFOC_DEV int rowg(int n1, int k) { return n1 * P + k * (NB * P + SKEW); }
    // Slot of element n1 of pass-A output column k2 inside a row pair: a
    // permutation of n1 that differs between columns (bank spreading).
    static SFOC_DEV int swz(int n1, int k2) {
        if constexpr ((NB & (NB - 1)) == 0) return n1 ^ (k2 & (NB - 1));
        else return (n1 + k2) % NB;
    }
    static constexpr size_t lds_bytes = sizeof(float2) * (buf_elems + L) + 1024;
};

// Bin index (within the transform) of value q of a pass-B task with j.
template <int L>
SFOC_DEV int bin_of(int j, int q) {
    using C = MatchCfg<L>;
    const int k1 = q % C::NB;
    const int kk = q < C::NB ? j : (j == 0 ? C::HA : C::NA - j);
    return C::NA * k1 + kk;
}
// Packed DC / Nyquist column (C = F_dc + i F_nyq, both Hermitian): replace
// each mirrored pair of slots (k, L-k) by (F_dc[k], F_nyq[k]).  Self-mirrored
// slots (k = 0, L/2) already hold (F_dc, F_nyq) as (re, im).
SFOC_DEV void sep_pair(float2& x, float2& y) {
    const float2 a = x, b = cconj(y);
    x = cscale(cadd(a, b), 0.5f);
    y = cscale(mul_mi<false>(csub(a, b)), 0.5f);
}
template <int NB>
SFOC_DEV void separate_packed(float2 (&u)[NB], float2 (&v)[NB], int j) {
    if (j == 0) {
#pragma unroll
        for (int k1 = 1; k1 < NB / 2; ++k1) sep_pair(u[k1], u[NB - k1]);
#pragma unroll
        for (int k1 = 0; k1 < NB / 2; ++k1) sep_pair(v[k1], v[NB - 1 - k1]);
    } else {
#pragma unroll
        for (int k1 = 0; k1 < NB; ++k1) sep_pair(u[k1], v[NB - 1 - k1]);
    }
}
// Inverse of the above on the accumulated products (Q_dc, Q_nyq) -> the
// packed spectrum P = Q_dc + i Q_nyq at both bins of each pair.
SFOC_DEV void join_pair(float2& x, float2& y) {
    const float2 q0 = x, qn = y;
    x = make_float2(q0.x - qn.y, q0.y + qn.x);
    y = make_float2(q0.x + qn.y, -q0.y + qn.x);
}
template <int NB>
SFOC_DEV void join_packed(float2 (&u)[NB], float2 (&v)[NB], int j) {
    if (j == 0) {
#pragma unroll
        for (int k1 = 1; k1 < NB / 2; ++k1) join_pair(u[k1], u[NB - k1]);
#pragma unroll
        for (int k1 = 0; k1 < NB / 2; ++k1) join_pair(v[k1], v[NB - 1 - k1]);
    } else {
#pragma unroll
        for (int k1 = 0; k1 < NB; ++k1) join_pair(u[k1], v[NB - 1 - k1]);
    }
}

// ---- row stage: real rows -> half spectra -------------------------------
// Rows [0, nrows) x columns [0, ncols) of one descriptor plane, zero padded
// to L; result: buf row a holds the half spectrum (bins 0..L/2) of row a.
// s1 / s2 (if given) accumulate the sum and sum of squares of the values.
template <int L, int DT, bool PIPE>
SFOC_DEV void row_stage(const void* plane, int pitch, int y0, int x0, int nrows, int ncols, float2* buf,
                        const float2* tw, double* s1, double* s2) {
    using C = MatchCfg<L>;
    const int tid = tid_local();
    const int npair = (nrows + 1) / 2;
    const int tasksA = npair * C::NB;
    // Loads from one pointer per row and task (32-bit offsets from the plane
    // base: a plane holds < 2^30 elements); element n2 lies NB * n2 elements
    // further on, a constant offset the load instruction encodes, so the
    // loads need no per-element address arithmetic.  The window lies inside
    // the image; a missing second row re-reads the first (then zeroed).
    // Full-width windows (ncols == L) need no column test; narrower ones load
    // only the columns below ncols and zero the rest.
    const bool full = ncols == L;
    auto load = [&](int task, float2(&x)[C::NA]) {
        const int p = task / C::NB, n1 = task - p * C::NB;
        const bool two = 2 * p + 1 < nrows;
        const int oa = (y0 + 2 * p) * pitch + x0 + n1;
        const int ob = oa + (two ? pitch : 0);
        const void* ra = elem_ptr<DT>(plane, oa);
        const void* rb = elem_ptr<DT>(plane, ob);
        if (full) {
#pragma unroll
            for (int n2 = 0; n2 < C::NA; ++n2) {
                const float re = ldd<DT>(ra, C::NB * n2), im = ldd<DT>(rb, C::NB * n2);
                x[n2] = make_float2(re, two ? im : 0.f);
            }
        } else {
#pragma unroll
            for (int n2 = 0; n2 < C::NA; ++n2) {
                float re = 0.f, im = 0.f;
                if (n1 + C::NB * n2 < ncols) {
                    re = ldd<DT>(ra, C::NB * n2);
                    im = ldd<DT>(rb, C::NB * n2);
                }
                x[n2] = make_float2(re, two ? im : 0.f);
            }
        }
    };
    auto finish = [&](int task, float2(&x)[C::NA]) {
        const int p = task / C::NB, n1 = task - p * C::NB;
        if (s1) {
            double a = 0.0, q = 0.0;
#pragma unroll
            for (int n2 = 0; n2 < C::NA; ++n2) {
                const double dr = x[n2].x, di = x[n2].y;
                a += dr + di;
                q += dr * dr + di * di;
            }
            *s1 += a;
            *s2 += q;
        }
        dftn<C::NA, false>(x);
        float2* reg = buf + C::row(2 * p);
#pragma unroll
        for (int k2 = 0; k2 < C::NA; ++k2)
            reg[k2 * C::NB + C::swz(n1, k2)] = k2 == 0 ? x[0] : cmul(x[k2], tw[n1 * k2]);
    };
    if (PIPE) {
        // Two tasks per iteration with both tasks' loads issued first.
#pragma unroll 1
        for (int task = tid; task < tasksA; task += 2 * C::NT) {
            float2 xa[C::NA], xb[C::NA];
            const bool second = task + C::NT < tasksA;
            load(task, xa);
            if (second) load(task + C::NT, xb);
            finish(task, xa);
            if (second) finish(task + C::NT, xb);
        }
    } else {
#pragma unroll 1
        for (int task = tid; task < tasksA; task += C::NT) {
            float2 x[C::NA];
            load(task, x);
            finish(task, x);
        }
    }
    __syncthreads();
    const int tasksB = npair * C::HA;
    const int rounds = (tasksB + C::NT - 1) / C::NT;
#pragma unroll 1
    for (int rd = 0; rd < rounds; ++rd) {
        const int task = rd * C::NT + tid;
        const bool act = task < tasksB;
        const int p = task / C::HA, j = task - p * C::HA;
        float2 u[C::NB], v[C::NB];
        float2* reg = buf + C::row(2 * p);
        if (act) {
            const int ka = j, kb = j == 0 ? C::HA : C::NA - j;
#pragma unroll
            for (int n1 = 0; n1 < C::NB; ++n1) {
                u[n1] = reg[ka * C::NB + C::swz(n1, ka)];
                v[n1] = reg[kb * C::NB + C::swz(n1, kb)];
            }
            dftn<C::NB, false>(u);
            dftn<C::NB, false>(v);
        }
        pair_sync<C::HA>();   // this pair's reads before its in-place writes
        if (act) {
            // half spectra of the two real rows: A = (X + conj X~)/2, B = -i (X - conj X~)/2
            float2* ra = buf + C::row(2 * p);
            float2* rb = ra + C::P;
            const int ka = j, kb = j == 0 ? C::HA : C::NA - j;
#pragma unroll
            for (int k1 = 0; k1 <= C::NB / 2; ++k1) {
                if (k1 < C::NB / 2 || j == 0) {
                    const float2 za = u[k1];
                    const float2 zb = cconj(pick(j == 0, u[(C::NB - k1) % C::NB], v[C::NB - 1 - k1]));
                    const int k = C::NA * k1 + ka;
                    ra[k] = cscale(cadd(za, zb), 0.5f);
                    rb[k] = cscale(mul_mi<false>(csub(za, zb)), 0.5f);
                }
            }
#pragma unroll
            for (int k1 = 0; k1 < C::NB / 2; ++k1) {
                const float2 za = v[k1];
                const float2 zb = cconj(pick(j == 0, v[C::NB - 1 - k1], u[C::NB - 1 - k1]));
                const int k = C::NA * k1 + kb;
                ra[k] = cscale(cadd(za, zb), 0.5f);
                rb[k] = cscale(mul_mi<false>(csub(za, zb)), 0.5f);
            }
        }
    }
    __syncthreads();
}

// ---- column stage: buf columns -> spectrum bins in registers --------------
// Column transforms over rows 0..L-1 of columns 1..L/2-1 and of the packed
// column 0 (forward: DC + i Nyquist taken from columns 0 and L/2; inverse:
// column 0 as stored).  Rows >= nvalid read as zero.  out[rd][q] receives
// bin bin_of(j, q) of task rd (column cc = task / HA, j = task % HA):
// sink(rd, cc, j, u, v) gets values q < NB in u and q >= NB in v (writable).
template <int L, bool INV, bool PIPE, typename Sink>
SFOC_DEV void col_stage(float2* buf, const float2* tw, int nvalid, Sink&& sink) {
    using C = MatchCfg<L>;
    const int tid = tid_local();
    // task (cc, n1) reads and rewrites rows n1 + NB m of column cc only
    auto load = [&](int task, float2(&x)[C::NA]) {
        const int cc = task / C::NB, n1 = task - cc * C::NB;
#pragma unroll
        for (int n2 = 0; n2 < C::NA; ++n2) {
            const int row = n1 + C::NB * n2;
            float2 v = make_float2(0.f, 0.f);
            if (row < nvalid) {
                if (cc == 0 && !INV) v = make_float2(buf[C::rowg(n1, n2)].x, buf[C::rowg(n1, n2) + L / 2].x);
                else v = buf[C::rowg(n1, n2) + cc];
            }
            x[n2] = v;
        }
    };
    auto finish = [&](int task, float2(&x)[C::NA]) {
        const int cc = task / C::NB, n1 = task - cc * C::NB;
        dftn<C::NA, INV>(x);
#pragma unroll
        for (int k2 = 0; k2 < C::NA; ++k2) {
            float2 w = tw[n1 * k2];
            if (INV) w.y = -w.y;
            buf[C::rowg(n1, k2) + cc] = k2 == 0 ? x[0] : cmul(x[k2], w);
        }
    };
    if (PIPE) {   // two tasks per iteration, both tasks' reads first
#pragma unroll 1
        for (int task = tid; task < C::COLS * C::NB; task += 2 * C::NT) {
            float2 xa[C::NA], xb[C::NA];
            const bool second = task + C::NT < C::COLS * C::NB;
            load(task, xa);
            if (second) load(task + C::NT, xb);
            finish(task, xa);
            if (second) finish(task + C::NT, xb);
        }
    } else {
#pragma unroll 1
        for (int task = tid; task < C::COLS * C::NB; task += C::NT) {
            float2 x[C::NA];
            load(task, x);
            finish(task, x);
        }
    }
    __syncthreads();
#pragma unroll
    for (int rd = 0; rd < C::RB; ++rd) {
        const int task = rd * C::NT + tid;
        const int cc = task / C::HA, j = task - cc * C::HA;
        const int ka = j, kb = j == 0 ? C::HA : C::NA - j;
        float2 u[C::NB], v[C::NB];
#pragma unroll
        for (int n1 = 0; n1 < C::NB; ++n1) {
            u[n1] = buf[C::rowg(n1, ka) + cc];
            v[n1] = buf[C::rowg(n1, kb) + cc];
        }
        dftn<C::NB, INV>(u);
        dftn<C::NB, INV>(v);
        sink(rd, cc, j, u, v);
    }
}

SFOC_DEV bool in_image(int64_t y, int64_t x, int h, int w, int64_t H, int64_t W) {
    return y >= 0 && x >= 0 && y + h <= H && x + w <= W;
}

// Twiddles W_L^k, k < L, into LDS (once per workgroup).
template <int L>
SFOC_DEV void init_twiddles(float2* tw) {
    for (int k = threadIdx.x; k < L; k += MatchCfg<L>::NT) {
        float sn, cs;
        sincospif(-2.0f * (float)k / (float)L, &sn, &cs);
        tw[k] = make_float2(cs, sn);
    }
}

// Template sums R_T, R_TT (Eq. 12): a block reduction in float64 of every
// thread's partial sums, left in red[64] and red[65] (red holds at least 66
// doubles); returns with the workgroup synchronised.
template <int NT>
SFOC_DEV void block_sum2(double s1, double s2, double* red) {
    const int t = threadIdx.x;
    const int lane = t & 63, wv = t >> 6;
    for (int d = 32; d >= 1; d >>= 1) {
        s1 += __shfl_down(s1, d, 64);
        s2 += __shfl_down(s2, d, 64);
    }
    if (lane == 0) {
        red[2 * wv] = s1;
        red[2 * wv + 1] = s2;
    }
    __syncthreads();
    if (t == 0) {
        double a = 0.0, b = 0.0;
        for (int w = 0; w < NT / 64; ++w) {
            a += red[2 * w];
            b += red[2 * w + 1];
        }
        red[64] = a;
        red[65] = b;
    }
    __syncthreads();
}

// NCC (Eq. 9), the argmax, the parabola refinement and the CP record of one
// work item, from its correlation surface R_ST: rst_at(u, v) for offsets
// (u, v) of the block [u0, u0 + Vu) x [v0, v0 + Vv), readable by every
// thread.  RT, RTT are the template sums; red is workgroup scratch of at
// least 66 doubles.  Every thread of the workgroup calls it.
template <int NT, typename Rst>
SFOC_DEV void ncc_peak(const MatchArgs& A, int i, int slot, int u0, int v0, int Vu, int Vv, double RT, double RTT,
                       double* red, Rst rst_at) {
    const int nblk = A.nbu * A.nbv;
    const int t = threadIdx.x;
    const int m = A.m, r = A.r, M = m + 2 * r, V = 2 * r + 1;
    const int py = A.ips[2 * i], px = A.ips[2 * i + 1];
    const int pry = A.prior ? A.prior[2 * i] : 0, prx = A.prior ? A.prior[2 * i + 1] : 0;
    const int64_t sy = (int64_t)py - m / 2 - r + pry, sx = (int64_t)px - m / 2 - r + prx;
    float* nout = A.ncc ? A.ncc + (int64_t)i * V * V : (nblk > 1 ? A.surf + (int64_t)i * V * V : nullptr);
    sfoc_cp out;
    out.sen_row = py;
    out.sen_col = px;
    out.dy = out.dx = 0;
    out.sub_dy = out.sub_dx = 0.f;
    out.score = 0.f;
    out.flags = 0;
    const double mnz = (double)m * m * A.z;
    const double tau = 1e-12 * mnz;
    const double varT = RTT - RT * RT / mnz;
    // NCC (Eq. 9) with integral-image box sums (Eq. 16), float64 variance.
    // The integral images are the reference image's, or this IP's own over
    // its search window (origin (sy, sx), side M + 1).
    const int64_t IW = A.integ_win ? (int64_t)M + 1 : A.Wr + 1;
    const double* __restrict__ I1 = A.integ_win ? A.integ1 + (int64_t)i * IW * IW : A.integ1;
    const double* __restrict__ I2 = A.integ_win ? A.integ2 + (int64_t)i * IW * IW : A.integ2;
    const int64_t oy = A.integ_win ? 0 : sy, ox = A.integ_win ? 0 : sx;
    const bool flatT = !(varT > tau);
    const bool badT = !isfinite(RT) || !isfinite(RTT);
    // NCC at offset (u, v); flags: bit 0 non-flat search window, bit 1 non-finite.
    // (u, v) are offsets within this block; the surface offset is (u0 + u, v0 + v).
    auto ncc_at = [&](int u, int v, int& fl) -> float {
        const float rst = rst_at(u, v);
        const int64_t y = oy + u0 + u, x = ox + v0 + v;
        const int64_t a00 = y * IW + x, a01 = a00 + m, a10 = a00 + (int64_t)m * IW, a11 = a10 + m;
        const double RS = I1[a11] - I1[a10] - I1[a01] + I1[a00];
        const double RSS = I2[a11] - I2[a10] - I2[a01] + I2[a00];
        const double varS = RSS - RS * RS / mnz;
        float val = 0.f;
        fl = 0;
        if (!isfinite(rst) || !isfinite(RS) || !isfinite(varS)) fl |= 2;
        if (varS > tau && !flatT) {
            fl |= 1;
            const double num = (double)rst - RS * RT / mnz;
            val = (float)(num / sqrt(varS * varT));
        }
        return val;
    };
    int nonflat = 0, nonfin = 0;
    float best = -INFINITY;
    int bidx = 0x7fffffff;
    for (int e = t; e < Vu * Vv; e += NT) {
        const int u = e / Vv, v = e - u * Vv;
        int fl;
        const float val = ncc_at(u, v, fl);
        nonflat |= fl & 1;
        nonfin |= fl >> 1;
        const int eg = (u0 + u) * V + v0 + v;   // row-major index on the whole surface
        if (nout) nout[eg] = val;
        if (val > best) {   // strictly greater: the first index wins ties
            best = val;
            bidx = eg;
        }
    }
    // block reduce (max value, min index), and the flags.
    {
        const int lane = t & 63, wv = t >> 6;
        for (int d = 32; d >= 1; d >>= 1) {
            const float ob = __shfl_down(best, d, 64);
            const int oi = __shfl_down(bidx, d, 64);
            if (ob > best || (ob == best && oi < bidx)) {
                best = ob;
                bidx = oi;
            }
            nonflat |= __shfl_down(nonflat, d, 64);
            nonfin |= __shfl_down(nonfin, d, 64);
        }
        __syncthreads();
        float* rf = reinterpret_cast<float*>(red);
        int* ri = reinterpret_cast<int*>(red) + 64;
        if (lane == 0) {
            rf[wv] = best;
            ri[wv] = bidx;
            ri[16 + wv] = nonflat;
            ri[32 + wv] = nonfin;
        }
        __syncthreads();
        if (t == 0) {
            for (int w = 1; w < NT / 64; ++w) {
                if (rf[w] > rf[0] || (rf[w] == rf[0] && ri[w] < ri[0])) {
                    rf[0] = rf[w];
                    ri[0] = ri[w];
                }
                ri[16] |= ri[16 + w];
                ri[32] |= ri[32 + w];
            }
        }
        __syncthreads();
        best = rf[0];
        bidx = ri[0];
        nonflat = ri[16];
        nonfin = ri[32];
    }
    if (nblk > 1) {
        if (t == 0) {
            const int fl = (nonflat ? kBlkNonflat : 0) | (nonfin ? kBlkNonfin : 0) | (flatT ? kBlkFlatT : 0) |
                           (badT ? kBlkBadT : 0);
            A.blk[slot] = make_float4(best, __int_as_float(bidx), __int_as_float(fl), 0.f);
        }
        return;
    }
    if (t == 0) {
        if (badT || (nonfin && !flatT)) {
            out.flags = SFOC_CP_NONFINITE;
        } else if (flatT) {
            out.flags = SFOC_CP_FLAT_T;
        } else if (!nonflat || bidx >= V * V) {
            out.flags = SFOC_CP_FLAT_S;
        } else {
            const int u = bidx / V, v = bidx - u * V;
            out.dy = u - r;
            out.dx = v - r;
            out.score = best;
            if (u == 0 || v == 0 || u == V - 1 || v == V - 1) {
                out.flags = SFOC_CP_EDGE_PEAK;
            } else {
                int fl;
                const float c0 = best;
                const float cu = ncc_at(u - 1, v, fl), cd = ncc_at(u + 1, v, fl);
                const float cl = ncc_at(u, v - 1, fl), cr = ncc_at(u, v + 1, fl);
                float den = cu - 2.f * c0 + cd;
                float d = 0.f;
                if (den < 0.f) d = fminf(0.5f, fmaxf(-0.5f, (cu - cd) / (2.f * den)));
                out.sub_dy = d;
                den = cl - 2.f * c0 + cr;
                d = 0.f;
                if (den < 0.f) d = fminf(0.5f, fmaxf(-0.5f, (cl - cr) / (2.f * den)));
                out.sub_dx = d;
            }
        }
        A.cps[i] = out;
    }
}

// One work item: interest point i, offset block bq (record slot `slot`).
// With M <= L there is one block and this workgroup finishes the CP;
// otherwise each block covers offsets [u0, u0 + Vu) x [v0, v0 + Vv) with a
// search window of (m + Vu - 1) x (m + Vv - 1) <= L x L, writes its part of
// the surface and its best score, and peak_kernel combines the blocks.
// Every thread of the workgroup calls it with the same item; it returns
// with the workgroup synchronised.
template <int L, int DT, bool SPLIT = false>
SFOC_DEV void match_item(const MatchArgs& A, int i, int bq, int slot, const float2* tw, float2* buf, double* red) {
    using C = MatchCfg<L>;
    const int nblk = A.nbu * A.nbv;
    const int bu = bq / A.nbv, bv = bq - bu * A.nbv;
    const int t = threadIdx.x;
    const int m = A.m, r = A.r, M = m + 2 * r, V = 2 * r + 1;
    const int u0 = bu * A.Vb, v0 = bv * A.Vb;
    const int Vu = min(A.Vb, V - u0), Vv = min(A.Vb, V - v0);
    const int Mu = m + Vu - 1, Mv = m + Vv - 1;
    const int py = A.ips[2 * i], px = A.ips[2 * i + 1];
    const int pry = A.prior ? A.prior[2 * i] : 0, prx = A.prior ? A.prior[2 * i + 1] : 0;
    const int64_t ty = (int64_t)py - m / 2, tx = (int64_t)px - m / 2;
    const int64_t sy = ty - r + pry, sx = tx - r + prx;
    float* nout = A.ncc ? A.ncc + (int64_t)i * V * V : (nblk > 1 ? A.surf + (int64_t)i * V * V : nullptr);
    sfoc_cp out;
    out.sen_row = py;
    out.sen_col = px;
    out.dy = out.dx = 0;
    out.sub_dy = out.sub_dx = 0.f;
    out.score = 0.f;
    out.flags = 0;
    if (!in_image(ty, tx, m, m, A.Hs, A.Ws) || !in_image(sy, sx, M, M, A.Hr, A.Wr)) {
        if (t == 0) {
            if (nblk == 1) {
                out.flags = SFOC_CP_OOB;
                A.cps[i] = out;
            } else {
                A.blk[slot] = make_float4(0.f, __int_as_float(0), __int_as_float(kBlkOOB), 0.f);
            }
        }
        if (nout)
            for (int e = t; e < Vu * Vv; e += C::NT) {
                const int u = e / Vv, v = e - u * Vv;
                nout[(u0 + u) * V + v0 + v] = 0.f;
            }
        return;
    }

    float2 acc[C::RB][C::BINS];   // sum over channels of F(S_h) conj(F(T_h))
#pragma unroll
    for (int rd = 0; rd < C::RB; ++rd)
#pragma unroll
        for (int q = 0; q < C::BINS; ++q) acc[rd][q] = make_float2(0.f, 0.f);
    double s1 = 0.0, s2 = 0.0;
    const int64_t plane_s = A.Hs * A.Ws, plane_r = A.Hr * A.Wr;
    const int mpair2 = 2 * ((m + 1) / 2), Mpair2 = 2 * ((Mu + 1) / 2);
    // Per channel: the search window first (only the running sum is live
    // during its larger row stage), its spectrum kept in registers, then the
    // template, whose column stage accumulates F(S_h) conj(F(T_h)).
    float2 xsp[C::RB][C::BINS];   // search-window spectrum of the current channel
    for (int h = 0; h < A.z; ++h) {
        stage_fence();
        row_stage<L, DT, C::PIPE>(elem_ptr<DT>(A.desc_ref, h * plane_r), (int)A.Wr, (int)(sy + u0), (int)(sx + v0), Mu, Mv,
                         buf, tw, nullptr, nullptr);
        stage_fence();
        col_stage<L, false, C::PIPE>(buf, tw, Mpair2, [&](int rd, int cc, int j, float2(&u)[C::NB], float2(&v)[C::NB]) {
            if (cc == 0) separate_packed<C::NB>(u, v, j);
#pragma unroll
            for (int q = 0; q < C::NB; ++q) {
                xsp[rd][q] = u[q];
                xsp[rd][C::NB + q] = v[q];
            }
        });
        __syncthreads();
        stage_fence();
        row_stage<L, DT, false>(elem_ptr<DT>(A.desc_sen, h * plane_s), (int)A.Ws, (int)ty, (int)tx, m, m, buf, tw, &s1, &s2);
        stage_fence();
        col_stage<L, false, false>(buf, tw, mpair2, [&](int rd, int cc, int j, float2(&u)[C::NB], float2(&v)[C::NB]) {
            if (cc == 0) separate_packed<C::NB>(u, v, j);
            const bool self = cc == 0 && j == 0;   // slots 0 and NB/2 hold (F_dc, F_nyq) as reals
#pragma unroll
            for (int q = 0; q < C::BINS; ++q) {
                const float2 xs = xsp[rd][q];
                const float2 yt = q < C::NB ? u[q] : v[q - C::NB];
                if ((q == 0 || q == C::NB / 2) && self)
                    acc[rd][q] = make_float2(fmaf(xs.x, yt.x, acc[rd][q].x), fmaf(xs.y, yt.y, acc[rd][q].y));
                else
                    acc[rd][q] = cadd(acc[rd][q], cmulc(xs, yt));
            }
        });
        __syncthreads();
    }

    block_sum2<C::NT>(s1, s2, red);

    // inverse, columns first: spectrum bins back to LDS (natural order), then
    // column transforms k1 -> u.
#pragma unroll
    for (int rd = 0; rd < C::RB; ++rd) {
        const int task = rd * C::NT + t;
        const int cc = task / C::HA, j = task - cc * C::HA;
        if (cc == 0) {
            float2 u[C::NB], v[C::NB];
#pragma unroll
            for (int q = 0; q < C::NB; ++q) {
                u[q] = acc[rd][q];
                v[q] = acc[rd][C::NB + q];
            }
            join_packed<C::NB>(u, v, j);
#pragma unroll
            for (int q = 0; q < C::NB; ++q) {
                acc[rd][q] = u[q];
                acc[rd][C::NB + q] = v[q];
            }
        }
#pragma unroll
        for (int q = 0; q < C::BINS; ++q) buf[C::row(bin_of<L>(j, q)) + cc] = acc[rd][q];
    }
    __syncthreads();
    {
        float2 zc[C::RB][C::BINS];
        col_stage<L, true, C::PIPE>(buf, tw, L, [&](int rd, int, int, float2(&u)[C::NB], float2(&v)[C::NB]) {
#pragma unroll
            for (int q = 0; q < C::NB; ++q) {
                zc[rd][q] = u[q];
                zc[rd][C::NB + q] = v[q];
            }
        });
        __syncthreads();
#pragma unroll
        for (int rd = 0; rd < C::RB; ++rd) {
            const int task = rd * C::NT + t;
            const int cc = task / C::HA, j = task - cc * C::HA;
#pragma unroll
            for (int q = 0; q < C::BINS; ++q) {
                const int u = bin_of<L>(j, q);
                if (u < Vu) buf[C::row(u) + cc] = zc[rd][q];
            }
        }
    }
    __syncthreads();
    // rows: pairs (u, u+1) of Hermitian half spectra -> one complex inverse;
    // real part row u, imaginary part row u+1.
    const int vpair = (Vu + 1) / 2;
    {
        const int tasksA = vpair * C::NB;
        const int rounds = (tasksA + C::NT - 1) / C::NT;
        for (int rd = 0; rd < rounds; ++rd) {
            const int task = rd * C::NT + t;
            const bool act = task < tasksA;
            const int p = task / C::NB, n1 = task - p * C::NB;
            float2 x[C::NA];
            if (act) {
                const float2* ra = buf + C::row(2 * p);
                const float2* rb = ra + C::P;
#pragma unroll
                for (int n2 = 0; n2 < C::NA; ++n2) {
                    const int k2 = n1 + C::NB * n2;
                    float2 ha, hb;
                    if (k2 == 0) {
                        ha = make_float2(ra[0].x, 0.f);
                        hb = make_float2(rb[0].x, 0.f);
                    } else if (k2 == L / 2) {
                        ha = make_float2(ra[0].y, 0.f);
                        hb = make_float2(rb[0].y, 0.f);
                    } else if (k2 < L / 2) {
                        ha = ra[k2];
                        hb = rb[k2];
                    } else {
                        ha = cconj(ra[L - k2]);
                        hb = cconj(rb[L - k2]);
                    }
                    x[n2] = make_float2(ha.x - hb.y, ha.y + hb.x);
                }
                dftn<C::NA, true>(x);
            }
            pair_sync<C::NB>();   // this pair's reads before its in-place writes
            if (act) {
                float2* reg = buf + C::row(2 * p);
#pragma unroll
                for (int k2 = 0; k2 < C::NA; ++k2)
                    reg[k2 * C::NB + C::swz(n1, k2)] = k2 == 0 ? x[0] : cmul(x[k2], cconj(tw[n1 * k2]));
            }
        }
        __syncthreads();
        const float inv = 1.0f / ((float)L * (float)L);
        const int tasksB = vpair * C::HA;
        const int roundsB = (tasksB + C::NT - 1) / C::NT;
        for (int rd = 0; rd < roundsB; ++rd) {
            const int task = rd * C::NT + t;
            const bool act = task < tasksB;
            const int p = task / C::HA, j = task - p * C::HA;
            float2 u[C::NB], v[C::NB];
            float2* reg = buf + C::row(2 * p);
            const int ka = j, kb = j == 0 ? C::HA : C::NA - j;
            if (act) {
#pragma unroll
                for (int n1 = 0; n1 < C::NB; ++n1) {
                    u[n1] = reg[ka * C::NB + C::swz(n1, ka)];
                    v[n1] = reg[kb * C::NB + C::swz(n1, kb)];
                }
                dftn<C::NB, true>(u);
                dftn<C::NB, true>(v);
            }
            pair_sync<C::HA>();   // this pair's reads before its in-place writes
            if (act) {
                float* rr = reinterpret_cast<float*>(reg);   // R[2p][v] at rr[v], R[2p+1][v] at rr[L + v]
#pragma unroll
                for (int k1 = 0; k1 < C::NB; ++k1) {
                    const int va = C::NA * k1 + ka, vb = C::NA * k1 + kb;
                    rr[va] = u[k1].x * inv;
                    rr[L + va] = u[k1].y * inv;
                    rr[vb] = v[k1].x * inv;
                    rr[L + vb] = v[k1].y * inv;
                }
            }
        }
        __syncthreads();
    }

    if constexpr (SPLIT) {   // split form: R_ST and the template sums for ncc_finish_kernel
        float* __restrict__ o = A.rst + (int64_t)i * V * V;
        for (int e = t; e < Vu * Vv; e += C::NT) {
            const int u = e / Vv, v = e - u * Vv;
            const float* rr = reinterpret_cast<const float*>(buf + C::row((u >> 1) * 2));
            o[(u0 + u) * V + v0 + v] = rr[(u & 1) * L + v];
        }
        if (t == 0) {
            A.tsum[2 * i] = red[64];
            A.tsum[2 * i + 1] = red[65];
        }
    } else {
        ncc_peak<C::NT>(A, i, slot, u0, v0, Vu, Vv, red[64], red[65], red, [&](int u, int v) {
            const float* rr = reinterpret_cast<const float*>(buf + C::row((u >> 1) * 2));
            return rr[(u & 1) * L + v];
        });
    }
}

// Split form, second launch: one workgroup per IP assembles the NCC surface
// (Eq. 9 with the box sums of Eq. 16) from the R_ST and template sums the
// transforms left, and takes its peak, as the fused form does.  IPs whose
// template or search window leaves its image got their record from the
// transforms' launch.
constexpr int kFinishNT = 256;
__global__ __launch_bounds__(kFinishNT) void ncc_finish_kernel(const MatchArgs A) {
    __shared__ double red[66];
    const int i = (int)blockIdx.x;
    const int m = A.m, r = A.r, M = m + 2 * r, V = 2 * r + 1;
    const int py = A.ips[2 * i], px = A.ips[2 * i + 1];
    const int pry = A.prior ? A.prior[2 * i] : 0, prx = A.prior ? A.prior[2 * i + 1] : 0;
    const int64_t ty = (int64_t)py - m / 2, tx = (int64_t)px - m / 2;
    const int64_t sy = ty - r + pry, sx = tx - r + prx;
    if (!in_image(ty, tx, m, m, A.Hs, A.Ws) || !in_image(sy, sx, M, M, A.Hr, A.Wr)) return;
    const float* __restrict__ R = A.rst + (int64_t)i * V * V;
    ncc_peak<kFinishNT>(A, i, i, 0, 0, V, V, A.tsum[2 * i], A.tsum[2 * i + 1], red,
                        [&](int u, int v) { return R[u * V + v]; });
}

template <int L, int DT, bool BATCH, bool SPLIT = false>
__global__ __launch_bounds__(MatchCfg<L>::NT, MatchCfg<L>::WAVES_PER_SIMD) void match_kernel(const MatchArgs single,
                                                                   const MatchArgs* __restrict__ pairs,
                                                                   const int4* __restrict__ items) {
    using C = MatchCfg<L>;
    extern __shared__ float4 lds_raw[];
    float2* tw = reinterpret_cast<float2*>(lds_raw);
    float2* buf = tw + L;
    double* red = reinterpret_cast<double*>(buf + C::buf_elems);   // 1 KB scratch
    // One pair per launch (blockIdx.x -> IP, block), or (BATCH) a table of
    // (pair, IP, block) items over several pairs.
    init_twiddles<L>(tw);
    __syncthreads();
    if (BATCH) {
        const int4 it = items[blockIdx.x];
        const MatchArgs A = load_table(pairs, it.x);
        match_item<L, DT>(A, it.y, it.z, it.y * A.nbu * A.nbv + it.z, tw, buf, red);
    } else {
        // Workgroups are dealt to the eight XCDs in turn; renumbered so that
        // each XCD takes a contiguous run of IPs, whose overlapping search
        // windows then meet in one L2.
        const int n = (int)gridDim.x, q8 = n / 8 * 8, id = (int)blockIdx.x;
        const int k = id < q8 ? (id % 8) * (q8 / 8) + id / 8 : id;
        const int nblk = single.nbu * single.nbv;
        const int i = k / nblk;
        match_item<L, DT, SPLIT>(single, i, k - i * nblk, k, tw, buf, red);
    }
}

// Persistent form for batched plans: a grid of about two workgroups per CU
// takes items in order from a counter (zeroed before the launch) until the
// table is exhausted; every workgroup then exits.
template <int L, int DT>
__global__ __launch_bounds__(MatchCfg<L>::NT, MatchCfg<L>::WAVES_PER_SIMD) void match_persistent_kernel(const MatchArgs* __restrict__ pairs,
                                                                              const int4* __restrict__ items,
                                                                              int nitems, int* __restrict__ counter) {
    using C = MatchCfg<L>;
    extern __shared__ float4 lds_raw[];
    float2* tw = reinterpret_cast<float2*>(lds_raw);
    float2* buf = tw + L;
    double* red = reinterpret_cast<double*>(buf + C::buf_elems);
    __shared__ int next;
    init_twiddles<L>(tw);
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(counter, 1);
        __syncthreads();
        const int k = next;
        __syncthreads();   // every thread has read `next` before it is replaced
        if (k >= nitems) break;
        const int4 it = items[k];
        const MatchArgs A = load_table(pairs, it.x);
        match_item<L, DT>(A, it.y, it.z, it.y * A.nbu * A.nbv + it.z, tw, buf, red);
        __syncthreads();
    }
}

__global__ void zero_counter_kernel(int* counter) { *counter = 0; }

// ---- direct correlation on the matrix cores -----------------------------
// R_ST(u, v) = sum_h sum_i sum_k S_h(i + u, k) T_h(i, k - v): Eq. 10 summed in
// space, with T_h(i, j) = 0 outside 0 <= j < m, for 16-bit descriptors and at
// most 32 offsets per axis.  For each channel h and template row i this is
// the product of the 32 window rows i .. i + 31 (32 x K; K = 16 ceil(M / 16)
// columns, zero beyond M) with the banded Toeplitz matrix of template row i
// (K x 32, B[k][v] = T_h(i, k - v)): K / 16 MFMAs of 32 x 32 x 16 with
// float32 accumulation.  The stored 16-bit values are exact operands; only
// the order of the float32 sums differs from the FFT path.
//
// MFMA 32 x 32 x 16 operands (lane l, c = 0..7): A[l % 32][8 (l / 32) + c],
// B[8 (l / 32) + c][l % 32]; result register q of lane l holds
// D[8 (q / 4) + 4 (l / 32) + q % 4][l % 32].
//
// LDS per channel: the window (m + 31 rows, pitch PW; rows and columns from
// M on stay zero), then two copies of the zero-padded template rows, with
// Tz(q) = T_h(i, q - 32): E[q] = Tz(q), O[q] = Tz(q + 1).  Lane (v, g) of
// chunk kb needs Tz(16 kb + 8 g - v + 32 + c), c = 0..7; it reads E when v is
// even and O one element earlier when v is odd, so that every read starts on
// a 4-byte boundary.  Wave w takes the template rows i = w (mod 4); the four
// partial surfaces are summed in wave order.
constexpr int kDirNT = 256;
constexpr int kDirMaxKB = (kDirectMaxM + kDirectMaxV - 1 + 15) / 16;   // chunks of the widest window (94): 6

// Chunks of a window of M = m + 2r columns; a launch runs a fixed chunk
// count NKB >= that of each of its IPs (further chunks multiply zeros).
inline SFOC_HOST_DEVICE int dir_nkb(int m, int r) { return (m + 2 * r + 15) / 16; }
struct DirGeom {
    int PW;      // window row pitch (elements): 16 NKB + 8
    int WR;      // window rows staged: m + 31
    int PT;      // template row pitch (elements): 16 NKB + 40
    int OE;      // offset of the O copy from E (elements): m PT, padded to 17 dwords mod 32
    int bytes;   // dynamic LDS: the operands, or the four 32 x 32 float partial surfaces
};
// A B-operand read by lanes v = 0..31 of one half-wave touches the E dwords
// d + 1 .. d + 16 (even v) and the O dwords d .. d + 15 (odd v), d = 8 kb +
// 4 g plus the row's offset, and one dword later for the second dword read.
// With O 17 dwords (mod 32) after E the two sets fall on disjoint banks of
// the 32-bank LDS.
inline SFOC_HOST_DEVICE DirGeom dir_geom(int m, int nkb) {
    DirGeom g;
    g.PW = 16 * nkb + 8;
    g.WR = m + 31;
    g.PT = 16 * nkb + 40;
    g.OE = m * g.PT + 2 * ((17 - (m * g.PT / 2) % 32 + 32) % 32);
    const int b = 2 * (g.WR * g.PW + g.OE + m * g.PT);
    g.bytes = b > 4 * 1024 * 4 ? b : 4 * 1024 * 4;
    return g;
}

typedef __bf16 dir_bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 dir_f16x8 __attribute__((ext_vector_type(8)));
typedef float dir_f32x16 __attribute__((ext_vector_type(16)));

template <int DT>
SFOC_DEV dir_f32x16 dir_mfma(uint4 a, uint4 b, dir_f32x16 c) {
    if constexpr (DT == 1)
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(dir_bf16x8, a),
                                                       __builtin_bit_cast(dir_bf16x8, b), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(dir_f16x8, a),
                                                      __builtin_bit_cast(dir_f16x8, b), c, 0, 0, 0);
}

// One interest point of the direct form (A.nbu = A.nbv = 1, V <= 32, m <= 64,
// dir_nkb(m, r) <= NKB).
template <int DT, int NKB>
SFOC_DEV void direct_item(const MatchArgs& A, int i, char* lds, double* red) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, ul = lane & 31, gl = lane >> 5;
    const int m = A.m, r = A.r, M = m + 2 * r, V = 2 * r + 1;
    const DirGeom g = dir_geom(m, NKB);
    const int py = A.ips[2 * i], px = A.ips[2 * i + 1];
    const int pry = A.prior ? A.prior[2 * i] : 0, prx = A.prior ? A.prior[2 * i + 1] : 0;
    const int64_t ty = (int64_t)py - m / 2, tx = (int64_t)px - m / 2;
    const int64_t sy = ty - r + pry, sx = tx - r + prx;
    if (!in_image(ty, tx, m, m, A.Hs, A.Ws) || !in_image(sy, sx, M, M, A.Hr, A.Wr)) {
        if (t == 0) {
            sfoc_cp out;
            out.sen_row = py;
            out.sen_col = px;
            out.dy = out.dx = 0;
            out.sub_dy = out.sub_dx = 0.f;
            out.score = 0.f;
            out.flags = SFOC_CP_OOB;
            A.cps[i] = out;
        }
        if (A.ncc)
            for (int e = t; e < V * V; e += kDirNT) A.ncc[(int64_t)i * V * V + e] = 0.f;
        return;
    }
    uint16_t* Wl = reinterpret_cast<uint16_t*>(lds);
    uint16_t* E = Wl + g.WR * g.PW;
    uint16_t* O = E + g.OE;
    {   // the zero bands of both operands stay zero for every channel
        uint32_t* zp = reinterpret_cast<uint32_t*>(lds);
        const int nz = (g.WR * g.PW + g.OE + m * g.PT) / 2;
        for (int e = t; e < nz; e += kDirNT) zp[e] = 0u;
    }
    __syncthreads();
    dir_f32x16 acc0 = {}, acc1 = {};   // even and odd chunks: two independent chains
    double s1 = 0.0, s2 = 0.0;
    const int64_t plane_s = A.Hs * A.Ws, plane_r = A.Hr * A.Wr;
    const uint16_t* refp = static_cast<const uint16_t*>(A.desc_ref) + sy * A.Wr + sx;
    const uint16_t* senp = static_cast<const uint16_t*>(A.desc_sen) + ty * A.Ws + tx;
    // A channel's operands go global -> registers -> LDS.  Wave w takes the
    // rows w, w + 4, ... (at most KR window and KT template rows: M <= 16 NKB,
    // m <= min(64, 16 NKB)); a lane the columns lane and, when the window is
    // wider than 64, lane + 64.  Rows and columns are clamped into the window,
    // so that every load is in bounds and unconditional; only the stores are
    // masked.  Up to NKB = 4 the next channel's loads are issued before this
    // channel's MFMAs and land while they run; wider windows (more registers
    // per lane) load each channel in one batch before its MFMAs.
    constexpr int KR = 4 * NKB, KC = 16 * NKB > 64 ? 2 : 1, KT = 4 * NKB < 16 ? 4 * NKB : 16;
    constexpr bool kPrefetch = NKB <= 4;
    uint16_t wv[KC][KR], tv[KT];
    auto load = [&](int h) {
        // (a laundered thread index: the address arithmetic is redone per
        // channel rather than hoisted out of the loop and kept live)
        const int tl = tid_local(), ln = tl & 63, wl = __builtin_amdgcn_readfirstlane(tl >> 6);
        const uint16_t* rp = refp + h * plane_r + (int64_t)wl * A.Wr;   // wave-uniform bases
        const uint16_t* sp = senp + h * plane_s + (int64_t)wl * A.Ws;
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            const uint32_t x = (uint32_t)min(ln + 64 * c, M - 1);
#pragma unroll
            for (int j = 0; j < KR; ++j)
                wv[c][j] = rp[(uint32_t)(min(wl + 4 * j, M - 1) - wl) * (uint32_t)A.Wr + x];
        }
        const uint32_t xt = (uint32_t)min(ln, m - 1);
#pragma unroll
        for (int j = 0; j < KT; ++j) tv[j] = sp[(uint32_t)(min(wl + 4 * j, m - 1) - wl) * (uint32_t)A.Ws + xt];
    };
    auto store = [&]() {
        const int tl = tid_local(), ln = tl & 63, wl = __builtin_amdgcn_readfirstlane(tl >> 6);
        uint16_t* wrow = Wl + wl * g.PW + ln;
#pragma unroll
        for (int c = 0; c < KC; ++c)
#pragma unroll
            for (int j = 0; j < KR; ++j)
                if (wl + 4 * j < M && ln + 64 * c < M) wrow[4 * j * g.PW + 64 * c] = wv[c][j];
        uint16_t* erow = E + wl * g.PT + 32 + ln;
#pragma unroll
        for (int j = 0; j < KT; ++j)
            if (wl + 4 * j < m && ln < m) {
                erow[4 * j * g.PT] = tv[j];
                erow[4 * j * g.PT + g.OE - 1] = tv[j];   // O[y][31 + x]
                const double f = (double)(DT == 1 ? bf16_bits_to_f32(tv[j]) : f16_bits_to_f32(tv[j]));
                s1 += f;
                s2 += f * f;
            }
    };
    // per template row: every chunk's operands read first, then the MFMAs
    auto compute = [&]() {
        const int tl = tid_local(), ln = tl & 63, wl = __builtin_amdgcn_readfirstlane(tl >> 6), u = ln & 31,
                  gq = ln >> 5;
        for (int ii = wl; ii < m; ii += 4) {
            const uint16_t* arow = Wl + (ii + u) * g.PW + 8 * gq;
            const uint16_t* brow = ((u & 1) ? O : E) + ii * g.PT + 8 * gq + 32 - u - (u & 1);
            uint4 a[NKB], b[NKB];
#pragma unroll
            for (int kb = 0; kb < NKB; ++kb) {
                a[kb] = *reinterpret_cast<const uint4*>(arow + 16 * kb);
                const uint32_t* bp = reinterpret_cast<const uint32_t*>(brow + 16 * kb);
                b[kb] = make_uint4(bp[0], bp[1], bp[2], bp[3]);
            }
#pragma unroll
            for (int kb = 0; kb < NKB; ++kb) {
                if (kb & 1)
                    acc1 = dir_mfma<DT>(a[kb], b[kb], acc1);
                else
                    acc0 = dir_mfma<DT>(a[kb], b[kb], acc0);
            }
        }
    };
    if constexpr (kPrefetch) {
        load(0);
        for (int h = 0; h < A.z; ++h) {
            store();
            __syncthreads();
            if (h + 1 < A.z) load(h + 1);
            compute();
            __syncthreads();
        }
    } else {
        for (int h = 0; h < A.z; ++h) {
            load(h);
            store();
            __syncthreads();
            compute();
            __syncthreads();
        }
    }
    float* P = reinterpret_cast<float*>(lds);   // wave w's partial surface at P + 1024 w
#pragma unroll
    for (int q = 0; q < 16; ++q) P[1024 * w + (8 * (q >> 2) + 4 * gl + (q & 3)) * 32 + ul] = acc0[q] + acc1[q];
    __syncthreads();
    for (int e = t; e < V * V; e += kDirNT) {
        const int u = e / V, o = u * 32 + (e - u * V);
        P[o] = ((P[o] + P[1024 + o]) + P[2048 + o]) + P[3072 + o];
    }
    block_sum2<kDirNT>(s1, s2, red);
    ncc_peak<kDirNT>(A, i, i, 0, 0, V, V, red[64], red[65], red, [&](int u, int v) { return P[u * 32 + v]; });
}

// One pair (blockIdx.x -> IP, dealt to the XCDs in contiguous runs), or
// (BATCH) a table of (pair, IP) items.
template <int DT, int NKB, bool BATCH>
__global__ __launch_bounds__(kDirNT, 4) void match_direct_kernel(const MatchArgs single,
                                                               const MatchArgs* __restrict__ pairs,
                                                               const int4* __restrict__ items) {
    extern __shared__ float4 lds_raw[];
    __shared__ double red[66];
    char* lds = reinterpret_cast<char*>(lds_raw);
    if (BATCH) {
        const int4 it = items[blockIdx.x];
        const MatchArgs A = load_table(pairs, it.x);
        direct_item<DT, NKB>(A, it.y, lds, red);
    } else {
        const int n = (int)gridDim.x, q8 = n / 8 * 8, id = (int)blockIdx.x;
        direct_item<DT, NKB>(single, id < q8 ? (id % 8) * (q8 / 8) + id / 8 : id, lds, red);
    }
}

// ---- combining offset blocks --------------------------------------------
// One thread per interest point: the best score over its blocks (ties: the
// smallest row-major surface index), the flags, and the parabola from the
// surface the blocks wrote.  Same decisions as the single-block path.
template <bool BATCH>
__global__ __launch_bounds__(256) void peak_kernel(const MatchArgs single, const MatchArgs* __restrict__ pairs,
                                                   const int4* __restrict__ items) {
    const MatchArgs A = BATCH ? load_table(pairs, items[blockIdx.x].x) : single;
    const int i = (BATCH ? items[blockIdx.x].y : (int)(blockIdx.x * blockDim.x)) + (int)threadIdx.x;
    if (i >= A.n) return;
    const int nblk = A.nbu * A.nbv;
    const int r = A.r, V = 2 * r + 1;
    sfoc_cp out;
    out.sen_row = A.ips[2 * i];
    out.sen_col = A.ips[2 * i + 1];
    out.dy = out.dx = 0;
    out.sub_dy = out.sub_dx = 0.f;
    out.score = 0.f;
    out.flags = 0;
    float best = -INFINITY;
    int bidx = 0x7fffffff, fl = 0;
    for (int b = 0; b < nblk; ++b) {
        const float4 q = A.blk[(int64_t)i * nblk + b];
        const int qi = __float_as_int(q.y);
        fl |= __float_as_int(q.z);
        if (q.x > best || (q.x == best && qi < bidx)) {
            best = q.x;
            bidx = qi;
        }
    }
    const float* surf = (A.ncc ? A.ncc : A.surf) + (int64_t)i * V * V;
    if (fl & kBlkOOB) {
        out.flags = SFOC_CP_OOB;
    } else if ((fl & kBlkBadT) || ((fl & kBlkNonfin) && !(fl & kBlkFlatT))) {
        out.flags = SFOC_CP_NONFINITE;
    } else if (fl & kBlkFlatT) {
        out.flags = SFOC_CP_FLAT_T;
    } else if (!(fl & kBlkNonflat) || bidx >= V * V) {
        out.flags = SFOC_CP_FLAT_S;
    } else {
        const int u = bidx / V, v = bidx - u * V;
        out.dy = u - r;
        out.dx = v - r;
        out.score = best;
        if (u == 0 || v == 0 || u == V - 1 || v == V - 1) {
            out.flags = SFOC_CP_EDGE_PEAK;
        } else {
            const float c0 = best;
            const float cu = surf[bidx - V], cd = surf[bidx + V], cl = surf[bidx - 1], cr = surf[bidx + 1];
            float den = cu - 2.f * c0 + cd;
            float d = 0.f;
            if (den < 0.f) d = fminf(0.5f, fmaxf(-0.5f, (cu - cd) / (2.f * den)));
            out.sub_dy = d;
            den = cl - 2.f * c0 + cr;
            d = 0.f;
            if (den < 0.f) d = fminf(0.5f, fmaxf(-0.5f, (cl - cr) / (2.f * den)));
            out.sub_dx = d;
        }
    }
    A.cps[i] = out;
}

// ---- consistency: median displacement, 1.5 px (Section 4.1) ------------
// One workgroup; exact k-th smallest by 8-bit radix selection on
// order-preserving keys, so any n works without a sort buffer.
constexpr int kConsNT = 256;
constexpr uint32_t kBad = SFOC_CP_OOB | SFOC_CP_FLAT_T | SFOC_CP_FLAT_S | SFOC_CP_EDGE_PEAK | SFOC_CP_NONFINITE;

SFOC_DEV uint32_t fkey(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
SFOC_DEV float fkey_inv(uint32_t k) {
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}
SFOC_DEV float cp_disp(const sfoc_cp& c, const int32_t* prior, int i, int axis) {
    const int pr = prior ? prior[2 * i + axis] : 0;
    return axis == 0 ? (float)(pr + c.dy) + c.sub_dy : (float)(pr + c.dx) + c.sub_dx;
}

// Keys of the eligible CPs' displacements are cached in LDS up to this many
// CPs (both axes); larger pairs read them from the records on every pass.
constexpr int kConsCache = 6144;

// The k-th smallest (0-based) key among the eligible CPs for four (axis,
// rank) targets at once: four 8-bit radix passes, each building the four
// targets' histograms in one sweep over the keys; wave q then scans
// histogram q (four bins per lane) for the bin holding its rank.
static_assert(kConsNT == 256, "one scanning wave per target");
SFOC_DEV void select_kth4(const sfoc_cp* cps, const int32_t* prior, int n, const int (&axis)[4], int (&k)[4],
                          const uint32_t* const (&cache)[2], int ncache, uint32_t (*hist)[256], uint32_t* sel,
                          uint32_t (&prefix)[4]) {
    uint32_t mask = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) prefix[q] = 0;
    for (int shift = 24; shift >= 0; shift -= 8) {
        for (int b = threadIdx.x; b < 4 * 256; b += kConsNT) hist[b >> 8][b & 255] = 0;
        __syncthreads();
        const int cnt = cache[0] ? ncache : n;
        for (int i = threadIdx.x; i < cnt; i += kConsNT) {
            uint32_t key[2];
            if (cache[0]) {
                key[0] = cache[0][i];
                key[1] = cache[1][i];
            } else {
                const sfoc_cp c = cps[i];
                if (c.flags & kBad) continue;
                key[0] = fkey(cp_disp(c, prior, i, 0));
                key[1] = fkey(cp_disp(c, prior, i, 1));
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t kq = key[axis[q]];
                if ((kq & mask) == prefix[q]) atomicAdd(&hist[q][(kq >> shift) & 255u], 1u);
            }
        }
        __syncthreads();
        {
            const int q = threadIdx.x >> 6, lane = threadIdx.x & 63;
            const uint32_t* h = hist[q];
            const uint32_t h0 = h[4 * lane], h1 = h[4 * lane + 1], h2 = h[4 * lane + 2], h3 = h[4 * lane + 3];
            const uint32_t own = h0 + h1 + h2 + h3;
            uint32_t incl = own;   // inclusive prefix over lanes
            for (int d = 1; d < 64; d <<= 1) {
                const uint32_t u = __shfl_up(incl, d, 64);
                if (lane >= d) incl += u;
            }
            const uint32_t before = incl - own;   // keys in bins below this lane's four
            uint32_t kq = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (j == q) kq = (uint32_t)k[j];
            if (before <= kq && kq < incl) {   // exactly one lane per target
                uint32_t cum = before;
                int b = 4 * lane;
                const uint32_t hs[4] = {h0, h1, h2, h3};
                for (int j = 0; j < 4; ++j, ++b) {
                    if (cum + hs[j] > kq) break;
                    cum += hs[j];
                }
                sel[2 * q] = (uint32_t)b;
                sel[2 * q + 1] = cum;
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            prefix[q] |= sel[2 * q] << shift;
            k[q] -= (int)sel[2 * q + 1];
        }
        mask |= 255u << shift;
        __syncthreads();
    }
}

__global__ __launch_bounds__(kConsNT) void consistency_kernel(sfoc_cp* cps, const int32_t* prior, int n,
                                                              const MatchArgs* __restrict__ pairs) {
    if (pairs) {   // one workgroup per pair of a batched plan
        const MatchArgs P = load_table(pairs, (int)blockIdx.x);
        cps = P.cps;
        prior = P.prior;
        n = P.n;
    }
    __shared__ uint32_t hist[4][256];
    __shared__ uint32_t sel[8];
    __shared__ int cnt;
    __shared__ uint32_t keys[2][kConsCache];
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    // eligible CPs: count, and (for small pairs) their keys, compacted in
    // any order (the selection does not depend on it)
    const bool cached = n <= kConsCache;
    for (int i = threadIdx.x; i < n; i += kConsNT) {
        const sfoc_cp c = cps[i];
        if (c.flags & kBad) continue;
        const int slot = atomicAdd(&cnt, 1);
        if (cached) {
            keys[0][slot] = fkey(cp_disp(c, prior, i, 0));
            keys[1][slot] = fkey(cp_disp(c, prior, i, 1));
        }
    }
    __syncthreads();
    const int ne = cnt;
    if (ne == 0) return;
    // the median per axis: the middle key, or the mean of the two middle
    // ones (ranks ne/2 - 1 and ne/2) when ne is even
    const int axis[4] = {0, 0, 1, 1};
    int k[4] = {(ne - 1) / 2, ne / 2, (ne - 1) / 2, ne / 2};
    const uint32_t* const cache[2] = {cached ? keys[0] : nullptr, cached ? keys[1] : nullptr};
    uint32_t sk[4];
    select_kth4(cps, prior, n, axis, k, cache, ne, hist, sel, sk);
    float med[2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
        med[a] = (ne & 1) ? fkey_inv(sk[2 * a + 1]) : 0.5f * (fkey_inv(sk[2 * a]) + fkey_inv(sk[2 * a + 1]));
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += kConsNT) {
        sfoc_cp c = cps[i];
        if (c.flags & kBad) continue;
        const float ey = cp_disp(c, prior, i, 0) - med[0];
        const float ex = cp_disp(c, prior, i, 1) - med[1];
        c.flags |= (sqrtf(ey * ey + ex * ex) > 1.5f) ? SFOC_CP_INCONSISTENT : SFOC_CP_VALID;
        cps[i].flags = c.flags;
    }
}

// ---- per-window integral images (Eq. 14-16 over one search window) --------
// One workgroup per IP: G1 / G2 are the (M+1) x (M+1) exclusive prefix sums
// of sum_c g and sum_c g^2 (float64, of the stored values) over the IP's
// M x M search window, zero first row and column.  The per-pixel sums run
// over the channels in order, then each row is summed left to right and
// each column top to bottom: a fixed order, so results are reproducible.
// An IP whose windows leave the images is skipped (the match flags it and
// reads nothing).
template <int DT>
__global__ __launch_bounds__(256) void window_integral_kernel(const MatchArgs A) {
    const int i = blockIdx.x, t = threadIdx.x;
    const int m = A.m, r = A.r, M = m + 2 * r, P = M + 1;
    const int py = A.ips[2 * i], px = A.ips[2 * i + 1];
    const int pry = A.prior ? A.prior[2 * i] : 0, prx = A.prior ? A.prior[2 * i + 1] : 0;
    const int64_t ty = (int64_t)py - m / 2, tx = (int64_t)px - m / 2;
    const int64_t sy = ty - r + pry, sx = tx - r + prx;
    if (!in_image(ty, tx, m, m, A.Hs, A.Ws) || !in_image(sy, sx, M, M, A.Hr, A.Wr)) return;
    double* __restrict__ G1 = const_cast<double*>(A.integ1) + (int64_t)i * P * P;
    double* __restrict__ G2 = const_cast<double*>(A.integ2) + (int64_t)i * P * P;
    const int64_t plane = A.Hr * A.Wr;
    for (int e = t; e < P * P; e += 256) {
        const int y = e / P, x = e - y * P;
        double s1 = 0.0, s2 = 0.0;
        if (y > 0 && x > 0) {
            const int o = (int)((sy + y - 1) * A.Wr + sx + x - 1);   // within one plane (< 2^30)
            for (int h = 0; h < A.z; ++h) {
                const double g = (double)ldd<DT>(elem_ptr<DT>(A.desc_ref, h * plane), o);
                s1 += g;
                s2 = fma(g, g, s2);
            }
        }
        G1[e] = s1;
        G2[e] = s2;
    }
    __syncthreads();
    for (int y = 1 + t; y < P; y += 256) {   // rows, left to right
        double a = 0.0, b = 0.0;
        for (int x = 1; x < P; ++x) {
            a += G1[(int64_t)y * P + x];
            b += G2[(int64_t)y * P + x];
            G1[(int64_t)y * P + x] = a;
            G2[(int64_t)y * P + x] = b;
        }
    }
    __syncthreads();
    for (int x = 1 + t; x < P; x += 256) {   // columns, top to bottom
        double a = 0.0, b = 0.0;
        for (int y = 1; y < P; ++y) {
            a += G1[(int64_t)y * P + x];
            b += G2[(int64_t)y * P + x];
            G1[(int64_t)y * P + x] = a;
            G2[(int64_t)y * P + x] = b;
        }
    }
}

// ---- launch -------------------------------------------------------------
void match_args_layout(MatchArgs& a, const MatchPlan& mp, void* ws) {
    a.nbu = a.nbv = mp.nb;
    a.Vb = mp.Vb;
    a.surf = nullptr;
    a.blk = nullptr;
    if (mp.nb > 1) {
        const int V = 2 * a.r + 1;
        a.surf = (float*)ws;
        a.blk = (float4*)((char*)ws + align_up((size_t)a.n * V * V * sizeof(float), 256));
    }
}

template <int L, int DT, bool SPLIT = false>
static hipError_t launch_match_L(const MatchArgs& a, hipStream_t st) {
    using C = MatchCfg<L>;
    auto kern = match_kernel<L, DT, false, SPLIT>;
    hipError_t e = ensure_dynamic_lds((const void*)kern, (int)C::lds_bytes);
    if (e != hipSuccess) return e;
    trace_begin(st, SFOC_K_MATCH);
    hipLaunchKernelGGL(kern, dim3(a.n * a.nbu * a.nbv), dim3(C::NT), C::lds_bytes, st, a, (const MatchArgs*)nullptr,
                       (const int4*)nullptr);
    trace_end(st, SFOC_K_MATCH);
    return hipGetLastError();
}

template <int DT, int NKB, bool BATCH>
static hipError_t launch_direct_K(const MatchArgs& a, const MatchArgs* pairs, const int4* items, int nblocks,
                                  int lds, hipStream_t st) {
    auto kern = match_direct_kernel<DT, NKB, BATCH>;
    hipError_t e = ensure_dynamic_lds((const void*)kern, lds);
    if (e != hipSuccess) return e;
    trace_begin(st, SFOC_K_MATCH);
    hipLaunchKernelGGL(kern, dim3(nblocks), dim3(kDirNT), lds, st, a, pairs, items);
    trace_end(st, SFOC_K_MATCH);
    return hipGetLastError();
}

template <int DT, bool BATCH>
static hipError_t launch_direct_DT(const MatchArgs& a, const MatchArgs* pairs, const int4* items, int nblocks,
                                   DirLaunch d, hipStream_t st) {
    const int lds = dir_geom(d.m, d.nkb).bytes;
    switch (d.nkb) {
        case 1: return launch_direct_K<DT, 1, BATCH>(a, pairs, items, nblocks, lds, st);
        case 2: return launch_direct_K<DT, 2, BATCH>(a, pairs, items, nblocks, lds, st);
        case 3: return launch_direct_K<DT, 3, BATCH>(a, pairs, items, nblocks, lds, st);
        case 4: return launch_direct_K<DT, 4, BATCH>(a, pairs, items, nblocks, lds, st);
        case 5: return launch_direct_K<DT, 5, BATCH>(a, pairs, items, nblocks, lds, st);
        case 6: return launch_direct_K<DT, 6, BATCH>(a, pairs, items, nblocks, lds, st);
        default: return hipErrorInvalidValue;
    }
}

// The direct form: one workgroup per IP of one pair (items null), or per
// (pair, IP) item; d holds the largest m and chunk count of the IPs' pairs.
static hipError_t launch_direct(const MatchArgs& a, const MatchArgs* pairs, const int4* items, int nblocks,
                                DirLaunch d, int dtype, hipStream_t st) {
    if (dtype == 1)
        return items ? launch_direct_DT<1, true>(a, pairs, items, nblocks, d, st)
                     : launch_direct_DT<1, false>(a, pairs, items, nblocks, d, st);
    if (dtype == 2)
        return items ? launch_direct_DT<2, true>(a, pairs, items, nblocks, d, st)
                     : launch_direct_DT<2, false>(a, pairs, items, nblocks, d, st);
    return hipErrorInvalidValue;
}

DirLaunch direct_launch_of(int m, int r) { return DirLaunch{m, dir_nkb(m, r)}; }

template <int L, bool SPLIT = false>
static hipError_t launch_match_side(const MatchArgs& a, int dtype, hipStream_t st) {
    return dtype == 0 ? launch_match_L<L, 0, SPLIT>(a, st)
                      : dtype == 1 ? launch_match_L<L, 1, SPLIT>(a, st) : launch_match_L<L, 2, SPLIT>(a, st);
}

// ---- split form: transforms, then NCC and peaks ----------------------------
bool match_split_ok(int n, int m, int r, int dtype) {
    const MatchPlan mp = match_plan_dt(n, m, r, dtype);
    return n > 0 && mp.L != kDirectSide && mp.L != 0 && mp.nb == 1;
}

static size_t split_rst_bytes(int n, int r) {
    const size_t V = 2 * (size_t)r + 1;
    return ((size_t)n * V * V * sizeof(float) + 255) / 256 * 256;
}

size_t match_split_bytes(int n, int r) { return split_rst_bytes(n, r) + (size_t)n * 2 * sizeof(double); }

static MatchArgs split_args(const void* desc_sen, int64_t Hs, int64_t Ws, const void* desc_ref, int64_t Hr,
                            int64_t Wr, const double* i1, const double* i2, int z, int dtype, const int32_t* ips,
                            const int32_t* prior, int n, int m, int r, float* ncc, sfoc_cp* cps, void* ws,
                            void* split) {
    MatchArgs a;
    a.desc_sen = desc_sen;
    a.desc_ref = desc_ref;
    a.integ1 = i1;
    a.integ2 = i2;
    a.ips = ips;
    a.prior = prior;
    a.ncc = ncc;
    a.cps = cps;
    a.Hs = Hs;
    a.Ws = Ws;
    a.Hr = Hr;
    a.Wr = Wr;
    a.z = z;
    a.dtype = dtype;
    a.n = n;
    a.m = m;
    a.r = r;
    match_args_layout(a, match_plan_dt(n, m, r, dtype), ws);
    a.integ_win = 0;
    a.rst = (float*)split;
    a.tsum = (double*)((char*)split + split_rst_bytes(n, r));
    return a;
}

hipError_t launch_match_fft(const void* desc_sen, int64_t Hs, int64_t Ws, const void* desc_ref, int64_t Hr,
                            int64_t Wr, int z, int dtype, const int32_t* ips, const int32_t* prior, int n, int m,
                            int r, float* ncc, sfoc_cp* cps, void* ws, void* split, hipStream_t st) {
    if (!match_split_ok(n, m, r, dtype)) return hipErrorInvalidValue;
    const MatchArgs a = split_args(desc_sen, Hs, Ws, desc_ref, Hr, Wr, nullptr, nullptr, z, dtype, ips, prior, n, m,
                                   r, ncc, cps, ws, split);
    switch (match_plan_dt(n, m, r, dtype).L) {
        case 64: return launch_match_side<64, true>(a, dtype, st);
        case 128: return launch_match_side<128, true>(a, dtype, st);
        case 160: return launch_match_side<160, true>(a, dtype, st);
        case 192: return launch_match_side<192, true>(a, dtype, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_match_finish(const void* desc_sen, int64_t Hs, int64_t Ws, const void* desc_ref, int64_t Hr,
                               int64_t Wr, const double* i1, const double* i2, int z, int dtype, const int32_t* ips,
                               const int32_t* prior, int n, int m, int r, float* ncc, sfoc_cp* cps, void* ws,
                               void* split, hipStream_t st, bool consistency) {
    if (!match_split_ok(n, m, r, dtype) || !i1 || !i2) return hipErrorInvalidValue;
    const MatchArgs a = split_args(desc_sen, Hs, Ws, desc_ref, Hr, Wr, i1, i2, z, dtype, ips, prior, n, m, r, ncc,
                                   cps, ws, split);
    trace_begin(st, SFOC_K_PEAK);
    hipLaunchKernelGGL(ncc_finish_kernel, dim3(n), dim3(kFinishNT), 0, st, a);
    trace_end(st, SFOC_K_PEAK);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !consistency) return e;
    return launch_consistency(cps, prior, n, st);
}

hipError_t launch_match(const void* desc_sen, int64_t Hs, int64_t Ws, const void* desc_ref, int64_t Hr, int64_t Wr,
                        const double* i1, const double* i2, int z, int dtype, const int32_t* ips,
                        const int32_t* prior, int n, int m, int r, float* ncc, sfoc_cp* cps, void* ws,
                        hipStream_t st, bool consistency) {
    MatchArgs a;
    a.desc_sen = desc_sen;
    a.desc_ref = desc_ref;
    a.integ1 = i1;
    a.integ2 = i2;
    a.ips = ips;
    a.prior = prior;
    a.ncc = ncc;
    a.cps = cps;
    a.Hs = Hs;
    a.Ws = Ws;
    a.Hr = Hr;
    a.Wr = Wr;
    a.z = z;
    a.dtype = dtype;
    a.n = n;
    a.m = m;
    a.r = r;
    const MatchPlan mp = match_plan_dt(n, m, r, dtype);
    const int L = mp.L;
    match_args_layout(a, mp, ws);
    a.integ_win = 0;
    hipError_t e;
    if (!i1) {   // per-window integral images, after the split-offset scratch
        double* g = (double*)((char*)ws + mp.ws_bytes);
        const size_t per = (size_t)(m + 2 * r + 1) * (m + 2 * r + 1);
        a.integ1 = g;
        a.integ2 = g + (size_t)n * per;
        a.integ_win = 1;
        trace_begin(st, SFOC_K_INTEGRAL);
        if (dtype == 0) hipLaunchKernelGGL(window_integral_kernel<0>, dim3(n), dim3(256), 0, st, a);
        else if (dtype == 1) hipLaunchKernelGGL(window_integral_kernel<1>, dim3(n), dim3(256), 0, st, a);
        else hipLaunchKernelGGL(window_integral_kernel<2>, dim3(n), dim3(256), 0, st, a);
        trace_end(st, SFOC_K_INTEGRAL);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    switch (L) {
        case 64: e = launch_match_side<64>(a, dtype, st); break;
        case 128: e = launch_match_side<128>(a, dtype, st); break;
        case 160: e = launch_match_side<160>(a, dtype, st); break;
        case 192: e = launch_match_side<192>(a, dtype, st); break;
        case kDirectSide: e = launch_direct(a, nullptr, nullptr, n, direct_launch_of(m, r), dtype, st); break;
        default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    if (mp.nb > 1) {
        trace_begin(st, SFOC_K_PEAK);
        hipLaunchKernelGGL(peak_kernel<false>, dim3((n + 255) / 256), dim3(256), 0, st, a, (const MatchArgs*)nullptr,
                           (const int4*)nullptr);
        trace_end(st, SFOC_K_PEAK);
    }
    if (!consistency) return hipGetLastError();
    return launch_consistency(cps, prior, n, st);
}

hipError_t launch_consistency(sfoc_cp* cps, const int32_t* prior, int n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    trace_begin(st, SFOC_K_CONSISTENCY);
    hipLaunchKernelGGL(consistency_kernel, dim3(1), dim3(kConsNT), 0, st, cps, prior, n, (const MatchArgs*)nullptr);
    trace_end(st, SFOC_K_CONSISTENCY);
    return hipGetLastError();
}

// Adds dy to the sensed row of n CP records (records of IPs matched in a
// band of rows, whose coordinates were taken relative to the band).
__global__ __launch_bounds__(256) void cp_row_shift_kernel(sfoc_cp* cps, int n, int dy) {
    const int i = (int)(blockIdx.x * 256 + threadIdx.x);
    if (i < n) cps[i].sen_row += dy;
}

hipError_t launch_cp_row_shift(sfoc_cp* cps, int n, int dy, hipStream_t st) {
    if (n == 0 || dy == 0) return hipSuccess;
    hipLaunchKernelGGL(cp_row_shift_kernel, dim3((n + 255) / 256), dim3(256), 0, st, cps, n, dy);
    return hipGetLastError();
}

// ---- batched launches ---------------------------------------------------
template <int L, int DT>
static hipError_t launch_match_items_L(const MatchArgs* pairs, const int4* items, int nitems, int* counter, int grid,
                                       hipStream_t st) {
    using C = MatchCfg<L>;
    MatchArgs none{};
    hipError_t e;
    if (counter) {
        auto kern = match_persistent_kernel<L, DT>;
        if ((e = ensure_dynamic_lds((const void*)kern, (int)C::lds_bytes)) != hipSuccess) return e;
        trace_begin(st, SFOC_K_MATCH);
        hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(1), 0, st, counter);
        const int g = grid * C::MINB;   // `grid` counts CUs
        hipLaunchKernelGGL(kern, dim3(g < nitems ? g : nitems), dim3(C::NT), C::lds_bytes, st, pairs, items,
                           nitems, counter);
        trace_end(st, SFOC_K_MATCH);
    } else {
        auto kern = match_kernel<L, DT, true>;
        if ((e = ensure_dynamic_lds((const void*)kern, (int)C::lds_bytes)) != hipSuccess) return e;
        trace_begin(st, SFOC_K_MATCH);
        hipLaunchKernelGGL(kern, dim3(nitems), dim3(C::NT), C::lds_bytes, st, none, pairs, items);
        trace_end(st, SFOC_K_MATCH);
    }
    return hipGetLastError();
}

template <int L>
static hipError_t launch_match_items_side(int dtype, const MatchArgs* pairs, const int4* items, int nitems,
                                          int* counter, int grid, hipStream_t st) {
    return dtype == 0 ? launch_match_items_L<L, 0>(pairs, items, nitems, counter, grid, st)
         : dtype == 1 ? launch_match_items_L<L, 1>(pairs, items, nitems, counter, grid, st)
                      : launch_match_items_L<L, 2>(pairs, items, nitems, counter, grid, st);
}

// One launch over (pair, IP, block) items that share the transform side L:
// one workgroup per item, or (counter != null) a persistent grid of `grid`
// workgroups taking items from *counter.  The direct form (L = kDirectSide)
// takes one workgroup per item, sized by `dir`.
hipError_t launch_match_items(int L, int dtype, const MatchArgs* pairs, const int4* items, int nitems, int* counter,
                              int grid, DirLaunch dir, hipStream_t st) {
    if (nitems == 0) return hipSuccess;
    if (L == kDirectSide) {
        if (counter) return hipErrorInvalidValue;
        MatchArgs none{};
        return launch_direct(none, pairs, items, nitems, dir, dtype, st);
    }
    switch (L) {
        case 64: return launch_match_items_side<64>(dtype, pairs, items, nitems, counter, grid, st);
        case 128: return launch_match_items_side<128>(dtype, pairs, items, nitems, counter, grid, st);
        case 160: return launch_match_items_side<160>(dtype, pairs, items, nitems, counter, grid, st);
        case 192: return launch_match_items_side<192>(dtype, pairs, items, nitems, counter, grid, st);
        default: return hipErrorInvalidValue;
    }
}

// Peak of split pairs: items {pair, first IP of a run of 256}.
hipError_t launch_peak_batched(const MatchArgs* pairs, const int4* items, int nitems, hipStream_t st) {
    if (nitems == 0) return hipSuccess;
    MatchArgs none{};
    trace_begin(st, SFOC_K_PEAK);
    hipLaunchKernelGGL(peak_kernel<true>, dim3(nitems), dim3(256), 0, st, none, pairs, items);
    trace_end(st, SFOC_K_PEAK);
    return hipGetLastError();
}

// Consistency of every pair of a plan: one workgroup per pair.
hipError_t launch_consistency_batched(const MatchArgs* pairs, int npairs, hipStream_t st) {
    if (npairs == 0) return hipSuccess;
    trace_begin(st, SFOC_K_CONSISTENCY);
    hipLaunchKernelGGL(consistency_kernel, dim3(npairs), dim3(kConsNT), 0, st, (sfoc_cp*)nullptr,
                       (const int32_t*)nullptr, 0, pairs);
    trace_end(st, SFOC_K_CONSISTENCY);
    return hipGetLastError();
}

}  // namespace sfoc
