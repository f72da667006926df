// RANSAC outlier rejection over CP records (Section 3.2.3: after matching,
// random sample consensus removes mismatched CPs under a projective model,
// or an affine one).  Four launches, all float64:
//
//  1. prepare   (one workgroup): ordered compaction of the CPs with an
//               interior peak into candidate correspondences, in
//               normalised coordinates.
//  2. fit      (a thread per hypothesis): sample indices from the caller's
//               random words, degeneracy test, closed-form minimal fit
//               (Cramer's rule for three points; for four, the projective
//               map of the unit square onto each quadrilateral, one
//               composed with the adjugate of the other); count zeroed.
//  3. score    (hypothesis blocks x candidate chunks): each workgroup
//               stages one chunk of candidates in LDS, every lane of a
//               wave reading the same address (broadcast), counts the
//               inliers of its hypotheses and adds them to the totals with
//               integer atomics (exact in any order).
//  4. finish   (one workgroup): best hypothesis (most inliers, lowest
//               index on ties), least-squares refits over the inliers from
//               normal equations accumulated in a fixed order and solved
//               by a register-resident Cholesky factorisation (so the
//               result is bit-reproducible), the final inlier set, the CP
//               flags and the model in pixel coordinates.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "sfoc_dev.h"
#include "sfoc_launch.h"
#include "sfoc_plan.h"
#include "sfoc_trace.h"

namespace sfoc {
namespace ransac {

constexpr uint32_t kBad = SFOC_CP_OOB | SFOC_CP_FLAT_T | SFOC_CP_FLAT_S | SFOC_CP_EDGE_PEAK | SFOC_CP_NONFINITE;
constexpr double kCollinearEps = 1e-9;   // |cross| in normalised units
constexpr double kSingular = 1e-12;      // relative pivot of a refit system
constexpr int kPrepNT = 1024, kHypNT = 256, kTile = 1024, kFinNT = 256;
constexpr int kScoreBlocks = 1024, kMinChunk = 32;   // target grid of the score launch
constexpr int kMaxN = 1 << 22, kMaxHyp = 1 << 20, kMaxRefine = 16;

struct Norm {
    double cr, cc, s;   // v_n = (v - c) * s
};

struct Args {
    const sfoc_cp* cps_in;
    sfoc_cp* cps;
    const int32_t* prior;
    int n;
    Norm ns, nr;
    double s_ref;       // reference pixels per normalised unit
    double thr_n2;      // (threshold / s_ref)^2
    int model, k, n_hyp, n_refine;
    int chunk;          // candidates per score workgroup
    const uint32_t* words;
    double4* cand;      // (src row, src col, dst row, dst col), normalised
    int* cidx;          // candidate -> CP index
    int* ncand;
    int* counts;        // per hypothesis (-1: degenerate)
    double* hyp;        // per hypothesis, 9 doubles (normalised coordinates)
    uint8_t* inl;
    double* model_out;  // 9 doubles, pixels
    int32_t* info;      // n_cand, inliers, best, status
};

// ---- small FP64 helpers ----------------------------------------------------
// Exact evaluation order matters for the degeneracy decision: it is taken
// without fused multiply-adds so that it is the same decision as a plain
// IEEE evaluation of the same expression.
SFOC_DEV double cross3(double ax, double ay, double bx, double by, double cx, double cy) {
#pragma clang fp contract(off)
    const double p = (bx - ax) * (cy - ay);
    const double q = (by - ay) * (cx - ax);
    return p - q;
}

// Projective map of the unit square onto the quadrilateral q (corners
// (0,0), (1,0), (1,1), (0,1) to q[0..3]); false if three corners are
// collinear (the divisor vanishes).
SFOC_DEV bool square_to_quad(const double (&qx)[4], const double (&qy)[4], double (&M)[9]) {
    const double sx = qx[0] - qx[1] + qx[2] - qx[3], sy = qy[0] - qy[1] + qy[2] - qy[3];
    const double dx1 = qx[1] - qx[2], dx2 = qx[3] - qx[2], dy1 = qy[1] - qy[2], dy2 = qy[3] - qy[2];
    const double den = dx1 * dy2 - dx2 * dy1;
    if (den == 0.0) return false;
    const double g = (sx * dy2 - dx2 * sy) / den, h = (dx1 * sy - sx * dy1) / den;
    M[0] = qx[1] - qx[0] + g * qx[1];
    M[1] = qx[3] - qx[0] + h * qx[3];
    M[2] = qx[0];
    M[3] = qy[1] - qy[0] + g * qy[1];
    M[4] = qy[3] - qy[0] + h * qy[3];
    M[5] = qy[0];
    M[6] = g;
    M[7] = h;
    M[8] = 1.0;
    return true;
}

SFOC_DEV void adjugate(const double (&M)[9], double (&A)[9]) {
    A[0] = M[4] * M[8] - M[5] * M[7];
    A[1] = M[2] * M[7] - M[1] * M[8];
    A[2] = M[1] * M[5] - M[2] * M[4];
    A[3] = M[5] * M[6] - M[3] * M[8];
    A[4] = M[0] * M[8] - M[2] * M[6];
    A[5] = M[2] * M[3] - M[0] * M[5];
    A[6] = M[3] * M[7] - M[4] * M[6];
    A[7] = M[1] * M[6] - M[0] * M[7];
    A[8] = M[0] * M[4] - M[1] * M[3];
}

SFOC_DEV bool inlier(const double (&M)[9], bool proj, double4 c, double thr_n2) {
    const double x = c.x, y = c.y;
    double w = 1.0;
    if (proj) {
        w = fma(M[6], x, fma(M[7], y, M[8]));
        if (!(w > 0.0)) return false;
    }
    const double ex = fma(M[0], x, fma(M[1], y, M[2])) - c.z * w;
    const double ey = fma(M[3], x, fma(M[4], y, M[5])) - c.w * w;
    return fma(ex, ex, ey * ey) <= thr_n2 * (w * w);
}

// ---- 1. candidates ---------------------------------------------------------
// Rounds of kPrepU * kPrepNT consecutive CPs; in each round every thread
// loads kPrepU flags at once (coalesced), then the kPrepU blocks of kPrepNT
// CPs are compacted in CP order: wave ballots give the rank within a wave,
// a prefix over the wave totals the rank within the workgroup.
constexpr int kPrepU = 4;
__global__ __launch_bounds__(kPrepNT) void prepare_kernel(Args a) {
    constexpr int kW = kPrepNT / 64;
    __shared__ int wsum[kW];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    int base = 0;
    for (int r0 = 0; r0 < a.n; r0 += kPrepU * kPrepNT) {
        uint32_t fl[kPrepU];
#pragma unroll
        for (int u = 0; u < kPrepU; ++u) {
            const int i = r0 + u * kPrepNT + t;
            fl[u] = i < a.n ? a.cps_in[i].flags : kBad;
        }
#pragma unroll
        for (int u = 0; u < kPrepU; ++u) {
            const int i = r0 + u * kPrepNT + t;
            const bool e = (fl[u] & kBad) == 0;
            const uint64_t bal = __ballot(e);
            if (lane == 0) wsum[wv] = __popcll(bal);
            __syncthreads();
            int off = base, tot = 0;
            for (int w = 0; w < kW; ++w) {
                off += w < wv ? wsum[w] : 0;
                tot += wsum[w];
            }
            if (e) {
                const int o = off + __popcll(bal & ((1ull << lane) - 1ull));
                const sfoc_cp p = a.cps_in[i];
                const int py = a.prior ? a.prior[2 * i] : 0, px = a.prior ? a.prior[2 * i + 1] : 0;
                const double sr = (double)p.sen_row, sc = (double)p.sen_col;
                const double dr = (double)(p.sen_row + py + p.dy) + (double)p.sub_dy;
                const double dc = (double)(p.sen_col + px + p.dx) + (double)p.sub_dx;
                a.cand[o] = make_double4((sr - a.ns.cr) * a.ns.s, (sc - a.ns.cc) * a.ns.s,
                                         (dr - a.nr.cr) * a.nr.s, (dc - a.nr.cc) * a.nr.s);
                a.cidx[o] = i;
            }
            base += tot;
            __syncthreads();   // wsum is rewritten by the next block
        }
    }
    if (t == 0) *a.ncand = base;
}

// ---- 2. minimal fits ---------------------------------------------------------
__global__ __launch_bounds__(kHypNT) void fit_kernel(Args a) {
    const int h = blockIdx.x * kHypNT + threadIdx.x;
    const int n = *a.ncand;
    const bool proj = a.model == SFOC_MODEL_PROJECTIVE;
    const int k = a.k;
    bool ok = h < a.n_hyp && n >= k;
    double M[9];
    if (ok) {
        int idx[4];
        double sx[4], sy[4], dx[4], dy[4];
        for (int j = 0; j < k; ++j) {
            idx[j] = (int)(((uint64_t)a.words[(int64_t)h * k + j] * (uint64_t)n) >> 32);
            for (int q = 0; q < j; ++q) ok = ok && idx[q] != idx[j];
        }
        if (ok) {
            for (int j = 0; j < k; ++j) {
                const double4 c = a.cand[idx[j]];
                sx[j] = c.x;
                sy[j] = c.y;
                dx[j] = c.z;
                dy[j] = c.w;
            }
            for (int p = 0; p < k; ++p)
                for (int q = p + 1; q < k; ++q)
                    for (int r = q + 1; r < k; ++r) {
                        ok = ok && fabs(cross3(sx[p], sy[p], sx[q], sy[q], sx[r], sy[r])) > kCollinearEps;
                        ok = ok && fabs(cross3(dx[p], dy[p], dx[q], dy[q], dx[r], dy[r])) > kCollinearEps;
                    }
        }
        if (ok && !proj) {
            // Cramer's rule on the two edge vectors of the source triangle
            const double e1x = sx[1] - sx[0], e1y = sy[1] - sy[0], e2x = sx[2] - sx[0], e2y = sy[2] - sy[0];
            const double det = e1x * e2y - e1y * e2x;
            const double f1 = dx[1] - dx[0], f2 = dx[2] - dx[0];
            const double g1 = dy[1] - dy[0], g2 = dy[2] - dy[0];
            M[0] = (f1 * e2y - f2 * e1y) / det;
            M[1] = (e1x * f2 - e2x * f1) / det;
            M[2] = dx[0] - M[0] * sx[0] - M[1] * sy[0];
            M[3] = (g1 * e2y - g2 * e1y) / det;
            M[4] = (e1x * g2 - e2x * g1) / det;
            M[5] = dy[0] - M[3] * sx[0] - M[4] * sy[0];
            M[6] = 0.0;
            M[7] = 0.0;
            M[8] = 1.0;
        } else if (ok) {
            double Qs[9], Qd[9], As[9];
            ok = square_to_quad(sx, sy, Qs) && square_to_quad(dx, dy, Qd);
            if (ok) {
                adjugate(Qs, As);
                double big = 0.0;
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) {
                        double v = 0.0;
                        for (int q = 0; q < 3; ++q) v = fma(Qd[3 * i + q], As[3 * q + j], v);
                        M[3 * i + j] = v;
                        big = fmax(big, fabs(v));
                    }
                ok = fabs(M[8]) > 1e-12 * big && isfinite(big);
                if (ok) {
                    const double inv = 1.0 / M[8];
                    for (int q = 0; q < 9; ++q) M[q] *= inv;
                    M[8] = 1.0;
                }
            }
        }
        if (ok)
            for (int q = 0; q < 9; ++q) a.hyp[(int64_t)h * 9 + q] = M[q];
    }
    if (h < a.n_hyp) a.counts[h] = ok ? 0 : -1;
}

// ---- 3. inlier counts -----------------------------------------------------------
// blockIdx.x: a block of kHypNT hypotheses; blockIdx.y: candidates
// [y * chunk, (y + 1) * chunk).
__global__ __launch_bounds__(kHypNT) void score_kernel(Args a) {
    __shared__ double4 tile[kTile];
    const int h = blockIdx.x * kHypNT + threadIdx.x;
    const int n = *a.ncand;
    const int c0 = blockIdx.y * a.chunk, c1 = min(n, c0 + a.chunk);
    if (c0 >= c1) return;   // uniform over the workgroup
    const bool proj = a.model == SFOC_MODEL_PROJECTIVE;
    const bool ok = h < a.n_hyp && a.counts[h] >= 0;
    double M[9];
    if (ok)
        for (int q = 0; q < 9; ++q) M[q] = a.hyp[(int64_t)h * 9 + q];
    int cnt = 0;
    for (int base = c0; base < c1; base += kTile) {
        const int len = min(kTile, c1 - base);
        __syncthreads();
        for (int e = threadIdx.x; e < len; e += kHypNT) tile[e] = a.cand[base + e];
        __syncthreads();
        if (ok)
            for (int e = 0; e < len; ++e) cnt += inlier(M, proj, tile[e], a.thr_n2);
    }
    if (ok && cnt) atomicAdd(&a.counts[h], cnt);
}

// ---- 4. selection, refinement, flags ---------------------------------------
// Solve A x = b for the NR right-hand sides in b, A symmetric positive
// definite (a normal matrix; only its lower triangle is read), by a
// Cholesky factorisation held in registers (every index is a compile-time
// constant).  False if a squared pivot falls to kSingular times the largest
// diagonal entry or below (the inliers do not determine the model).
template <int N, int NR>
SFOC_DEV bool cholesky_solve(double (&A)[N][N], double (&b)[NR][N]) {
    double big = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) big = fmax(big, A[i][i]);
    if (!(big > 0.0) || !isfinite(big)) return false;
    bool ok = true;
    double invd[N];   // 1 / L[j][j]: the substitutions multiply instead of dividing
#pragma unroll
    for (int j = 0; j < N; ++j) {
        double d = A[j][j];
#pragma unroll
        for (int q = 0; q < j; ++q) d = fma(-A[j][q], A[j][q], d);
        ok = ok && d > kSingular * big;
        const double l = sqrt(fmax(d, kSingular * big));
        const double inv = 1.0 / l;
        invd[j] = inv;
        A[j][j] = l;
#pragma unroll
        for (int i = j + 1; i < N; ++i) {
            double v = A[i][j];
#pragma unroll
            for (int q = 0; q < j; ++q) v = fma(-A[i][q], A[j][q], v);
            A[i][j] = v * inv;
        }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
#pragma unroll
        for (int i = 0; i < N; ++i) {   // L y = b
            double v = b[r][i];
#pragma unroll
            for (int q = 0; q < i; ++q) v = fma(-A[i][q], b[r][q], v);
            b[r][i] = v * invd[i];
        }
#pragma unroll
        for (int i = N - 1; i >= 0; --i) {   // L^T x = y
            double v = b[r][i];
#pragma unroll
            for (int q = i + 1; q < N; ++q) v = fma(-A[q][i], b[r][q], v);
            b[r][i] = v * invd[i];
        }
    }
    return ok;
}

constexpr int kSumsAff = 12, kSumsProj = 44;

// Normal-equation terms of one inlier: affine: the six distinct entries of
// sum [x y 1]^T [x y 1], then sum X [x y 1] and sum Y [x y 1]; projective:
// the 36 distinct entries of A^T A and the 8 of A^T b for the two rows of
// the h22 = 1 system (u = (h0 x + h1 y + h2) - x u h6 - y u h7, same for v).
template <bool PROJ>
SFOC_DEV void terms(double4 c, double* s) {
    const double x = c.x, y = c.y, X = c.z, Y = c.w;
    if (!PROJ) {
        const double v[3] = {x, y, 1.0};
        int o = 0;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = i; j < 3; ++j) s[o++] += v[i] * v[j];
#pragma unroll
        for (int i = 0; i < 3; ++i) s[6 + i] += X * v[i];
#pragma unroll
        for (int i = 0; i < 3; ++i) s[9 + i] += Y * v[i];
    } else {
        const double r1[8] = {x, y, 1.0, 0.0, 0.0, 0.0, -x * X, -y * X};
        const double r2[8] = {0.0, 0.0, 0.0, x, y, 1.0, -x * Y, -y * Y};
        int o = 0;
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int j = i; j < 8; ++j) s[o++] += r1[i] * r1[j] + r2[i] * r2[j];
#pragma unroll
        for (int i = 0; i < 8; ++i) s[36 + i] += r1[i] * X + r2[i] * Y;
    }
}

template <bool PROJ>
__global__ __launch_bounds__(kFinNT) void finish_kernel(Args a) {
    __shared__ double sM[9];
    __shared__ double part[kFinNT / 64][kSumsProj];
    __shared__ int bc[kFinNT / 64], bi[kFinNT / 64], ci[kFinNT / 64];
    __shared__ int flag;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int n = *a.ncand;
    constexpr bool proj = PROJ;
    const int k = a.k;
    // best hypothesis: most inliers, lowest index on ties
    int best = -1, bidx = 0x7fffffff;
    for (int h = t; h < a.n_hyp; h += kFinNT) {
        const int c = a.counts[h];
        if (c > best) {   // increasing h: the first maximum of this thread
            best = c;
            bidx = h;
        }
    }
    for (int d = 32; d >= 1; d >>= 1) {
        const int ob = __shfl_down(best, d, 64), oi = __shfl_down(bidx, d, 64);
        if (ob > best || (ob == best && oi < bidx)) {
            best = ob;
            bidx = oi;
        }
    }
    if (lane == 0) {
        bc[wv] = best;
        bi[wv] = bidx;
    }
    __syncthreads();
    if (t == 0) {
        for (int w = 1; w < kFinNT / 64; ++w)
            if (bc[w] > bc[0] || (bc[w] == bc[0] && bi[w] < bi[0])) {
                bc[0] = bc[w];
                bi[0] = bi[w];
            }
        flag = (n >= k && bc[0] >= 0) ? 1 : 0;
        if (flag)
            for (int q = 0; q < 9; ++q) sM[q] = a.hyp[(int64_t)bi[0] * 9 + q];
    }
    __syncthreads();
    if (!flag) {   // no model: every candidate INCONSISTENT
        for (int j = t; j < n; j += kFinNT) {
            const int i = a.cidx[j];
            a.cps[i].flags = (a.cps_in[i].flags & ~(SFOC_CP_VALID | SFOC_CP_INCONSISTENT)) | SFOC_CP_INCONSISTENT;
        }
        if (t == 0) {
            for (int q = 0; q < 9; ++q) a.model_out[q] = 0.0;
            a.info[0] = n;
            a.info[1] = 0;
            a.info[2] = -1;
            a.info[3] = 1;
        }
        return;
    }
    constexpr int nsum = PROJ ? kSumsProj : kSumsAff;
    int ninl = 0;
    for (int it = 0;; ++it) {
        double M[9];
        for (int q = 0; q < 9; ++q) M[q] = sM[q];
        // inlier set of the current model and its count
        int c = 0;
        for (int j = t; j < n; j += kFinNT) {
            const bool in = inlier(M, proj, a.cand[j], a.thr_n2);
            a.inl[j] = in;
            c += in;
        }
        for (int d = 32; d >= 1; d >>= 1) c += __shfl_down(c, d, 64);
        if (lane == 0) ci[wv] = c;
        __syncthreads();
        ninl = 0;
        for (int w = 0; w < kFinNT / 64; ++w) ninl += ci[w];
        if (it == a.n_refine || ninl < k) break;
        // least squares over the inliers: per-thread sums over a fixed
        // candidate subset, then fixed-order wave and workgroup reductions
        double s[nsum];
#pragma unroll
        for (int q = 0; q < nsum; ++q) s[q] = 0.0;
        for (int j = t; j < n; j += kFinNT)
            if (a.inl[j]) terms<PROJ>(a.cand[j], s);
        // all sums step by step, so each step's shuffles are independent
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1)
#pragma unroll
            for (int q = 0; q < nsum; ++q) s[q] += __shfl_down(s[q], d, 64);
        if (lane == 0)
#pragma unroll
            for (int q = 0; q < nsum; ++q) part[wv][q] = s[q];
        __syncthreads();
        if (t == 0) {
            double tot[nsum];
#pragma unroll
            for (int q = 0; q < nsum; ++q) {
                double v = 0.0;
                for (int w = 0; w < kFinNT / 64; ++w) v += part[w][q];
                tot[q] = v;
            }
            bool good;
            if (!proj) {   // [x y 1] normal matrix, right-hand sides X and Y
                double A[3][3], b[2][3];
                int o = 0;
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = i; j < 3; ++j, ++o) {
                        A[i][j] = tot[o];
                        A[j][i] = tot[o];
                    }
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    b[0][i] = tot[6 + i];
                    b[1][i] = tot[9 + i];
                }
                good = cholesky_solve<3, 2>(A, b);
                if (good) {
                    for (int j = 0; j < 3; ++j) {
                        sM[j] = b[0][j];
                        sM[3 + j] = b[1][j];
                    }
                    sM[6] = 0.0;
                    sM[7] = 0.0;
                    sM[8] = 1.0;
                }
            } else {
                double A[8][8], b[1][8];
                int o = 0;
#pragma unroll
                for (int i = 0; i < 8; ++i)
#pragma unroll
                    for (int j = i; j < 8; ++j, ++o) {
                        A[i][j] = tot[o];
                        A[j][i] = tot[o];
                    }
#pragma unroll
                for (int i = 0; i < 8; ++i) b[0][i] = tot[36 + i];
                good = cholesky_solve<8, 1>(A, b);
                if (good) {
                    for (int i = 0; i < 8; ++i) sM[i] = b[0][i];
                    sM[8] = 1.0;
                }
            }
            flag = good ? 1 : 0;
        }
        __syncthreads();
        if (!flag) {   // singular refit: keep the model whose inliers are in a.inl
            break;
        }
    }
    __syncthreads();
    for (int j = t; j < n; j += kFinNT) {
        const int i = a.cidx[j];
        a.cps[i].flags = (a.cps_in[i].flags & ~(SFOC_CP_VALID | SFOC_CP_INCONSISTENT)) |
                         (a.inl[j] ? SFOC_CP_VALID : SFOC_CP_INCONSISTENT);
    }
    if (t == 0) {
        // pixels: P = Tr^-1 M Ts with Ts = [[s, 0, -cr s], [0, s, -cc s], [0, 0, 1]]
        // for the sensed image and Tr^-1 = [[1/s, 0, cr], [0, 1/s, cc], [0, 0, 1]]
        // for the reference; scaled so that P[2][2] = 1.
        const double Ts[9] = {a.ns.s, 0.0, -a.ns.cr * a.ns.s, 0.0, a.ns.s, -a.ns.cc * a.ns.s, 0.0, 0.0, 1.0};
        const double Ti[9] = {1.0 / a.nr.s, 0.0, a.nr.cr, 0.0, 1.0 / a.nr.s, a.nr.cc, 0.0, 0.0, 1.0};
        double A[9], P[9];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double v = 0.0;
                for (int q = 0; q < 3; ++q) v += sM[3 * i + q] * Ts[3 * q + j];
                A[3 * i + j] = v;
            }
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double v = 0.0;
                for (int q = 0; q < 3; ++q) v += Ti[3 * i + q] * A[3 * q + j];
                P[3 * i + j] = v;
            }
        const double inv = 1.0 / P[8];
        for (int q = 0; q < 9; ++q) a.model_out[q] = P[q] * inv;
        a.model_out[8] = 1.0;
        a.info[0] = n;
        a.info[1] = ninl;
        a.info[2] = bi[0];
        a.info[3] = 0;
    }
}

struct Layout {
    size_t cand, cidx, ncand, inl, counts, hyp, total;
};
Layout layout(int n, int n_hyp) {
    Layout L;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += align_up(bytes, 256);
        return at;
    };
    L.cand = take(sizeof(double4) * (size_t)std::max(n, 1));
    L.cidx = take(sizeof(int) * (size_t)std::max(n, 1));
    L.ncand = take(sizeof(int));
    L.inl = take((size_t)std::max(n, 1));
    L.counts = take(sizeof(int) * (size_t)n_hyp);
    L.hyp = take(sizeof(double) * 9 * (size_t)n_hyp);
    L.total = o;
    return L;
}

int check(int n, const sfoc_ransac_params* p) {
    if (!p || n < 0) return SFOC_E_INVALID_ARG;
    if (p->model != SFOC_MODEL_AFFINE && p->model != SFOC_MODEL_PROJECTIVE) return SFOC_E_INVALID_ARG;
    if (p->n_hyp < 1 || p->n_refine < 0 || p->n_refine > kMaxRefine) return SFOC_E_INVALID_ARG;
    if (!(p->threshold > 0.0) || !isfinite(p->threshold)) return SFOC_E_INVALID_ARG;
    if (p->Hs < 1 || p->Ws < 1 || p->Hr < 1 || p->Wr < 1) return SFOC_E_INVALID_ARG;
    if (n > kMaxN || p->n_hyp > kMaxHyp) return SFOC_E_UNSUPPORTED;
    return SFOC_OK;
}

}  // namespace ransac
}  // namespace sfoc

using namespace sfoc;

extern "C" int sfoc_ransac_workspace(int32_t n, const sfoc_ransac_params* p, size_t* bytes) {
    const int rc = ransac::check(n, p);
    if (rc != SFOC_OK) return rc;
    if (!bytes) return SFOC_E_INVALID_ARG;
    *bytes = ransac::layout(n, p->n_hyp).total;
    return SFOC_OK;
}

extern "C" int sfoc_ransac_cps(sfoc_cp* cps, const int32_t* prior, int32_t n, const uint32_t* words,
                               const sfoc_ransac_params* p, void* ws, size_t ws_bytes, double* model,
                               int32_t* info, int32_t* counts, double* hyp_models, void* stream) {
    using namespace ransac;
    const int rc = check(n, p);
    if (rc != SFOC_OK) return rc;
    if ((n > 0 && !cps) || !words || !ws || !model || !info) return SFOC_E_INVALID_ARG;
    const Layout L = layout(n, p->n_hyp);
    if (ws_bytes < L.total) return SFOC_E_WORKSPACE;
    char* w = (char*)ws;
    auto norm = [](int H, int W) {
        Norm q;
        q.cr = 0.5 * (H - 1);
        q.cc = 0.5 * (W - 1);
        q.s = 1.0 / (0.5 * (double)std::max(H, W));
        return q;
    };
    Args a;
    a.cps_in = cps;
    a.cps = cps;
    a.prior = prior;
    a.n = n;
    a.ns = norm(p->Hs, p->Ws);
    a.nr = norm(p->Hr, p->Wr);
    a.s_ref = 0.5 * (double)std::max(p->Hr, p->Wr);
    const double tn = p->threshold / a.s_ref;
    a.thr_n2 = tn * tn;
    a.model = p->model;
    a.k = p->model == SFOC_MODEL_AFFINE ? 3 : 4;
    a.n_hyp = p->n_hyp;
    a.n_refine = p->n_refine;
    a.words = words;
    a.cand = (double4*)(w + L.cand);
    a.cidx = (int*)(w + L.cidx);
    a.ncand = (int*)(w + L.ncand);
    a.inl = (uint8_t*)(w + L.inl);
    a.counts = counts ? counts : (int*)(w + L.counts);
    a.hyp = hyp_models ? hyp_models : (double*)(w + L.hyp);
    a.model_out = model;
    a.info = info;
    hipStream_t st = (hipStream_t)stream;
    trace_begin(st, SFOC_K_RANSAC);
    hipLaunchKernelGGL(prepare_kernel, dim3(1), dim3(kPrepNT), 0, st, a);
    const int hblocks = (p->n_hyp + kHypNT - 1) / kHypNT;
    const int chunks = std::max(1, std::min(std::max(1, kScoreBlocks / hblocks), (n + kMinChunk - 1) / kMinChunk));
    a.chunk = std::max(1, (n + chunks - 1) / chunks);
    hipLaunchKernelGGL(fit_kernel, dim3(hblocks), dim3(kHypNT), 0, st, a);
    hipLaunchKernelGGL(score_kernel, dim3(hblocks, chunks), dim3(kHypNT), 0, st, a);
    if (p->model == SFOC_MODEL_PROJECTIVE)
        hipLaunchKernelGGL(finish_kernel<true>, dim3(1), dim3(kFinNT), 0, st, a);
    else
        hipLaunchKernelGGL(finish_kernel<false>, dim3(1), dim3(kFinNT), 0, st, a);
    trace_end(st, SFOC_K_RANSAC);
    return hip_status(hipGetLastError());
}
