// Fast-NCC_SFOC CP detection (Section 2.2, Eq. 9-16; Section 3.2.2) on gfx950.
//
// One workgroup per interest point.  For each descriptor channel h the
// template T_h (m x m, zero padded) and the search window S_h (M x M) get a
// real 2-D FFT of side L >= M in LDS:
//   rows    : two real rows packed as one complex row, in-place radix-2^2
//             decimation-in-time FFT over bit-reversed input;
//   unpack  : the two row spectra separated with the conjugate-symmetry
//             identity into the half spectrum k2 = 0..L/2, transposed so
//             that columns are contiguous;
//   columns : the same FFT along the rows' axis.
// The template spectrum is kept in registers and the product
// F(S_h) conj(F(T_h)) is accumulated over channels in registers (summing in
// the spectrum is exact by linearity, so only one inverse is needed, Eq. 13).
// The inverse runs columns first, then rows packed in pairs, giving R_ST on
// the (2r+1)^2 valid offsets.  R_S and R_SS come from four lookups in the
// float64 integral images of the reference descriptor (Eq. 16); R_T and R_TT
// are accumulated in float64 while the template is read.  The NCC of Eq. 9
// is assembled with the variance subtraction in float64, then the argmax,
// the parabola refinement and the per-CP flags are written.
#include "sfoc_dev.h"
#include "sfoc_plan.h"
#include "sfoc_trace.h"

namespace sfoc {

struct MatchArgs {
    const void* desc_sen;
    const void* desc_ref;
    const double* integ1;
    const double* integ2;
    const int32_t* ips;
    const int32_t* prior;
    float* ncc;
    sfoc_cp* cps;
    int64_t Hs, Ws, Hr, Wr;
    int32_t z, dtype, n, m, r;
};

SFOC_DEV float2 cmul(float2 a, float2 b) { return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
SFOC_DEV float2 cmulc(float2 a, float2 b) {  // a * conj(b)
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
SFOC_DEV float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
SFOC_DEV float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

template <int LOG>
SFOC_DEV int bitrev(int i) {
    return (int)(__brev((unsigned)i) >> (32 - LOG));
}

// In-place DIT FFT of nb transforms of length L (input bit-reversed, output
// natural order), transform b at buf + b * pitch.  tw[k] = exp(-2 pi i k / L);
// inverse uses conj(tw) (no 1/L scaling).  Two radix-2 stages per LDS pass.
template <int L, int NT>
SFOC_DEV void fft_inplace(float2* buf, int nb, int pitch, const float2* tw, bool inverse) {
    constexpr int LOG = __builtin_ctz(L);
    const float sg = inverse ? -1.f : 1.f;
    int s = 0;
    for (; s + 1 < LOG; s += 2) {
        const int h = 1 << s;
        const int tot = nb * (L / 4);
        for (int e = threadIdx.x; e < tot; e += NT) {
            const int b = e / (L / 4), q = e - b * (L / 4);
            const int blk = q >> s, j = q & (h - 1);
            float2* p = buf + b * pitch + blk * 4 * h + j;
            float2 x0 = p[0], x1 = p[h], x2 = p[2 * h], x3 = p[3 * h];
            float2 w = tw[j * (L / (2 * h))];
            w.y *= sg;
            float2 t = cmul(w, x1);
            float2 a0 = cadd(x0, t), a1 = csub(x0, t);
            t = cmul(w, x3);
            float2 a2 = cadd(x2, t), a3 = csub(x2, t);
            float2 w2 = tw[j * (L / (4 * h))];
            w2.y *= sg;
            float2 w3 = tw[(j + h) * (L / (4 * h))];
            w3.y *= sg;
            t = cmul(w2, a2);
            p[0] = cadd(a0, t);
            p[2 * h] = csub(a0, t);
            t = cmul(w3, a3);
            p[h] = cadd(a1, t);
            p[3 * h] = csub(a1, t);
        }
        __syncthreads();
    }
    if (s < LOG) {
        const int h = 1 << s;
        const int tot = nb * (L / 2);
        for (int e = threadIdx.x; e < tot; e += NT) {
            const int b = e / (L / 2), q = e - b * (L / 2);
            const int blk = q >> s, j = q & (h - 1);
            float2* p = buf + b * pitch + blk * 2 * h + j;
            float2 x0 = p[0], x1 = p[h];
            float2 w = tw[j * (L / (2 * h))];
            w.y *= sg;
            const float2 t = cmul(w, x1);
            p[0] = cadd(x0, t);
            p[h] = csub(x0, t);
        }
        __syncthreads();
    }
}

template <int L, int NT>
struct MatchCfg {
    static constexpr int LOG = __builtin_ctz(L);
    static constexpr int H2 = L / 2 + 1;          // half-spectrum columns
    static constexpr int CP = L + 1;              // column-buffer pitch (float2)
    static constexpr int NBIN = H2 * L;           // spectrum bins kept
    static constexpr int NB = (NBIN + NT - 1) / NT;
    static constexpr size_t lds_bytes = sizeof(float2) * ((size_t)L + (size_t)(L / 2) * L + (size_t)H2 * CP) + 1024;
};

// Real 2-D FFT of rows [0, nrows) x cols [0, ncols) of one descriptor
// channel, zero padded to L x L, into colbuf (layout [k2][k1], pitch CP).
template <int L, int NT>
SFOC_DEV void real_fft2(const void* desc, int dt, int64_t plane_off, int64_t pitch, int y0, int x0, int nrows,
                        int ncols, float2* rowbuf, float2* colbuf, const float2* tw, double* s1, double* s2) {
    using C = MatchCfg<L, NT>;
    const int npair = (nrows + 1) / 2;
    // rows: load (coalesced along x), pack two rows per complex row, bit reverse.
    for (int e = threadIdx.x; e < npair * L; e += NT) {
        const int p = e / L, b = e - p * L;
        float re = 0.f, im = 0.f;
        if (b < ncols) {
            const int64_t base = plane_off + (int64_t)(y0 + 2 * p) * pitch + x0 + b;
            re = load_desc(desc, base, dt);
            if (2 * p + 1 < nrows) im = load_desc(desc, base + pitch, dt);
            if (s1) {
                const double dr = re, di = im;
                *s1 += dr + di;
                *s2 += dr * dr + di * di;
            }
        }
        rowbuf[p * L + bitrev<C::LOG>(b)] = make_float2(re, im);
    }
    __syncthreads();
    fft_inplace<L, NT>(rowbuf, npair, L, tw, false);
    // unpack the two real-row spectra, transpose to columns, bit reverse rows.
    for (int e = threadIdx.x; e < C::H2 * L; e += NT) {
        const int row = e / C::H2, k2 = e - row * C::H2;
        float2 v = make_float2(0.f, 0.f);
        if (row < 2 * npair) {
            const int p = row >> 1;
            const float2 za = rowbuf[p * L + k2];
            float2 zb = rowbuf[p * L + ((L - k2) & (L - 1))];
            zb.y = -zb.y;
            if ((row & 1) == 0) v = make_float2(0.5f * (za.x + zb.x), 0.5f * (za.y + zb.y));
            else v = make_float2(0.5f * (za.y - zb.y), -0.5f * (za.x - zb.x));   // -i (za - zb) / 2
        }
        colbuf[k2 * C::CP + bitrev<C::LOG>(row)] = v;
    }
    __syncthreads();
    fft_inplace<L, NT>(colbuf, C::H2, C::CP, tw, false);
}

SFOC_DEV bool in_image(int64_t y, int64_t x, int h, int w, int64_t H, int64_t W) {
    return y >= 0 && x >= 0 && y + h <= H && x + w <= W;
}

template <int L, int NT>
__global__ __launch_bounds__(NT) void match_kernel(const MatchArgs A) {
    using C = MatchCfg<L, NT>;
    extern __shared__ float4 lds_raw[];
    float2* tw = reinterpret_cast<float2*>(lds_raw);
    float2* rowbuf = tw + L;
    float2* colbuf = rowbuf + (L / 2) * L;
    double* red = reinterpret_cast<double*>(colbuf + C::H2 * C::CP);   // 1 KB scratch

    const int i = blockIdx.x;
    const int t = threadIdx.x;
    const int m = A.m, r = A.r, M = m + 2 * r, V = 2 * r + 1;
    const int py = A.ips[2 * i], px = A.ips[2 * i + 1];
    const int pry = A.prior ? A.prior[2 * i] : 0, prx = A.prior ? A.prior[2 * i + 1] : 0;
    const int64_t ty = (int64_t)py - m / 2, tx = (int64_t)px - m / 2;
    const int64_t sy = ty - r + pry, sx = tx - r + prx;
    sfoc_cp out;
    out.sen_row = py;
    out.sen_col = px;
    out.dy = out.dx = 0;
    out.sub_dy = out.sub_dx = 0.f;
    out.score = 0.f;
    out.flags = 0;
    if (!in_image(ty, tx, m, m, A.Hs, A.Ws) || !in_image(sy, sx, M, M, A.Hr, A.Wr)) {
        if (t == 0) {
            out.flags = SFOC_CP_OOB;
            A.cps[i] = out;
        }
        if (A.ncc)
            for (int e = t; e < V * V; e += NT) A.ncc[(int64_t)i * V * V + e] = 0.f;
        return;
    }
    for (int k = t; k < L; k += NT) {
        float sn, cs;
        sincospif(-2.0f * (float)k / (float)L, &sn, &cs);
        tw[k] = make_float2(cs, sn);
    }
    __syncthreads();

    float2 ysp[C::NB];   // template spectrum of the current channel
    float2 acc[C::NB];   // sum over channels of F(S_h) conj(F(T_h))
#pragma unroll
    for (int j = 0; j < C::NB; ++j) acc[j] = make_float2(0.f, 0.f);
    double s1 = 0.0, s2 = 0.0;
    const int64_t plane_s = A.Hs * A.Ws, plane_r = A.Hr * A.Wr;
    for (int h = 0; h < A.z; ++h) {
        real_fft2<L, NT>(A.desc_sen, A.dtype, h * plane_s, A.Ws, (int)ty, (int)tx, m, m, rowbuf, colbuf, tw, &s1, &s2);
#pragma unroll
        for (int j = 0; j < C::NB; ++j) {
            const int e = t + j * NT;
            if (e < C::NBIN) {
                const int k2 = e / L, k1 = e - k2 * L;
                ysp[j] = colbuf[k2 * C::CP + k1];
            }
        }
        __syncthreads();
        real_fft2<L, NT>(A.desc_ref, A.dtype, h * plane_r, A.Wr, (int)sy, (int)sx, M, M, rowbuf, colbuf, tw, nullptr,
                         nullptr);
#pragma unroll
        for (int j = 0; j < C::NB; ++j) {
            const int e = t + j * NT;
            if (e < C::NBIN) {
                const int k2 = e / L, k1 = e - k2 * L;
                const float2 xs = colbuf[k2 * C::CP + k1];
                const float2 pr = cmulc(xs, ysp[j]);
                acc[j] = cadd(acc[j], pr);
            }
        }
        __syncthreads();
    }

    // template sums R_T, R_TT (Eq. 12): block reduction in float64.
    {
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
    const double RT = red[64], RTT = red[65];
    const double mnz = (double)m * m * A.z;
    const double tau = 1e-12 * mnz;
    const double varT = RTT - RT * RT / mnz;

    // inverse: columns (k1 -> u) for k2 = 0..L/2, then rows (k2 -> v) in pairs.
#pragma unroll
    for (int j = 0; j < C::NB; ++j) {
        const int e = t + j * NT;
        if (e < C::NBIN) {
            const int k2 = e / L, k1 = e - k2 * L;
            colbuf[k2 * C::CP + bitrev<C::LOG>(k1)] = acc[j];
        }
    }
    __syncthreads();
    fft_inplace<L, NT>(colbuf, C::H2, C::CP, tw, true);
    const int vpair = (V + 1) / 2;
    for (int e = t; e < vpair * L; e += NT) {
        const int p = e / L, k2 = e - p * L;
        const int u0 = 2 * p, u1 = 2 * p + 1;
        float2 ha, hb;
        if (k2 <= L / 2) {
            ha = colbuf[k2 * C::CP + u0];
            hb = colbuf[k2 * C::CP + u1];
        } else {
            ha = colbuf[(L - k2) * C::CP + u0];
            hb = colbuf[(L - k2) * C::CP + u1];
            ha.y = -ha.y;
            hb.y = -hb.y;
        }
        rowbuf[p * L + bitrev<C::LOG>(k2)] = make_float2(ha.x - hb.y, ha.y + hb.x);
    }
    __syncthreads();
    fft_inplace<L, NT>(rowbuf, vpair, L, tw, true);

    // NCC (Eq. 9) with integral-image box sums (Eq. 16), float64 variance.
    float* surf = reinterpret_cast<float*>(colbuf);
    const float inv = 1.0f / ((float)L * (float)L);
    const int64_t IW = A.Wr + 1;
    int nonflat = 0, nonfin = 0;
    float best = -INFINITY;
    int bidx = 0x7fffffff;
    const bool flatT = !(varT > tau);
    const bool badT = !isfinite(RT) || !isfinite(RTT);
    for (int e = t; e < V * V; e += NT) {
        const int u = e / V, v = e - u * V;
        const float2 rr = rowbuf[(u >> 1) * L + v];
        const float rst = ((u & 1) ? rr.y : rr.x) * inv;
        const int64_t y = sy + u, x = sx + v;
        const int64_t a00 = y * IW + x, a01 = a00 + m, a10 = a00 + (int64_t)m * IW, a11 = a10 + m;
        const double RS = A.integ1[a11] - A.integ1[a10] - A.integ1[a01] + A.integ1[a00];
        const double RSS = A.integ2[a11] - A.integ2[a10] - A.integ2[a01] + A.integ2[a00];
        const double varS = RSS - RS * RS / mnz;
        float val = 0.f;
        if (!isfinite(rst) || !isfinite(RS) || !isfinite(varS)) nonfin = 1;
        if (varS > tau && !flatT) {
            nonflat = 1;
            const double num = (double)rst - RS * RT / mnz;
            val = (float)(num / sqrt(varS * varT));
        }
        surf[e] = val;
        if (val > best) {   // strictly greater: the first index wins ties
            best = val;
            bidx = e;
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
    if (A.ncc)
        for (int e = t; e < V * V; e += NT) A.ncc[(int64_t)i * V * V + e] = surf[e];
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
                const float c0 = surf[bidx];
                const float cu = surf[bidx - V], cd = surf[bidx + V];
                const float cl = surf[bidx - 1], cr = surf[bidx + 1];
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

// k-th smallest (0-based) displacement along axis over eligible CPs.
SFOC_DEV float select_kth(const sfoc_cp* cps, const int32_t* prior, int n, int axis, int k, uint32_t* hist,
                          uint32_t* shared_sel) {
    uint32_t prefix = 0, mask = 0;
    for (int shift = 24; shift >= 0; shift -= 8) {
        for (int b = threadIdx.x; b < 256; b += kConsNT) hist[b] = 0;
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += kConsNT) {
            const sfoc_cp c = cps[i];
            if (c.flags & kBad) continue;
            const uint32_t key = fkey(cp_disp(c, prior, i, axis));
            if ((key & mask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t cum = 0;
            int b = 0;
            for (; b < 256; ++b) {
                if (cum + hist[b] > (uint32_t)k) break;
                cum += hist[b];
            }
            shared_sel[0] = (uint32_t)b;
            shared_sel[1] = cum;
        }
        __syncthreads();
        const uint32_t b = shared_sel[0];
        k -= (int)shared_sel[1];
        prefix |= b << shift;
        mask |= 255u << shift;
        __syncthreads();
    }
    return fkey_inv(prefix);
}

__global__ __launch_bounds__(kConsNT) void consistency_kernel(sfoc_cp* cps, const int32_t* prior, int n) {
    __shared__ uint32_t hist[256];
    __shared__ uint32_t sel[2];
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    int local = 0;
    for (int i = threadIdx.x; i < n; i += kConsNT)
        if (!(cps[i].flags & kBad)) ++local;
    atomicAdd(&cnt, local);
    __syncthreads();
    const int ne = cnt;
    if (ne == 0) return;
    float med[2];
    for (int axis = 0; axis < 2; ++axis) {
        if (ne & 1) {
            med[axis] = select_kth(cps, prior, n, axis, ne / 2, hist, sel);
        } else {
            const float a = select_kth(cps, prior, n, axis, ne / 2 - 1, hist, sel);
            const float b = select_kth(cps, prior, n, axis, ne / 2, hist, sel);
            med[axis] = 0.5f * (a + b);
        }
    }
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

// ---- launch -------------------------------------------------------------
template <int L, int NT>
static hipError_t launch_match_L(const MatchArgs& a, hipStream_t st) {
    using C = MatchCfg<L, NT>;
    auto kern = match_kernel<L, NT>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)C::lds_bytes);
    if (e != hipSuccess) return e;
    trace_begin(st, SFOC_K_MATCH);
    hipLaunchKernelGGL(kern, dim3(a.n), dim3(NT), C::lds_bytes, st, a);
    trace_end(st, SFOC_K_MATCH);
    return hipGetLastError();
}

hipError_t launch_match(const void* desc_sen, int64_t Hs, int64_t Ws, const void* desc_ref, int64_t Hr, int64_t Wr,
                        const double* i1, const double* i2, int z, int dtype, const int32_t* ips,
                        const int32_t* prior, int n, int m, int r, float* ncc, sfoc_cp* cps, hipStream_t st) {
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
    const int L = fft_size_for(m + 2 * r);
    hipError_t e;
    if (L == 64) e = launch_match_L<64, 256>(a, st);
    else if (L == 128) e = launch_match_L<128, 512>(a, st);
    else return hipErrorInvalidValue;
    if (e != hipSuccess) return e;
    trace_begin(st, SFOC_K_CONSISTENCY);
    hipLaunchKernelGGL(consistency_kernel, dim3(1), dim3(kConsNT), 0, st, cps, prior, n);
    trace_end(st, SFOC_K_CONSISTENCY);
    return hipGetLastError();
}

}  // namespace sfoc
