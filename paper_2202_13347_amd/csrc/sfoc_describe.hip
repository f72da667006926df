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
#include "sfoc_plan.h"
#include "sfoc_trace.h"

namespace sfoc {

constexpr int kTS = 32;       // output tile side
constexpr int kNT = 256;      // threads per tile
constexpr int kPXT = kTS * kTS / kNT;

struct DescribeLds {
    int BS, IS, rowN;     // basis side, image-region side, row-buffer rows (max)
    int off_img, off_row, off_basis, off_chan;
    size_t bytes;
};

static DescribeLds describe_lds(const DescribeConsts& c, int CG) {
    DescribeLds L;
    L.BS = kTS + 2 * c.Q;
    L.IS = L.BS + 2 * c.R;
    L.rowN = L.BS + 2 * c.R;
    L.off_img = 0;
    L.off_row = L.IS * L.IS;
    L.off_basis = L.off_row + 3 * L.rowN * L.BS;
    L.off_chan = 0;   // aliases img + row once the basis is complete
    int need = L.off_basis + 5 * L.BS * L.BS;
    L.bytes = (size_t)need * sizeof(float);
    (void)CG;
    return L;
}

template <int Z, int CG>
__global__ __launch_bounds__(kNT) void describe_kernel(const float* __restrict__ img, int H, int W, int64_t ld,
                                                       void* __restrict__ desc, double* __restrict__ integ1,
                                                       double* __restrict__ integ2, const DescribeConsts C,
                                                       int BS, int IS) {
    extern __shared__ float lds[];
    const int t = threadIdx.x;
    const int ty0 = blockIdx.y * kTS, tx0 = blockIdx.x * kTS;
    const int Q = C.Q, R = C.R;
    const int rowN = BS + 2 * R;
    float* simg = lds;
    float* srow = lds + IS * IS;
    float* sbas = srow + 3 * rowN * BS;
    const int BB = BS * BS;

    // 1. input region with reflect-101 borders.
    for (int e = t; e < IS * IS; e += kNT) {
        const int a = e / IS, b = e - a * IS;
        const int gy = reflect101(ty0 - Q - R + a, H);
        const int gx = reflect101(tx0 - Q - R + b, W);
        simg[e] = img[(int64_t)gy * ld + gx];
    }
    for (int e = t; e < 5 * BB; e += kNT) sbas[e] = 0.f;
    __syncthreads();

    // 2. basis responses summed over sigma.
    for (int s = 0; s < C.nsig; ++s) {
        const int rho = C.rad[s];
        const float* tg = C.taps + C.off[s];
        const float* td = tg + (rho + 1);
        const float* tdd = td + (rho + 1);
        const float cn = C.cnorm[s];
        const int rows = BS + 2 * rho;
        // row pass: correlation form of the convolution; odd taps flip sign.
        for (int e = t; e < rows * BS; e += kNT) {
            const int a = e / BS, b = e - a * BS;
            const float* p = simg + (a + R - rho) * IS + (b + R);
            const float x0 = p[0];
            float ag = tg[0] * x0, add = tdd[0] * x0, ad = 0.f;
            for (int k = 1; k <= rho; ++k) {
                const float xp = p[k], xm = p[-k];
                const float sm = xp + xm, df = xm - xp;
                ag = fmaf(tg[k], sm, ag);
                add = fmaf(tdd[k], sm, add);
                ad = fmaf(td[k], df, ad);
            }
            srow[e] = cn * ag;
            srow[rows * BS + e] = cn * ad;
            srow[2 * rows * BS + e] = cn * add;
        }
        __syncthreads();
        const float* rg = srow;
        const float* rd = srow + rows * BS;
        const float* rdd = srow + 2 * rows * BS;
        const int use = C.use[s];
        for (int e = t; e < BB; e += kNT) {
            const int a = e / BS, b = e - a * BS;
            const int c0 = (a + rho) * BS + b;
            float bx = tg[0] * rd[c0], by = 0.f;
            float bxx = tg[0] * rdd[c0], byy = tdd[0] * rg[c0], bxy = 0.f;
            for (int k = 1; k <= rho; ++k) {
                const int up = c0 - k * BS, dn = c0 + k * BS;
                const float gs = rg[up] + rg[dn], gdf = rg[up] - rg[dn];
                const float ds = rd[up] + rd[dn], ddf = rd[up] - rd[dn];
                const float dds = rdd[up] + rdd[dn];
                bx = fmaf(tg[k], ds, bx);
                by = fmaf(td[k], gdf, by);
                bxx = fmaf(tg[k], dds, bxx);
                byy = fmaf(tdd[k], gs, byy);
                bxy = fmaf(td[k], ddf, bxy);
            }
            if (use & 1) {
                sbas[e] += bx;
                sbas[BB + e] += by;
            }
            if (use & 2) {
                sbas[2 * BB + e] += bxx;
                sbas[3 * BB + e] += byy;
                sbas[4 * BB + e] += bxy;
            }
        }
        __syncthreads();
    }

    // 3. steer + rectify per channel group, then dilated smoothing.
    float acc[Z][kPXT];
    float* schan = lds;   // img/row regions are free now
    const int N = C.N;
    const int B = 2 * C.K + 1;
#pragma unroll
    for (int c0 = 0; c0 < Z; c0 += CG) {
        for (int e = t; e < BB; e += kNT) {
#pragma unroll
            for (int cc = 0; cc < CG; ++cc) {
                const int c = c0 + cc;
                if (c < Z) {
                    float v;
                    if (c < N) {
                        v = C.c1[c] * sbas[e] + C.s1[c] * sbas[BB + e];
                    } else {
                        const int k = c - N;
                        v = C.cc[k] * sbas[2 * BB + e] + C.ss[k] * sbas[3 * BB + e] + C.sc2[k] * sbas[4 * BB + e];
                    }
                    if (C.rectify == SFOC_RECTIFY_ABS) v = fabsf(v);
                    else if (C.rectify == SFOC_RECTIFY_RELU) v = fmaxf(v, 0.f);
                    schan[cc * BB + e] = v;
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int px = 0; px < kPXT; ++px) {
            const int oy = t / kTS + px * (kNT / kTS), ox = t % kTS;
            const int base = (oy + Q) * BS + ox + Q;
#pragma unroll
            for (int cc = 0; cc < CG; ++cc) {
                const int c = c0 + cc;
                if (c < Z) {
                    const float* w = (c < N) ? C.w1 : C.w2;
                    const float* ch = schan + cc * BB + base;
                    float a = 0.f;
                    for (int di = 0; di < C.ndil; ++di) {
                        const int r = C.dil[di];
                        for (int i = 0; i < B; ++i)
                            for (int j = 0; j < B; ++j)
                                a = fmaf(w[i * B + j], ch[(i - C.K) * r * BS + (j - C.K) * r], a);
                    }
                    acc[c][px] = a;
                }
            }
        }
        __syncthreads();
    }

    // 4. per-order normalisation, rounding, store, channel sums.
    const int64_t plane = (int64_t)H * W;
    const int nord = C.second ? 2 : 1;
#pragma unroll
    for (int px = 0; px < kPXT; ++px) {
        const int oy = t / kTS + px * (kNT / kTS), ox = t % kTS;
        const int gy = ty0 + oy, gx = tx0 + ox;
        float inv[2];
        for (int o = 0; o < 2; ++o) {
            float s2 = 0.f;
#pragma unroll
            for (int c = 0; c < Z; ++c)
                if ((c < N) == (o == 0)) s2 = fmaf(acc[c][px], acc[c][px], s2);
            inv[o] = 1.0f / sqrtf(s2 + C.eps);
        }
        (void)nord;
        if (gy < H && gx < W) {
            const int64_t o = (int64_t)gy * W + gx;
            double d1 = 0.0, d2 = 0.0;
#pragma unroll
            for (int c = 0; c < Z; ++c) {
                float v = acc[c][px] * inv[c < N ? 0 : 1];
                if (C.dtype == SFOC_DTYPE_F32) {
                    ((float*)desc)[c * plane + o] = v;
                } else if (C.dtype == SFOC_DTYPE_BF16) {
                    const uint16_t b = f32_to_bf16_bits(v);
                    ((uint16_t*)desc)[c * plane + o] = b;
                    v = bf16_bits_to_f32(b);
                } else {
                    const uint16_t b = f32_to_f16_bits(v);
                    ((uint16_t*)desc)[c * plane + o] = b;
                    v = f16_bits_to_f32(b);
                }
                const double dv = (double)v;
                d1 += dv;
                d2 = fma(dv, dv, d2);
            }
            if (integ1) {
                const int64_t io = (int64_t)(gy + 1) * (W + 1) + gx + 1;
                integ1[io] = d1;
                integ2[io] = d2;
            }
        }
    }
}

// ---- integral images (Eq. 15 as two scans) -----------------------------
// Row pass: in place, inclusive prefix along each row 1..H of the
// (H+1) x (W+1) image, column 0 and row 0 set to zero.
constexpr int kScanNT = 256;
constexpr int kScanPer = 8;

__global__ __launch_bounds__(kScanNT) void integral_row_scan(double* __restrict__ g1, double* __restrict__ g2,
                                                              int H, int W) {
    __shared__ double sh[2][kScanNT * kScanPer];
    __shared__ double wsum[2][kScanNT / 64];
    const int y = blockIdx.x;  // 0..H
    const int t = threadIdx.x;
    const int64_t rowoff = (int64_t)y * (W + 1);
    if (y == 0) {
        for (int x = t; x <= W; x += kScanNT) {
            g1[x] = 0.0;
            g2[x] = 0.0;
        }
        return;
    }
    double carry[2] = {0.0, 0.0};
    if (t == 0) {
        g1[rowoff] = 0.0;
        g2[rowoff] = 0.0;
    }
    const int seg = kScanNT * kScanPer;
    for (int x0 = 1; x0 <= W; x0 += seg) {
        for (int q = 0; q < 2; ++q) {
            double* g = q ? g2 : g1;
            for (int i = 0; i < kScanPer; ++i) {
                const int e = i * kScanNT + t;
                const int x = x0 + e;
                sh[q][e] = x <= W ? g[rowoff + x] : 0.0;
            }
        }
        __syncthreads();
        double tot[2];
        for (int q = 0; q < 2; ++q) {
            double s = 0.0;
            for (int i = 0; i < kScanPer; ++i) {
                s += sh[q][t * kScanPer + i];
                sh[q][t * kScanPer + i] = s;
            }
            tot[q] = s;
        }
        // inclusive scan of per-thread totals within the wave
        const int lane = t & 63, wv = t >> 6;
        for (int q = 0; q < 2; ++q) {
            double v = tot[q];
            for (int d = 1; d < 64; d <<= 1) {
                const double u = __shfl_up(v, d, 64);
                if (lane >= d) v += u;
            }
            if (lane == 63) wsum[q][wv] = v;
            const double ex = __shfl_up(v, 1, 64);
            tot[q] = lane == 0 ? 0.0 : ex;   // exclusive within wave
        }
        __syncthreads();
        for (int q = 0; q < 2; ++q) {
            double pre = carry[q];
            for (int w = 0; w < wv; ++w) pre += wsum[q][w];
            const double add = pre + tot[q];
            for (int i = 0; i < kScanPer; ++i) sh[q][t * kScanPer + i] += add;
            double all = carry[q];
            for (int w = 0; w < kScanNT / 64; ++w) all += wsum[q][w];
            carry[q] = all;
        }
        __syncthreads();
        for (int q = 0; q < 2; ++q) {
            double* g = q ? g2 : g1;
            for (int i = 0; i < kScanPer; ++i) {
                const int e = i * kScanNT + t;
                const int x = x0 + e;
                if (x <= W) g[rowoff + x] = sh[q][e];
            }
        }
        __syncthreads();
    }
}

// Column pass, phase 1: per block of kScanRows rows, the column totals.
__global__ __launch_bounds__(kScanNT) void integral_col_blocksum(const double* __restrict__ g1,
                                                                  const double* __restrict__ g2, int H, int W,
                                                                  double* __restrict__ bs1, double* __restrict__ bs2) {
    const int x = blockIdx.x * kScanNT + threadIdx.x;
    const int b = blockIdx.y;
    if (x > W) return;
    const int y0 = 1 + b * kScanRows, y1 = min(H, y0 + kScanRows - 1);
    double s1 = 0.0, s2 = 0.0;
    for (int y = y0; y <= y1; ++y) {
        s1 += g1[(int64_t)y * (W + 1) + x];
        s2 += g2[(int64_t)y * (W + 1) + x];
    }
    bs1[(int64_t)b * (W + 1) + x] = s1;
    bs2[(int64_t)b * (W + 1) + x] = s2;
}

// Column pass, phase 2: carry from the blocks above, then the in-block scan.
__global__ __launch_bounds__(kScanNT) void integral_col_apply(double* __restrict__ g1, double* __restrict__ g2,
                                                               int H, int W, const double* __restrict__ bs1,
                                                               const double* __restrict__ bs2) {
    const int x = blockIdx.x * kScanNT + threadIdx.x;
    const int b = blockIdx.y;
    if (x > W) return;
    double c1 = 0.0, c2 = 0.0;
    for (int q = 0; q < b; ++q) {
        c1 += bs1[(int64_t)q * (W + 1) + x];
        c2 += bs2[(int64_t)q * (W + 1) + x];
    }
    const int y0 = 1 + b * kScanRows, y1 = min(H, y0 + kScanRows - 1);
    for (int y = y0; y <= y1; ++y) {
        const int64_t o = (int64_t)y * (W + 1) + x;
        c1 += g1[o];
        c2 += g2[o];
        g1[o] = c1;
        g2[o] = c2;
    }
}

// ---- launch -------------------------------------------------------------
template <int Z>
static hipError_t launch_describe_z(const float* img, int H, int W, int64_t ld, void* desc, double* i1, double* i2,
                                    const DescribeConsts& c, hipStream_t st) {
    constexpr int CG = Z >= 4 ? 4 : Z;
    const DescribeLds L = describe_lds(c, CG);
    dim3 grid((W + kTS - 1) / kTS, (H + kTS - 1) / kTS);
    auto kern = describe_kernel<Z, CG>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.bytes);
    if (e != hipSuccess) return e;
    trace_begin(st, SFOC_K_DESCRIBE);
    hipLaunchKernelGGL(kern, grid, dim3(kNT), L.bytes, st, img, H, W, ld, desc, i1, i2, c, L.BS, L.IS);
    trace_end(st, SFOC_K_DESCRIBE);
    return hipGetLastError();
}

hipError_t launch_describe(const float* img, int H, int W, int64_t ld, void* desc, double* i1, double* i2,
                           const DescribeConsts& c, hipStream_t st) {
    switch (c.z) {
        case 2: return launch_describe_z<2>(img, H, W, ld, desc, i1, i2, c, st);
        case 3: return launch_describe_z<3>(img, H, W, ld, desc, i1, i2, c, st);
        case 4: return launch_describe_z<4>(img, H, W, ld, desc, i1, i2, c, st);
        case 6: return launch_describe_z<6>(img, H, W, ld, desc, i1, i2, c, st);
        case 8: return launch_describe_z<8>(img, H, W, ld, desc, i1, i2, c, st);
        case 12: return launch_describe_z<12>(img, H, W, ld, desc, i1, i2, c, st);
        case 16: return launch_describe_z<16>(img, H, W, ld, desc, i1, i2, c, st);
        case 24: return launch_describe_z<24>(img, H, W, ld, desc, i1, i2, c, st);
        case 32: return launch_describe_z<32>(img, H, W, ld, desc, i1, i2, c, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_integral(double* i1, double* i2, int H, int W, double* ws, hipStream_t st) {
    trace_begin(st, SFOC_K_INTEGRAL);
    hipLaunchKernelGGL(integral_row_scan, dim3(H + 1), dim3(kScanNT), 0, st, i1, i2, H, W);
    const int nb = (H + kScanRows - 1) / kScanRows;
    double* bs1 = ws;
    double* bs2 = ws + (size_t)nb * (W + 1);
    dim3 grid((W + 1 + kScanNT - 1) / kScanNT, nb);
    hipLaunchKernelGGL(integral_col_blocksum, grid, dim3(kScanNT), 0, st, i1, i2, H, W, bs1, bs2);
    hipLaunchKernelGGL(integral_col_apply, grid, dim3(kScanNT), 0, st, i1, i2, H, W, bs1, bs2);
    trace_end(st, SFOC_K_INTEGRAL);
    return hipGetLastError();
}

}  // namespace sfoc
