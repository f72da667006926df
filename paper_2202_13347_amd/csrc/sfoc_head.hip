// Learned CP-validity / sub-pixel head: features from the NCC surfaces,
// network forward, backward and Adam, and the inference decision.
//
// The network is small next to the matching (about 4 Mflop per sample), so
// the kernels favour simple, fixed-order arithmetic: one thread per output
// pixel with all 32 output channels in registers and the (bfloat16-rounded,
// transposed) weights read as wave-uniform scalars; weight gradients are
// per-chunk partial sums reduced in a fixed order, so every result is
// bit-reproducible.
#include <hip/hip_runtime.h>
#include <math.h>

#include "sfoc_dev.h"
#include "sfoc_launch.h"
#include "sfoc_trace.h"

namespace sfoc {
namespace head {

constexpr int kCrop = SFOC_HEAD_CROP, kHalf = kCrop / 2, kNStat = SFOC_HEAD_NSTAT, kCh = 32;
constexpr int kS0 = 33, kS1 = 33, kS2 = 17, kS3 = 9, kS4 = 5;   // map sides
constexpr int kFlat = kCh * kS4 * kS4;                           // 800
constexpr int kFcIn = kFlat + kNStat;                            // 808
// Parameter offsets (float32 vector, order of the header).
constexpr int kW1 = 0, kB1 = kW1 + kCh * 9;
constexpr int kW2 = kB1 + kCh, kB2 = kW2 + kCh * kCh * 9;
constexpr int kW3 = kB2 + kCh, kB3 = kW3 + kCh * kCh * 9;
constexpr int kW4 = kB3 + kCh, kB4 = kW4 + kCh * kCh * 9;
constexpr int kF1 = kB4 + kCh, kC1 = kF1 + kCh * kFcIn;
constexpr int kF2 = kC1 + kCh, kC2 = kF2 + 3 * kCh;
constexpr int kNParams = kC2 + 3;
static_assert(kNParams == SFOC_HEAD_PARAMS, "parameter layout");
constexpr float kLambda = 4.0f, kBeta = 0.1f, kClip = 1.5f;
constexpr int kMaxN = 65536;

SFOC_DEV float bf16_round(float w) { return bf16_bits_to_f32(f32_to_bf16_bits(w)); }

// ---- weights: rounded copies in the layouts the kernels read ------------
// wf[k]: [c][i][j][o] (forward, o fastest); wb[k]: [o][i][j][c] (backward
// data, c fastest); fc1q, fc2q: [o][k] as stored.
struct QWeights {
    float* wf[4];
    float* wb[4];
    float* fc1q;
    float* fc2q;
};

__global__ void prep_weights_kernel(const float* __restrict__ th, QWeights q) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int nconv1 = kCh * 9, nconv = kCh * kCh * 9;
    if (e < nconv1) {   // conv1: o = e / 9, tap = e % 9 (one input channel)
        const int o = e / 9, tap = e - o * 9;
        const float w = bf16_round(th[kW1 + e]);
        q.wf[0][tap * kCh + o] = w;
        q.wb[0][o * 9 + tap] = w;
        return;
    }
    int f = e - nconv1;
    if (f < 3 * nconv) {
        const int k = 1 + f / nconv;
        const int g = f - (k - 1) * nconv;
        const int o = g / (kCh * 9), rem = g - o * kCh * 9, c = rem / 9, tap = rem - c * 9;
        const int base = k == 1 ? kW2 : k == 2 ? kW3 : kW4;
        const float w = bf16_round(th[base + g]);
        q.wf[k][(c * 9 + tap) * kCh + o] = w;
        q.wb[k][(o * 9 + tap) * kCh + c] = w;
        return;
    }
    f -= 3 * nconv;
    if (f < kCh * kFcIn) {
        q.fc1q[f] = bf16_round(th[kF1 + f]);
        return;
    }
    f -= kCh * kFcIn;
    if (f < 3 * kCh) q.fc2q[f] = bf16_round(th[kF2 + f]);
}
constexpr int kPrepCount = kCh * 9 + 3 * kCh * kCh * 9 + kCh * kFcIn + 3 * kCh;

// ---- convolution forward --------------------------------------------------
// out[b][o][y][x] = relu(bias[o] + sum_{c,i,j} w[o][c][i][j] in[b][c][S y + i - 1][S x + j - 1]).
// One thread per output pixel with the 32 output channels in registers; the
// layer's weights are staged in LDS once per workgroup (read back as
// wave-uniform broadcasts) and the input loads of several channels are
// issued together.
constexpr int kOG = 4;            // output-channel groups per pixel
constexpr int kOPG = kCh / kOG;   // output channels per thread
template <int CIN, int S, int HIN, int HOUT>
__global__ __launch_bounds__(256) void conv_fwd_kernel(const float* __restrict__ in, const float* __restrict__ wf,
                                                       const float* __restrict__ bias, float* __restrict__ out,
                                                       int B) {
    __shared__ float4 sw[CIN * 9 * kCh / 4];
    for (int e = threadIdx.x; e < CIN * 9 * kCh / 4; e += 256) sw[e] = reinterpret_cast<const float4*>(wf)[e];
    __syncthreads();
    // thread -> (output pixel, group of kOPG output channels); the groups of
    // a pixel are adjacent lanes, so their input loads coincide
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= B * HOUT * HOUT * kOG) return;
    const int g = idx % kOG, pix = idx / kOG;
    const int b = pix / (HOUT * HOUT), p = pix - b * HOUT * HOUT;
    const int y = p / HOUT, x = p - y * HOUT;
    float acc[kOPG];
#pragma unroll
    for (int o = 0; o < kOPG; ++o) acc[o] = bias[g * kOPG + o];
    int off[9];
    bool ok[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int yy = S * y + i - 1, xx = S * x + j - 1;
            ok[i * 3 + j] = yy >= 0 && yy < HIN && xx >= 0 && xx < HIN;
            off[i * 3 + j] = ok[i * 3 + j] ? yy * HIN + xx : 0;
        }
    const float* src = in + (size_t)b * CIN * HIN * HIN;
    constexpr int CU = CIN >= 4 ? 4 : CIN;   // channels whose loads are issued together
#pragma unroll 1
    for (int c0 = 0; c0 < CIN; c0 += CU) {
        float v[CU][9];
#pragma unroll
        for (int cc = 0; cc < CU; ++cc)
#pragma unroll
            for (int k = 0; k < 9; ++k) v[cc][k] = ok[k] ? src[(size_t)(c0 + cc) * HIN * HIN + off[k]] : 0.f;
#pragma unroll
        for (int cc = 0; cc < CU; ++cc)
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                const float4* w = sw + ((c0 + cc) * 9 + k) * (kCh / 4) + g * (kOPG / 4);
#pragma unroll
                for (int q = 0; q < kOPG / 4; ++q) {
                    const float4 wq = w[q];
                    acc[4 * q] = fmaf(wq.x, v[cc][k], acc[4 * q]);
                    acc[4 * q + 1] = fmaf(wq.y, v[cc][k], acc[4 * q + 1]);
                    acc[4 * q + 2] = fmaf(wq.z, v[cc][k], acc[4 * q + 2]);
                    acc[4 * q + 3] = fmaf(wq.w, v[cc][k], acc[4 * q + 3]);
                }
            }
    }
#pragma unroll
    for (int o = 0; o < kOPG; ++o)
        out[(((size_t)b * kCh + g * kOPG + o) * HOUT + y) * HOUT + x] = fmaxf(acc[o], 0.f);
}

// ---- fully connected forward: one 64-thread workgroup per sample ----------
__global__ __launch_bounds__(64) void fc_fwd_kernel(const float* __restrict__ a4, const float* __restrict__ stats,
                                                    const float* __restrict__ fc1q, const float* __restrict__ th,
                                                    const float* __restrict__ fc2q, float* __restrict__ h1,
                                                    float* __restrict__ out) {
    __shared__ float hs[kCh];
    const int b = blockIdx.x, t = threadIdx.x;
    if (t < kCh) {
        const float* w = fc1q + t * kFcIn;
        const float* x = a4 + (size_t)b * kFlat;
        float acc = th[kC1 + t];
        for (int k = 0; k < kFlat; ++k) acc = fmaf(w[k], x[k], acc);
        for (int k = 0; k < kNStat; ++k) acc = fmaf(w[kFlat + k], stats[(size_t)b * kNStat + k], acc);
        const float h = fmaxf(acc, 0.f);
        hs[t] = h;
        h1[(size_t)b * kCh + t] = h;
    }
    __syncthreads();
    if (t < 3) {
        float acc = th[kC2 + t];
        for (int o = 0; o < kCh; ++o) acc = fmaf(fc2q[t * kCh + o], hs[o], acc);
        out[(size_t)b * 3 + t] = acc;
    }
}

// ---- loss and its gradient w.r.t. the outputs -------------------------------
SFOC_DEV float sigmoidf_(float l) {
    const float e = __expf(-fabsf(l));
    return l >= 0.f ? 1.f / (1.f + e) : e / (1.f + e);
}
SFOC_DEV float smooth_l1(float d) {
    const float a = fabsf(d);
    return a < kBeta ? 0.5f * d * d / kBeta : a - 0.5f * kBeta;
}
SFOC_DEV float smooth_l1_grad(float d) { return fabsf(d) < kBeta ? d / kBeta : (d > 0.f ? 1.f : -1.f); }

__global__ __launch_bounds__(256) void loss_kernel(const float* __restrict__ out, const float* __restrict__ label,
                                                   const float* __restrict__ target, int B, float* __restrict__ dout,
                                                   float* __restrict__ loss) {
    __shared__ double red[256];
    const int t = threadIdx.x;
    double part = 0.0;
    const float inv = 1.0f / (float)B;
    for (int b = t; b < B; b += 256) {
        const float l = out[b * 3], y = label[b];
        const float dy = out[b * 3 + 1] - target[2 * b], dx = out[b * 3 + 2] - target[2 * b + 1];
        const float bce = fmaxf(l, 0.f) - l * y + log1pf(__expf(-fabsf(l)));
        part += (double)(bce + kLambda * y * (smooth_l1(dy) + smooth_l1(dx)));
        dout[b * 3] = (sigmoidf_(l) - y) * inv;
        dout[b * 3 + 1] = kLambda * y * smooth_l1_grad(dy) * inv;
        dout[b * 3 + 2] = kLambda * y * smooth_l1_grad(dx) * inv;
    }
    red[t] = part;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) red[t] += red[t + s];
        __syncthreads();
    }
    if (t == 0 && loss) loss[0] = (float)(red[0] / B);
}

// ---- fully connected backward -------------------------------------------
// dh1[b][o] = relu'(h1) * sum_t fc2[t][o] d[b][t]
__global__ void fc2_bwd_data_kernel(const float* __restrict__ dout, const float* __restrict__ h1,
                                    const float* __restrict__ fc2q, float* __restrict__ dh1, int B) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= B * kCh) return;
    const int b = idx / kCh, o = idx - b * kCh;
    float g = 0.f;
    for (int t = 0; t < 3; ++t) g = fmaf(fc2q[t * kCh + o], dout[b * 3 + t], g);
    dh1[idx] = h1[idx] > 0.f ? g : 0.f;
}

// Weight and bias gradients of fc1 and fc2 (one thread per entry, batch sum
// in order): entries [0, 32*808) fc1.w, then 32 fc1.b, 96 fc2.w, 3 fc2.b.
__global__ void fc_bwd_weight_kernel(const float* __restrict__ dout, const float* __restrict__ h1,
                                     const float* __restrict__ dh1, const float* __restrict__ a4,
                                     const float* __restrict__ stats, float* __restrict__ grad, int B) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    float acc = 0.f;
    if (e < kCh * kFcIn) {
        const int o = e / kFcIn, k = e - o * kFcIn;
        for (int b = 0; b < B; ++b) {
            const float x = k < kFlat ? a4[(size_t)b * kFlat + k] : stats[(size_t)b * kNStat + k - kFlat];
            acc = fmaf(dh1[b * kCh + o], x, acc);
        }
        grad[kF1 + e] = acc;
        return;
    }
    e -= kCh * kFcIn;
    if (e < kCh) {
        for (int b = 0; b < B; ++b) acc += dh1[b * kCh + e];
        grad[kC1 + e] = acc;
        return;
    }
    e -= kCh;
    if (e < 3 * kCh) {
        const int t = e / kCh, o = e - t * kCh;
        for (int b = 0; b < B; ++b) acc = fmaf(dout[b * 3 + t], h1[b * kCh + o], acc);
        grad[kF2 + e] = acc;
        return;
    }
    e -= 3 * kCh;
    if (e < 3) {
        for (int b = 0; b < B; ++b) acc += dout[b * 3 + e];
        grad[kC2 + e] = acc;
    }
}
constexpr int kFcGradCount = kCh * kFcIn + kCh + 3 * kCh + 3;

// d_a4[b][k] = sum_o fc1[o][k] dh1[b][o] for the 800 conv values
__global__ void fc1_bwd_data_kernel(const float* __restrict__ dh1, const float* __restrict__ fc1q,
                                    float* __restrict__ da4, int B) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= B * kFlat) return;
    const int b = idx / kFlat, k = idx - b * kFlat;
    float g = 0.f;
    for (int o = 0; o < kCh; ++o) g = fmaf(fc1q[o * kFcIn + k], dh1[b * kCh + o], g);
    da4[idx] = g;
}

// ---- convolution backward -------------------------------------------------
// din[b][c][y][x] = sum_{o,i,j: S yo + i - 1 = y, S xo + j - 1 = x} w[o][c][i][j] g[b][o][yo][xo],
// g = dout * relu'(aout).
template <int CIN, int S, int HIN, int HOUT>
__global__ __launch_bounds__(256) void conv_bwd_data_kernel(const float* __restrict__ dout,
                                                            const float* __restrict__ aout,
                                                            const float* __restrict__ wb, float* __restrict__ din,
                                                            int B) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= B * HIN * HIN) return;
    const int b = idx / (HIN * HIN), p = idx - b * HIN * HIN;
    const int y = p / HIN, x = p - y * HIN;
    float acc[CIN];
#pragma unroll
    for (int c = 0; c < CIN; ++c) acc[c] = 0.f;
    for (int o = 0; o < kCh; ++o) {
        const size_t ob = ((size_t)b * kCh + o) * HOUT * HOUT;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const int ty = y + 1 - i;
            if (ty < 0 || ty % S) continue;
            const int yo = ty / S;
            if (yo >= HOUT) continue;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int tx = x + 1 - j;
                if (tx < 0 || tx % S) continue;
                const int xo = tx / S;
                if (xo >= HOUT) continue;
                const float a = aout[ob + yo * HOUT + xo];
                const float g = a > 0.f ? dout[ob + yo * HOUT + xo] : 0.f;
                const float* w = wb + (o * 9 + i * 3 + j) * CIN;
#pragma unroll
                for (int c = 0; c < CIN; ++c) acc[c] = fmaf(w[c], g, acc[c]);
            }
        }
    }
#pragma unroll
    for (int c = 0; c < CIN; ++c) din[(((size_t)b * CIN + c) * HIN + y) * HIN + x] = acc[c];
}

// Partial weight / bias gradients over a chunk of samples: thread t owns
// output channel o = t / (CIN / CPT) and CPT input channels, all 9 taps.
// part[chunk][(o * CIN + c) * 9 + tap], then the 32 bias entries.
template <int CIN, int S, int HIN, int HOUT>
__global__ __launch_bounds__(256) void conv_bwd_weight_kernel(const float* __restrict__ dout,
                                                              const float* __restrict__ aout,
                                                              const float* __restrict__ in, float* __restrict__ part,
                                                              int B, int spc) {
    constexpr int CPT = CIN >= 8 ? CIN / 8 : 1;
    constexpr int GPO = CIN / CPT;   // threads per output channel
    constexpr int NW = kCh * CIN * 9 + kCh;
    const int t = threadIdx.x;
    const int chunk = blockIdx.x;
    if (t >= kCh * GPO) return;
    const int o = t / GPO, c0 = (t - o * GPO) * CPT;
    float acc[CPT][9];
    float accb = 0.f;
#pragma unroll
    for (int cc = 0; cc < CPT; ++cc)
#pragma unroll
        for (int k = 0; k < 9; ++k) acc[cc][k] = 0.f;
    const int b0 = chunk * spc, b1 = min(B, b0 + spc);
    for (int b = b0; b < b1; ++b) {
        const size_t ob = ((size_t)b * kCh + o) * HOUT * HOUT;
        for (int p = 0; p < HOUT * HOUT; ++p) {
            const int yo = p / HOUT, xo = p - yo * HOUT;
            const float a = aout[ob + p];
            const float g = a > 0.f ? dout[ob + p] : 0.f;
            accb += g;
#pragma unroll
            for (int cc = 0; cc < CPT; ++cc) {
                const float* src = in + ((size_t)b * CIN + c0 + cc) * HIN * HIN;
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    const int yy = S * yo + i - 1;
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        const int xx = S * xo + j - 1;
                        const float v = (yy >= 0 && yy < HIN && xx >= 0 && xx < HIN) ? src[yy * HIN + xx] : 0.f;
                        acc[cc][i * 3 + j] = fmaf(g, v, acc[cc][i * 3 + j]);
                    }
                }
            }
        }
    }
    float* dst = part + (size_t)chunk * NW;
#pragma unroll
    for (int cc = 0; cc < CPT; ++cc)
#pragma unroll
        for (int k = 0; k < 9; ++k) dst[(o * CIN + c0 + cc) * 9 + k] = acc[cc][k];
    if (c0 == 0) dst[kCh * CIN * 9 + o] = accb;
}

// Sum of the chunk partials in chunk order: weights to grad[w0 ..], biases
// to grad[b0 ..].
__global__ void reduce_partials_kernel(const float* __restrict__ part, int nchunks, int nw, float* __restrict__ grad,
                                       int w0, int b0) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = nw + kCh;
    if (e >= n) return;
    float s = 0.f;
    for (int k = 0; k < nchunks; ++k) s += part[(size_t)k * n + e];
    grad[e < nw ? w0 + e : b0 + (e - nw)] = s;
}

// ---- Adam -------------------------------------------------------------------
__global__ void adam_kernel(float* __restrict__ th, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g, int n, float lr, float c1, float c2) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const float gg = g[e];
    const float mm = 0.9f * m[e] + 0.1f * gg;
    const float vv = 0.999f * v[e] + 0.001f * gg * gg;
    m[e] = mm;
    v[e] = vv;
    th[e] -= lr * (mm * c1) / (sqrtf(vv * c2) + 1e-8f);
}

// ---- features -------------------------------------------------------------
constexpr uint32_t kEligible = SFOC_CP_VALID | SFOC_CP_INCONSISTENT;

template <int DT>
SFOC_DEV float ld_desc(const void* p, int64_t i) {
    if (DT == SFOC_DTYPE_F32) return ((const float*)p)[i];
    if (DT == SFOC_DTYPE_BF16) return bf16_bits_to_f32(((const uint16_t*)p)[i]);
    return f16_bits_to_f32(((const uint16_t*)p)[i]);
}

struct FeatArgs {
    const void* desc_sen;
    const double* integ1;
    const double* integ2;
    const int32_t* ips;
    const int32_t* prior;
    const float* ncc;
    const sfoc_cp* cps;
    float* crops;
    float* stats;
    int64_t Hs, Ws, Wr;
    int z, m, r;
};

constexpr int kFeatNT = 1024;
template <int DT>
__global__ __launch_bounds__(kFeatNT) void features_kernel(const FeatArgs A) {
    __shared__ double rd[4][kFeatNT];
    __shared__ float rmax[kFeatNT];
    const int i = blockIdx.x, t = threadIdx.x;
    const sfoc_cp cp = A.cps[i];
    float* crop = A.crops + (size_t)i * kCrop * kCrop;
    float* st = A.stats + (size_t)i * kNStat;
    if (!(cp.flags & kEligible)) {
        for (int e = t; e < kCrop * kCrop; e += kFeatNT) crop[e] = 0.f;
        if (t < kNStat) st[t] = 0.f;
        return;
    }
    const int r = A.r, m = A.m, V = 2 * r + 1;
    const int u = cp.dy + r, v = cp.dx + r;
    const float* S = A.ncc + (size_t)i * V * V;
    for (int e = t; e < kCrop * kCrop; e += kFeatNT) {
        const int a = e / kCrop, b = e - a * kCrop;
        const int y = u - kHalf + a, x = v - kHalf + b;
        crop[e] = (y >= 0 && y < V && x >= 0 && x < V) ? S[y * V + x] : -1.f;
    }
    // surface sums and the best value outside the 3 x 3 block
    double s1 = 0.0, s2 = 0.0;
    float best = -1.f;
    for (int e = t; e < V * V; e += kFeatNT) {
        const int y = e / V, x = e - y * V;
        const float s = S[e];
        s1 += s;
        s2 += (double)s * s;
        if ((abs(y - u) > 1 || abs(x - v) > 1) && s > best) best = s;
    }
    // template sums (Eq. 12)
    const int py = A.ips[2 * i], px = A.ips[2 * i + 1];
    const int64_t ty = (int64_t)py - m / 2, tx = (int64_t)px - m / 2;
    const int64_t plane = A.Hs * A.Ws;
    double t1 = 0.0, t2 = 0.0;
    const int mm = m * m;
    // A thread takes template positions q = t, t + kFeatNT, ... and, for each,
    // all channels: one division per position instead of two per element,
    // eight channels' loads in flight per step.  The summation order is
    // fixed (position, then channel), so the sums are reproducible.
    for (int q = t; q < mm; q += kFeatNT) {
        const int yy = q / m, xx = q - yy * m;
        const int64_t pos = (ty + yy) * A.Ws + tx + xx;
        for (int h0 = 0; h0 < A.z; h0 += 8) {
            double d[8];
#pragma unroll
            for (int k = 0; k < 8; ++k)
                d[k] = h0 + k < A.z ? (double)ld_desc<DT>(A.desc_sen, (h0 + k) * plane + pos) : 0.0;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                t1 += d[k];
                t2 += d[k] * d[k];
            }
        }
    }
    rd[0][t] = s1;
    rd[1][t] = s2;
    rd[2][t] = t1;
    rd[3][t] = t2;
    rmax[t] = best;
    __syncthreads();
    for (int s = kFeatNT / 2; s > 0; s >>= 1) {
        if (t < s) {
#pragma unroll
            for (int k = 0; k < 4; ++k) rd[k][t] += rd[k][t + s];
            rmax[t] = fmaxf(rmax[t], rmax[t + s]);
        }
        __syncthreads();
    }
    if (t == 0) {
        const double n = (double)V * V;
        const double mean = rd[0][0] / n;
        const double var = fmax(rd[1][0] / n - mean * mean, 0.0);
        const double mnz = (double)m * m * A.z;
        const double RT = rd[2][0], RTT = rd[3][0];
        const double varT = RTT - RT * RT / mnz;
        const int pry = A.prior ? A.prior[2 * i] : 0, prx = A.prior ? A.prior[2 * i + 1] : 0;
        const int64_t y = ty - r + pry + u, x = tx - r + prx + v;   // search window at the peak
        const int64_t IW = A.Wr + 1;
        const int64_t a00 = y * IW + x, a01 = a00 + m, a10 = a00 + (int64_t)m * IW, a11 = a10 + m;
        const double RS = A.integ1[a11] - A.integ1[a10] - A.integ1[a01] + A.integ1[a00];
        const double RSS = A.integ2[a11] - A.integ2[a10] - A.integ2[a01] + A.integ2[a00];
        const double varS = RSS - RS * RS / mnz;
        const float c0 = S[u * V + v];
        const double d0 = c0;
        const double curv = 0.5 * (((double)S[(u - 1) * V + v] - 2.0 * d0 + S[(u + 1) * V + v]) +
                                   ((double)S[u * V + v - 1] - 2.0 * d0 + S[u * V + v + 1]));
        st[0] = c0;
        st[1] = rmax[0];
        st[2] = (float)mean;
        st[3] = (float)sqrt(var);
        st[4] = (float)sqrt(fmax(varT, 0.0) / mnz);
        st[5] = (float)sqrt(fmax(varS, 0.0) / mnz);
        st[6] = (float)(RT / mnz);
        st[7] = (float)curv;
    }
}

// ---- inference decision -----------------------------------------------------
__global__ void apply_kernel(const float* __restrict__ out, sfoc_cp* __restrict__ cps, int n, float threshold) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    sfoc_cp c = cps[i];
    if (!(c.flags & kEligible)) return;
    const float p = sigmoidf_(out[i * 3]);
    c.flags = (c.flags & ~kEligible) | SFOC_CP_LEARNED | (p >= threshold ? SFOC_CP_VALID : SFOC_CP_INCONSISTENT);
    c.sub_dy = fminf(kClip, fmaxf(-kClip, out[i * 3 + 1]));
    c.sub_dx = fminf(kClip, fmaxf(-kClip, out[i * 3 + 2]));
    cps[i] = c;
}

// ---- workspace ------------------------------------------------------------
struct Layout {
    size_t wf[4], wb[4], fc1q, fc2q, a1, a2, a3, a4, h1, out;   // forward
    size_t dout, dh1, da4, da3, da2, da1, part, grad, total;    // training
    int spc, nchunks;
};

static size_t take(size_t& off, size_t floats) {
    const size_t o = off;
    off = align_up(off + floats * sizeof(float), 256);
    return o;
}

static Layout layout(int n, bool train) {
    Layout L{};
    size_t off = 0;
    L.wf[0] = take(off, 9 * kCh);
    L.wb[0] = take(off, 9 * kCh);
    for (int k = 1; k < 4; ++k) {
        L.wf[k] = take(off, kCh * kCh * 9);
        L.wb[k] = take(off, kCh * kCh * 9);
    }
    L.fc1q = take(off, kCh * kFcIn);
    L.fc2q = take(off, 3 * kCh);
    L.a1 = take(off, (size_t)n * kCh * kS1 * kS1);
    L.a2 = take(off, (size_t)n * kCh * kS2 * kS2);
    L.a3 = take(off, (size_t)n * kCh * kS3 * kS3);
    L.a4 = take(off, (size_t)n * kFlat);
    L.h1 = take(off, (size_t)n * kCh);
    L.out = take(off, (size_t)n * 3);
    L.spc = (n + 511) / 512;
    L.nchunks = n > 0 ? (n + L.spc - 1) / L.spc : 0;
    if (train) {
        L.dout = take(off, (size_t)n * 3);
        L.dh1 = take(off, (size_t)n * kCh);
        L.da4 = take(off, (size_t)n * kFlat);
        L.da3 = take(off, (size_t)n * kCh * kS3 * kS3);
        L.da2 = take(off, (size_t)n * kCh * kS2 * kS2);
        L.da1 = take(off, (size_t)n * kCh * kS1 * kS1);
        L.part = take(off, (size_t)L.nchunks * (kCh * kCh * 9 + kCh));
        L.grad = take(off, kNParams);
    }
    L.total = off;
    return L;
}

static inline int blocks(size_t n, int t) { return (int)((n + t - 1) / t); }

static QWeights qweights(char* ws, const Layout& L) {
    QWeights q;
    for (int k = 0; k < 4; ++k) {
        q.wf[k] = (float*)(ws + L.wf[k]);
        q.wb[k] = (float*)(ws + L.wb[k]);
    }
    q.fc1q = (float*)(ws + L.fc1q);
    q.fc2q = (float*)(ws + L.fc2q);
    return q;
}

static hipError_t forward(const float* th, const float* crops, const float* stats, int n, float* out, char* ws,
                          const Layout& L, hipStream_t st) {
    const QWeights q = qweights(ws, L);
    float* a1 = (float*)(ws + L.a1);
    float* a2 = (float*)(ws + L.a2);
    float* a3 = (float*)(ws + L.a3);
    float* a4 = (float*)(ws + L.a4);
    float* h1 = (float*)(ws + L.h1);
    trace_begin(st, SFOC_K_HEAD_FWD);
    hipLaunchKernelGGL(prep_weights_kernel, dim3(blocks(kPrepCount, 256)), dim3(256), 0, st, th, q);
    hipLaunchKernelGGL((conv_fwd_kernel<1, 1, kS0, kS1>), dim3(blocks((size_t)n * kS1 * kS1 * kOG, 256)), dim3(256), 0, st,
                       crops, q.wf[0], th + kB1, a1, n);
    hipLaunchKernelGGL((conv_fwd_kernel<kCh, 2, kS1, kS2>), dim3(blocks((size_t)n * kS2 * kS2 * kOG, 256)), dim3(256), 0,
                       st, a1, q.wf[1], th + kB2, a2, n);
    hipLaunchKernelGGL((conv_fwd_kernel<kCh, 2, kS2, kS3>), dim3(blocks((size_t)n * kS3 * kS3 * kOG, 256)), dim3(256), 0,
                       st, a2, q.wf[2], th + kB3, a3, n);
    hipLaunchKernelGGL((conv_fwd_kernel<kCh, 2, kS3, kS4>), dim3(blocks((size_t)n * kS4 * kS4 * kOG, 256)), dim3(256), 0,
                       st, a3, q.wf[3], th + kB4, a4, n);
    hipLaunchKernelGGL(fc_fwd_kernel, dim3(n), dim3(64), 0, st, a4, stats, q.fc1q, th, q.fc2q, h1, out);
    trace_end(st, SFOC_K_HEAD_FWD);
    return hipGetLastError();
}

template <int CIN, int S, int HIN, int HOUT>
static void conv_bwd(const float* dout, const float* aout, const float* in, const float* wb, float* din, char* ws,
                     const Layout& L, int n, float* grad, int w0, int b0, hipStream_t st) {
    float* part = (float*)(ws + L.part);
    if (din)
        hipLaunchKernelGGL((conv_bwd_data_kernel<CIN, S, HIN, HOUT>), dim3(blocks((size_t)n * HIN * HIN, 256)),
                           dim3(256), 0, st, dout, aout, wb, din, n);
    hipLaunchKernelGGL((conv_bwd_weight_kernel<CIN, S, HIN, HOUT>), dim3(L.nchunks), dim3(256), 0, st, dout, aout, in,
                       part, n, L.spc);
    const int nw = kCh * CIN * 9;
    hipLaunchKernelGGL(reduce_partials_kernel, dim3(blocks(nw + kCh, 256)), dim3(256), 0, st, part, L.nchunks, nw,
                       grad, w0, b0);
}

}  // namespace head
}  // namespace sfoc

using namespace sfoc;
using namespace sfoc::head;

extern "C" {

int sfoc_head_workspace(int32_t n, int32_t train, size_t* bytes) {
    if (!bytes || n < 0) return SFOC_E_INVALID_ARG;
    if (n > kMaxN) return SFOC_E_UNSUPPORTED;
    *bytes = layout(n, train != 0).total;
    return SFOC_OK;
}

int sfoc_head_features(const void* desc_sen, int64_t Hs, int64_t Ws, const double* integ1, const double* integ2,
                       int64_t Hr, int64_t Wr, int32_t z, int32_t dtype, const int32_t* ips, const int32_t* prior,
                       int32_t n, int32_t m, int32_t r, const float* ncc, const sfoc_cp* cps, float* crops,
                       float* stats, void* stream) {
    int rc = check_match_shape(n, m, r);
    if (rc) return rc;
    if (z < 1 || dtype_size(dtype) == 0 || Hs < 1 || Ws < 1 || Hr < 1 || Wr < 1) return SFOC_E_INVALID_ARG;
    if (Hs > kMaxSide || Ws > kMaxSide || Hr > kMaxSide || Wr > kMaxSide) return SFOC_E_UNSUPPORTED;
    if (n == 0) return SFOC_OK;
    if (!desc_sen || !integ1 || !integ2 || !ips || !ncc || !cps || !crops || !stats) return SFOC_E_INVALID_ARG;
    FeatArgs A{desc_sen, integ1, integ2, ips, prior, ncc, cps, crops, stats, Hs, Ws, Wr, z, m, r};
    hipStream_t st = (hipStream_t)stream;
    trace_begin(st, SFOC_K_HEAD_FEAT);
    if (dtype == SFOC_DTYPE_F32) hipLaunchKernelGGL(features_kernel<SFOC_DTYPE_F32>, dim3(n), dim3(kFeatNT), 0, st, A);
    else if (dtype == SFOC_DTYPE_BF16) hipLaunchKernelGGL(features_kernel<SFOC_DTYPE_BF16>, dim3(n), dim3(kFeatNT), 0, st, A);
    else hipLaunchKernelGGL(features_kernel<SFOC_DTYPE_F16>, dim3(n), dim3(kFeatNT), 0, st, A);
    trace_end(st, SFOC_K_HEAD_FEAT);
    return hip_status(hipGetLastError());
}

int sfoc_head_forward(const float* params, const float* crops, const float* stats, int32_t n, float* out, void* ws,
                      size_t ws_bytes, void* stream) {
    if (n < 0) return SFOC_E_INVALID_ARG;
    if (n > kMaxN) return SFOC_E_UNSUPPORTED;
    if (n == 0) return SFOC_OK;
    if (!params || !crops || !stats || !out || !ws) return SFOC_E_INVALID_ARG;
    const Layout L = layout(n, false);
    if (ws_bytes < L.total) return SFOC_E_WORKSPACE;
    return hip_status(forward(params, crops, stats, n, out, (char*)ws, L, (hipStream_t)stream));
}

int sfoc_head_infer(const float* params, const float* crops, const float* stats, int32_t n, float threshold,
                    sfoc_cp* cps, float* out, void* ws, size_t ws_bytes, void* stream) {
    if (n < 0 || !(threshold >= 0.f && threshold <= 1.f)) return SFOC_E_INVALID_ARG;
    if (n > kMaxN) return SFOC_E_UNSUPPORTED;
    if (n == 0) return SFOC_OK;
    if (!params || !crops || !stats || !cps || !ws) return SFOC_E_INVALID_ARG;
    const Layout L = layout(n, false);
    if (ws_bytes < L.total) return SFOC_E_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    float* o = out ? out : (float*)((char*)ws + L.out);
    hipError_t e = forward(params, crops, stats, n, o, (char*)ws, L, st);
    if (e != hipSuccess) return hip_status(e);
    hipLaunchKernelGGL(apply_kernel, dim3(blocks(n, 256)), dim3(256), 0, st, o, cps, n, threshold);
    return hip_status(hipGetLastError());
}

int sfoc_head_train_step(float* params, float* adam_m, float* adam_v, int32_t t, float lr, const float* crops,
                         const float* stats, const float* label, const float* target, int32_t n, float* grad,
                         float* loss, void* ws, size_t ws_bytes, void* stream) {
    if (n < 0 || t < 1 || !(lr >= 0.f)) return SFOC_E_INVALID_ARG;
    if (n > kMaxN) return SFOC_E_UNSUPPORTED;
    if (n == 0) return SFOC_OK;
    if (!params || !adam_m || !adam_v || !crops || !stats || !label || !target || !ws) return SFOC_E_INVALID_ARG;
    const Layout L = layout(n, true);
    if (ws_bytes < L.total) return SFOC_E_WORKSPACE;
    char* w = (char*)ws;
    hipStream_t st = (hipStream_t)stream;
    float* out = (float*)(w + L.out);
    hipError_t e = forward(params, crops, stats, n, out, w, L, st);
    if (e != hipSuccess) return hip_status(e);
    const QWeights q = qweights(w, L);
    float* g = grad ? grad : (float*)(w + L.grad);
    float* dout = (float*)(w + L.dout);
    float* dh1 = (float*)(w + L.dh1);
    float* da4 = (float*)(w + L.da4);
    float* da3 = (float*)(w + L.da3);
    float* da2 = (float*)(w + L.da2);
    float* da1 = (float*)(w + L.da1);
    const float* a1 = (const float*)(w + L.a1);
    const float* a2 = (const float*)(w + L.a2);
    const float* a3 = (const float*)(w + L.a3);
    const float* a4 = (const float*)(w + L.a4);
    const float* h1 = (const float*)(w + L.h1);
    trace_begin(st, SFOC_K_HEAD_BWD);
    hipLaunchKernelGGL(loss_kernel, dim3(1), dim3(256), 0, st, out, label, target, n, dout, loss);
    hipLaunchKernelGGL(fc2_bwd_data_kernel, dim3(blocks((size_t)n * kCh, 256)), dim3(256), 0, st, dout, h1, q.fc2q,
                       dh1, n);
    hipLaunchKernelGGL(fc_bwd_weight_kernel, dim3(blocks(kFcGradCount, 256)), dim3(256), 0, st, dout, h1, dh1, a4,
                       stats, g, n);
    hipLaunchKernelGGL(fc1_bwd_data_kernel, dim3(blocks((size_t)n * kFlat, 256)), dim3(256), 0, st, dh1, q.fc1q, da4,
                       n);
    conv_bwd<kCh, 2, kS3, kS4>(da4, a4, a3, q.wb[3], da3, w, L, n, g, kW4, kB4, st);
    conv_bwd<kCh, 2, kS2, kS3>(da3, a3, a2, q.wb[2], da2, w, L, n, g, kW3, kB3, st);
    conv_bwd<kCh, 2, kS1, kS2>(da2, a2, a1, q.wb[1], da1, w, L, n, g, kW2, kB2, st);
    conv_bwd<1, 1, kS0, kS1>(da1, a1, crops, q.wb[0], nullptr, w, L, n, g, kW1, kB1, st);
    trace_end(st, SFOC_K_HEAD_BWD);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_status(e);
    // bias corrections in double on the host
    const double c1 = 1.0 / (1.0 - pow(0.9, (double)t)), c2 = 1.0 / (1.0 - pow(0.999, (double)t));
    trace_begin(st, SFOC_K_HEAD_ADAM);
    hipLaunchKernelGGL(adam_kernel, dim3(blocks(kNParams, 256)), dim3(256), 0, st, params, adam_m, adam_v, g,
                       kNParams, lr, (float)c1, (float)c2);
    trace_end(st, SFOC_K_HEAD_ADAM);
    return hip_status(hipGetLastError());
}

}  // extern "C"
