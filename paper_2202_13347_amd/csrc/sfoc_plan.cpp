// Host-side parameter checks, constant synthesis and workspace sizing.
#include "sfoc_plan.h"

#include <errno.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <set>

namespace sfoc {

static int radius_of(double s, double trunc) { return (int)ceil(trunc * s - 1e-9); }

size_t dtype_size(int32_t dtype) {
    switch (dtype) {
        case SFOC_DTYPE_F32: return 4;
        case SFOC_DTYPE_BF16: return 2;
        case SFOC_DTYPE_F16: return 2;
        default: return 0;
    }
}

static bool supported_z(int z) {
    switch (z) {
        case 2: case 3: case 4: case 6: case 8: case 12: case 16: case 24: case 32: return true;
        default: return false;
    }
}

int check_params(const sfoc_params* p, int32_t* zout) {
    if (!p) return SFOC_E_INVALID_ARG;
    if (p->n_orient < 1 || p->n_orient > SFOC_MAX_ORIENT) return SFOC_E_INVALID_ARG;
    if (p->n_s1 < 1 || p->n_s1 > SFOC_MAX_SIGMAS) return SFOC_E_INVALID_ARG;
    if (p->second_order != 0 && p->second_order != 1) return SFOC_E_INVALID_ARG;
    if (p->second_order && (p->n_s2 < 1 || p->n_s2 > SFOC_MAX_SIGMAS)) return SFOC_E_INVALID_ARG;
    if (!(p->trunc > 0.0) || !isfinite(p->trunc)) return SFOC_E_INVALID_ARG;
    if (!(p->sd1 > 0.0) || !(p->sd2 > 0.0) || !isfinite(p->sd1) || !isfinite(p->sd2)) return SFOC_E_INVALID_ARG;
    if (!(p->eps >= 0.0) || !isfinite(p->eps)) return SFOC_E_INVALID_ARG;
    if (p->K < 0 || p->n_dil < 1 || p->n_dil > SFOC_MAX_DIL) return SFOC_E_INVALID_ARG;
    if (p->rectify < 0 || p->rectify > 2) return SFOC_E_INVALID_ARG;
    if (dtype_size(p->desc_dtype) == 0) return SFOC_E_INVALID_ARG;
    int rmax = 0;
    for (int i = 0; i < p->n_dil; ++i) {
        if (p->dil[i] < 1) return SFOC_E_INVALID_ARG;
        if (p->dil[i] > rmax) rmax = p->dil[i];
    }
    const int nl = p->second_order ? 2 : 1;
    for (int l = 0; l < nl; ++l) {
        const int n = l ? p->n_s2 : p->n_s1;
        const double* s = l ? p->s2 : p->s1;
        for (int i = 0; i < n; ++i) {
            if (!(s[i] > 0.0) || !isfinite(s[i])) return SFOC_E_INVALID_ARG;
            if (radius_of(s[i], p->trunc) > kMaxRadius) return SFOC_E_UNSUPPORTED;
        }
    }
    if (p->K > 2 || p->K * rmax > kMaxQ) return SFOC_E_UNSUPPORTED;
    const int z = p->n_orient * (p->second_order ? 2 : 1);
    if (!supported_z(z)) return SFOC_E_UNSUPPORTED;
    // Tap storage.
    DescribeConsts tmp;
    int rc = build_describe_consts(p, &tmp);
    if (rc != SFOC_OK) return rc;
    if (zout) *zout = z;
    return SFOC_OK;
}

int build_describe_consts(const sfoc_params* p, DescribeConsts* c) {
    memset(c, 0, sizeof(*c));
    // Distinct sigmas over both order lists (a sigma used by both shares its
    // row pass).
    double sig[kMaxSig];
    int nsig = 0;
    const int nl = p->second_order ? 2 : 1;
    for (int l = 0; l < nl; ++l) {
        const int n = l ? p->n_s2 : p->n_s1;
        const double* s = l ? p->s2 : p->s1;
        for (int i = 0; i < n; ++i) {
            int j = 0;
            for (; j < nsig; ++j)
                if (sig[j] == s[i]) break;
            if (j == nsig) {
                sig[nsig] = s[i];
                c->use[nsig] = 0;
                ++nsig;
            }
            c->use[j] |= (1 << l);
        }
    }
    c->nsig = nsig;
    int off = 0, R = 0;
    for (int j = 0; j < nsig; ++j) {
        const double s = sig[j];
        const int r = radius_of(s, p->trunc);
        if (off + 3 * (r + 1) > kMaxHalfTaps) return SFOC_E_UNSUPPORTED;
        c->rad[j] = r;
        c->off[j] = off;
        c->cnorm[j] = (float)(1.0 / (2.0 * M_PI * s * s));
        // 1-D factors of Eq. 2, 3, 5: G = cnorm * e(x) e(y),
        // dG/dx = cnorm * (-x/s^2) e(x) e(y), d2G/dx2 = cnorm * (x^2/s^4 - 1/s^2) e(x) e(y).
        for (int k = 0; k <= r; ++k) {
            const double e = exp(-(double)k * k / (2.0 * s * s));
            c->taps[off + k] = (float)e;
            c->taps[off + (r + 1) + k] = (float)(-(double)k / (s * s) * e);
            c->taps[off + 2 * (r + 1) + k] = (float)(((double)k * k / (s * s * s * s) - 1.0 / (s * s)) * e);
        }
        off += 3 * (r + 1);
        if (r > R) R = r;
    }
    c->N = p->n_orient;
    c->second = p->second_order;
    c->z = p->n_orient * (p->second_order ? 2 : 1);
    int rmax = 0;
    for (int i = 0; i < p->n_dil; ++i) rmax = p->dil[i] > rmax ? p->dil[i] : rmax;
    c->K = p->K;
    c->Q = p->K * rmax;
    c->R = R;
    c->ndil = p->n_dil;
    for (int i = 0; i < p->n_dil; ++i) c->dil[i] = p->dil[i];
    for (int k = 0; k < p->n_orient; ++k) {
        const double th = k * M_PI / p->n_orient;   // Section 2.1: directions k*pi/N
        const double cs = cos(th), sn = sin(th);
        c->c1[k] = (float)cs;
        c->s1[k] = (float)sn;
        c->cc[k] = (float)(cs * cs);
        c->ss[k] = (float)(sn * sn);
        c->sc2[k] = (float)(2.0 * sn * cs);
    }
    for (int l = 0; l < 2; ++l) {
        const double sd = l ? p->sd2 : p->sd1;
        double w[5], sum = 0.0;
        for (int i = -p->K; i <= p->K; ++i) {
            w[i + p->K] = exp(-(double)i * i / (2.0 * sd * sd));
            sum += w[i + p->K];
        }
        const int B = 2 * p->K + 1;
        for (int i = 0; i < B; ++i)
            for (int j = 0; j < B; ++j) {
                const float v = (float)((w[i] / sum) * (w[j] / sum));
                (l ? c->w2 : c->w1)[i * B + j] = v;
            }
    }
    c->eps = (float)p->eps;
    c->rectify = p->rectify;
    c->dtype = p->desc_dtype;
    return SFOC_OK;
}

size_t describe_ws_bytes(int64_t H, int64_t W) {
    return align_up((size_t)integ_agg(H, W).total * sizeof(double), 256);
}

size_t tile_mask_bytes(int64_t H, int64_t W) {
    const IntegAgg g = integ_agg(H, W);
    return align_up((size_t)(g.ntx * g.nty), 256);
}

MatchPlan match_plan_L(int32_t n, int32_t m, int32_t r, int L) {
    MatchPlan p{0, 1, 0, 0};
    if (L == kDirectSide) {
        if (n >= 0 && direct_ok(m, r, SFOC_DTYPE_BF16)) {
            p.L = kDirectSide;
            p.Vb = 2 * r + 1;
        }
        return p;
    }
    if (m < 3 || m > kMaxTemplate || r < 1 || r > kMaxRadiusMatch || n < 0 || side_index(L) < 0) return p;
    const int M = m + 2 * r, V = 2 * r + 1;
    if (M <= L) {
        p.L = L;
        p.Vb = V;
    } else if (m <= L - 1) {
        // offsets split so that each block's search window fits L x L
        p.L = L;
        p.Vb = L - m + 1;
        p.nb = (V + p.Vb - 1) / p.Vb;
        p.ws_bytes = align_up((size_t)n * V * V * sizeof(float), 256) +
                     align_up((size_t)n * p.nb * p.nb * 4 * sizeof(float), 256);
    }
    return p;
}

size_t match_window_ws_bytes(int32_t n, int32_t m, int32_t r) {
    const size_t W1 = (size_t)(m + 2 * r + 1);
    return align_up((size_t)n * 2 * W1 * W1 * sizeof(double), 256);
}

// Transform work of one IP under a plan, in units of L^2 log2(L^2).
static double plan_cost(const MatchPlan& p) {
    const double L2 = (double)p.L * p.L;
    return (double)p.nb * p.nb * L2 * log2(L2);
}

MatchPlan match_plan(int32_t n, int32_t m, int32_t r) {
    // (the bounds also keep m + 2r far from int overflow)
    if (m < 3 || r < 1 || m > kMaxTemplate || r > kMaxRadiusMatch) return MatchPlan{0, 1, 0, 0};
    const int M = m + 2 * r;
    for (int k = 0; k < kNumSides; ++k)
        if (M <= kSides[k]) return match_plan_L(n, m, r, kSides[k]);
    MatchPlan best{0, 1, 0, 0};
    for (int k = 0; k < kNumSides; ++k) {
        const MatchPlan q = match_plan_L(n, m, r, kSides[k]);
        if (q.L != 0 && (best.L == 0 || plan_cost(q) < plan_cost(best))) best = q;
    }
    return best;
}

int match_candidates(int32_t m, int32_t r, int* Ls) {
    const MatchPlan d = match_plan(1, m, r);
    if (d.L == 0) return 0;
    int k = 0;
    Ls[k++] = d.L;
    for (int j = 0; j < kNumSides; ++j) {
        if (kSides[j] == d.L) continue;
        const MatchPlan o = match_plan_L(1, m, r, kSides[j]);
        if (o.L != 0 && o.nb <= kMaxTuneBlocks && o.Vb >= 2) Ls[k++] = kSides[j];
    }
    return k;
}

MatchPlan match_plan_dt(int32_t n, int32_t m, int32_t r, int32_t dtype) {
    return direct_ok(m, r, dtype) ? match_plan_L(n, m, r, kDirectSide) : match_plan(n, m, r);
}

int plan_candidates(int32_t m, int32_t r, int32_t dtype, int* Ls) {
    if (!direct_ok(m, r, dtype)) return match_candidates(m, r, Ls);
    Ls[0] = kDirectSide;
    return 1 + match_candidates(m, r, Ls + 1);
}

static bool is_candidate(int m, int r, int dtype, int L) {
    int Ls[kNumForms];
    const int n = plan_candidates(m, r, dtype, Ls);
    for (int k = 0; k < n; ++k)
        if (Ls[k] == L) return true;
    return false;
}

// One integer field of a cache line: optional sign and decimal digits,
// within [-2^30, 2^30]; false on anything else.
static bool parse_field(const char* tok, int* out) {
    if (!tok) return false;
    char* end = nullptr;
    errno = 0;
    const long v = strtol(tok, &end, 10);
    if (errno != 0 || end == tok || *end != '\0' || v < -(1L << 30) || v > (1L << 30)) return false;
    *out = (int)v;
    return true;
}

TuneCache tune_cache_read(const char* path) {
    TuneCache cache;
    if (!path) return cache;
    FILE* f = fopen(path, "r");
    if (!f) return cache;
    char line[512];
    while (fgets(line, sizeof line, f)) {
        // exactly six whitespace-separated fields: device z dtype m r L
        char* save = nullptr;
        const char* tok[7];
        int nt = 0;
        for (char* t = strtok_r(line, " \t\r\n", &save); t && nt < 7; t = strtok_r(nullptr, " \t\r\n", &save))
            tok[nt++] = t;
        if (nt != 6 || strlen(tok[0]) >= 160) continue;
        int v[5];
        bool ok = true;
        for (int k = 0; k < 5 && ok; ++k) ok = parse_field(tok[k + 1], &v[k]);
        if (!ok) continue;
        const int z = v[0], dt = v[1], m = v[2], r = v[3], L = v[4];
        if (z < 1 || dtype_size(dt) == 0 || !is_candidate(m, r, dt, L)) continue;
        cache[TuneKey(tok[0], z, dt, m, r)] = L;
    }
    fclose(f);
    return cache;
}

bool tune_cache_write(const char* path, const TuneCache& cache) {
    if (!path) return false;
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = fopen(tmp.c_str(), "w");
    if (!f) return false;
    bool ok = true;
    for (const auto& kv : cache)
        ok = ok && fprintf(f, "%s %d %d %d %d %d\n", std::get<0>(kv.first).c_str(), std::get<1>(kv.first),
                           std::get<2>(kv.first), std::get<3>(kv.first), std::get<4>(kv.first), kv.second) > 0;
    ok = (fclose(f) == 0) && ok;
    if (ok) ok = rename(tmp.c_str(), path) == 0;
    else remove(tmp.c_str());
    return ok;
}

int tune_cache_lookup(const TuneCache& cache, const std::string& dev, int z, int dtype, int m, int r) {
    const auto it = cache.find(TuneKey(dev, z, dtype, m, r));
    if (it == cache.end() || !is_candidate(m, r, dtype, it->second)) return 0;
    return it->second;
}

void sensed_tiles(const int32_t* ips, const int32_t* prior, int32_t n, int32_t m, int32_t r, int64_t Hs,
                  int64_t Ws, int64_t Hr, int64_t Wr, int T, int cover, std::vector<std::pair<int, int>>& out) {
    out.clear();
    if (cover == kCoverSmaller) {
        std::vector<std::pair<int, int>> g;
        sensed_tiles(ips, prior, n, m, r, Hs, Ws, Hr, Wr, T, kCoverTemplate, out);
        sensed_tiles(ips, prior, n, m, r, Hs, Ws, Hr, Wr, T, kCoverGrid, g);
        if (g.size() < out.size()) out.swap(g);
        return;
    }
    std::set<std::pair<int, int>> seen;
    for (int32_t i = 0; i < n; ++i) {
        int64_t ty, tx;
        if (!template_tile_range(ips[2 * i], ips[2 * i + 1], prior ? prior[2 * i] : 0, prior ? prior[2 * i + 1] : 0,
                                 m, r, Hs, Ws, Hr, Wr, &ty, &tx))
            continue;
        if (cover == kCoverGrid) {
            for (int64_t a = ty / T; a <= (ty + m - 1) / T; ++a)
                for (int64_t b = tx / T; b <= (tx + m - 1) / T; ++b)
                    seen.insert(std::pair<int, int>((int)(a * T), (int)(b * T)));
            continue;
        }
        for (int a = 0; a < template_tile_rows(m, T); ++a)
            for (int c = 0; c < template_tile_rows(m, T); ++c) {
                const std::pair<int, int> o((int)(ty + (int64_t)a * T), (int)(tx + (int64_t)c * T));
                if (seen.insert(o).second) out.push_back(o);
            }
    }
    if (cover == kCoverGrid) out.assign(seen.begin(), seen.end());   // row-major
}

void window_tile_mask(const int32_t* ips, const int32_t* prior, int32_t n, int32_t m, int32_t r, int64_t Hs,
                      int64_t Ws, int64_t Hr, int64_t Wr, int T, uint8_t* mask) {
    const int64_t ntx = (Wr + T - 1) / T, nty = (Hr + T - 1) / T;
    memset(mask, 0, (size_t)(ntx * nty));
    for (int32_t i = 0; i < n; ++i) {
        int64_t a0, a1, b0, b1;
        if (!window_tile_range(ips[2 * i], ips[2 * i + 1], prior ? prior[2 * i] : 0, prior ? prior[2 * i + 1] : 0, m,
                               r, Hs, Ws, Hr, Wr, T, &a0, &a1, &b0, &b1))
            continue;
        for (int64_t a = a0; a <= a1; ++a)
            for (int64_t b = b0; b <= b1; ++b) mask[a * ntx + b] = 1;
    }
}

}  // namespace sfoc
