// Batched plans: many image pairs of uneven sizes, templates and radii run
// as one describe launch, one set of integral-image scans, one match launch
// per transform side, one peak and one consistency launch, optionally
// captured into a hipGraph.  Each pair's arithmetic is exactly the per-pair
// path's (the kernels are shared; only where their arguments come from
// differs).  A timing autotuner picks the transform side per (m, r) class.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "sfoc_launch.h"

using namespace sfoc;

struct sfoc_plan {
    int device = 0;
    sfoc_params p{};
    DescribeConsts c{};
    int32_t z = 0, dtype = 0, flags = 0;
    std::vector<sfoc_pair> pairs;
    std::vector<int> side;          // chosen transform side per pair
    std::vector<MatchPlan> mp;      // its layout
    char* mem = nullptr;            // one device allocation
    size_t bytes = 0;
    DescribeJob* djobs = nullptr;
    int4* dtiles = nullptr;
    int ndt = 0, ndt_ref = 0;   // all tiles; reference tiles (first)
    int dvar = 0;               // describe launch configuration (describe_configs)
    IntegJob* ijobs = nullptr;
    int4* ipre = nullptr;     // integral prefix items (integral_prefix_items)
    int4* itiles = nullptr;   // integral tiles {job, tile row, tile column}
    int npre = 0, nitiles = 0;
    MatchArgs* margs = nullptr;
    int4* items[kNumForms] = {};        // per launch form kForms[b]
    int nitems[kNumForms] = {};
    int4* peak = nullptr;
    int npeak = 0;
    int* counters = nullptr;            // work counters of the persistent launches (one per form)
    bool persist[kNumForms] = {};       // persistent match launch per transform side
    DirLaunch dir{3, 1};                // size of the direct launch (largest over its pairs)
    int grid = 0;                       // CUs (a persistent grid has MINB workgroups per CU)
    hipStream_t side_stream = nullptr;   // second graph branch
    hipStream_t cap_stream = nullptr;    // capture happens here (the caller's may be the null stream)
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;     // match sides
    hipEvent_t ev_fork2 = nullptr, ev_join2 = nullptr;   // integral scans beside the sensed describe
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int tuned = 0, cached = 0;
};

namespace {

// Device memory of one pair inside the plan's allocation.
struct PairMem {
    size_t dref, dsen, i1, i2, scan, ws;
};

struct Cursor {
    size_t off = 0;
    size_t take(size_t n) {
        const size_t o = off;
        off = align_up(off + n, 256);
        return o;
    }
};

int bucket_of(int L) { return form_index(L); }

MatchArgs make_args(const sfoc_pair& q, const char* mem, const PairMem& pm, int32_t z, int32_t dtype,
                    const MatchPlan& mp) {
    MatchArgs a{};
    a.desc_sen = mem + pm.dsen;
    a.desc_ref = mem + pm.dref;
    a.integ1 = (const double*)(mem + pm.i1);
    a.integ2 = (const double*)(mem + pm.i2);
    a.ips = q.ips;
    a.prior = q.prior;
    a.ncc = q.ncc;
    a.cps = q.cps;
    a.Hs = q.Hs;
    a.Ws = q.Ws;
    a.Hr = q.Hr;
    a.Wr = q.Wr;
    a.z = z;
    a.dtype = dtype;
    a.n = q.n;
    a.m = q.m;
    a.r = q.r;
    match_args_layout(a, mp, (void*)(mem + pm.ws));
    return a;
}

// Match items of one pair: (pair, IP, block) for every IP and block.
void append_items(std::vector<int4>& out, int pair, int n, int nb) {
    const int nblk = nb * nb;
    for (int i = 0; i < n; ++i)
        for (int b = 0; b < nblk; ++b) out.push_back(make_int4(pair, i, b, 0));
}

// Autotuner cache key of a device: architecture and CU count.
std::string device_key(int dev) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    char buf[160];
    snprintf(buf, sizeof buf, "%s/%dcu", prop.gcnArchName, prop.multiProcessorCount);
    for (char* c = buf; *c; ++c)
        if (*c == ' ') *c = '_';
    return buf;
}

// Everything after the describe / integral stage for the plan's current
// tables.  The side-64 launch runs on a second stream (a second graph
// branch) beside the larger sides, which run in turn on the caller's.
hipError_t enqueue_match(sfoc_plan* P, hipStream_t st) {
    hipError_t e = hipSuccess;
    bool big = false;
    for (int b = 1; b < kNumForms; ++b) big = big || P->nitems[b] > 0;
    const bool fork = P->nitems[0] > 0 && big;
    if (fork) {
        if ((e = hipEventRecord(P->ev_fork, st)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(P->side_stream, P->ev_fork, 0)) != hipSuccess) return e;
    }
    for (int b = 0; b < kNumForms; ++b) {
        e = launch_match_items(kForms[b], P->dtype, P->margs, P->items[b], P->nitems[b],
                               P->persist[b] ? P->counters + b : nullptr, P->grid, P->dir,
                               b == 0 && fork ? P->side_stream : st);
        if (e != hipSuccess) return e;
        if (b == 0 && fork && (e = hipEventRecord(P->ev_join, P->side_stream)) != hipSuccess) return e;
    }
    if (fork && (e = hipStreamWaitEvent(st, P->ev_join, 0)) != hipSuccess) return e;
    if ((e = launch_peak_batched(P->margs, P->peak, P->npeak, st)) != hipSuccess) return e;
    return launch_consistency_batched(P->margs, (int)P->pairs.size(), st);
}

// Reference descriptors, then the integral scans on the second branch while
// the sensed tiles are described, then the match.
hipError_t enqueue_all(sfoc_plan* P, hipStream_t st) {
    hipError_t e = launch_describe_batched(P->djobs, P->dtiles, P->ndt_ref, P->c, st, P->dvar);
    if (e == hipSuccess) e = hipEventRecord(P->ev_fork2, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(P->side_stream, P->ev_fork2, 0);
    if (e == hipSuccess)
        e = launch_integral_batched(P->ijobs, P->ipre, P->npre, P->itiles, P->nitiles, P->side_stream);
    if (e == hipSuccess) e = hipEventRecord(P->ev_join2, P->side_stream);
    if (e == hipSuccess)
        e = launch_describe_batched(P->djobs, P->dtiles + P->ndt_ref, P->ndt - P->ndt_ref, P->c, st, P->dvar);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, P->ev_join2, 0);
    if (e == hipSuccess) e = enqueue_match(P, st);
    return e;
}

void free_plan(sfoc_plan* P) {
    if (P->exec) (void)hipGraphExecDestroy(P->exec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    if (P->ev_fork) (void)hipEventDestroy(P->ev_fork);
    if (P->ev_join) (void)hipEventDestroy(P->ev_join);
    if (P->ev_fork2) (void)hipEventDestroy(P->ev_fork2);
    if (P->ev_join2) (void)hipEventDestroy(P->ev_join2);
    if (P->side_stream) (void)hipStreamDestroy(P->side_stream);
    if (P->cap_stream) (void)hipStreamDestroy(P->cap_stream);
    if (P->mem) (void)hipFree(P->mem);
    delete P;
}

// Median time of `reps` launches of one candidate side over `items`.
float time_items(int L, int dtype, const MatchArgs* margs, const int4* items, int nitems, int* counter, int grid,
                 DirLaunch dir, hipStream_t st, int reps, hipError_t* err) {
    hipEvent_t a, b;
    *err = hipEventCreate(&a);
    if (*err != hipSuccess) return 0.f;
    *err = hipEventCreate(&b);
    if (*err != hipSuccess) {
        (void)hipEventDestroy(a);
        return 0.f;
    }
    std::vector<float> t;
    *err = launch_match_items(L, dtype, margs, items, nitems, counter, grid, dir, st);   // warm-up
    for (int k = 0; k < reps && *err == hipSuccess; ++k) {
        *err = hipEventRecord(a, st);
        if (*err == hipSuccess) *err = launch_match_items(L, dtype, margs, items, nitems, counter, grid, dir, st);
        if (*err == hipSuccess) *err = hipEventRecord(b, st);
        if (*err == hipSuccess) *err = hipEventSynchronize(b);
        float ms = 0.f;
        if (*err == hipSuccess) *err = hipEventElapsedTime(&ms, a, b);
        t.push_back(ms);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (t.empty()) return 0.f;
    std::sort(t.begin(), t.end());
    return t[t.size() / 2];
}

// Median time of the plan's whole describe launch in configuration var.
float time_describe(const sfoc_plan* P, int var, hipStream_t st, int reps, hipError_t* err) {
    hipEvent_t a, b;
    *err = hipEventCreate(&a);
    if (*err != hipSuccess) return 0.f;
    *err = hipEventCreate(&b);
    if (*err != hipSuccess) {
        (void)hipEventDestroy(a);
        return 0.f;
    }
    std::vector<float> t;
    *err = launch_describe_batched(P->djobs, P->dtiles, P->ndt, P->c, st, var);   // warm-up
    for (int k = 0; k < reps && *err == hipSuccess; ++k) {
        *err = hipEventRecord(a, st);
        if (*err == hipSuccess) *err = launch_describe_batched(P->djobs, P->dtiles, P->ndt, P->c, st, var);
        if (*err == hipSuccess) *err = hipEventRecord(b, st);
        if (*err == hipSuccess) *err = hipEventSynchronize(b);
        float ms = 0.f;
        if (*err == hipSuccess) *err = hipEventElapsedTime(&ms, a, b);
        t.push_back(ms);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (t.empty()) return 0.f;
    std::sort(t.begin(), t.end());
    return t[t.size() / 2];
}

}  // namespace

extern "C" {

int sfoc_plan_create(const sfoc_pair* pairs, int32_t n_pairs, const sfoc_params* p, int32_t flags,
                     const char* tune_cache, void* stream, sfoc_plan** plan) {
    if (!plan || !pairs || n_pairs < 1) return SFOC_E_INVALID_ARG;
    *plan = nullptr;
    if (flags & ~(SFOC_PLAN_GRAPH | SFOC_PLAN_AUTOTUNE | SFOC_PLAN_DENSE_SEN | SFOC_PLAN_PERSISTENT |
                  SFOC_PLAN_DESCRIBE_ALT))
        return SFOC_E_INVALID_ARG;
    int32_t z = 0;
    int rc = check_params(p, &z);
    if (rc) return rc;
    const size_t es = dtype_size(p->desc_dtype);
    const bool tune = (flags & SFOC_PLAN_AUTOTUNE) != 0;
    const bool sparse = !(flags & SFOC_PLAN_DENSE_SEN);
    // ---- validation (the checks of sfoc_register_cps, per pair) ----
    for (int k = 0; k < n_pairs; ++k) {
        const sfoc_pair& q = pairs[k];
        if ((rc = check_image(q.ref, q.Hr, q.Wr, q.ldr))) return rc;
        if ((rc = check_image(q.sen, q.Hs, q.Ws, q.lds))) return rc;
        if ((rc = check_match_shape(q.n, q.m, q.r))) return rc;
        if (q.Hs * q.Ws >= kMaxPlane || q.Hr * q.Wr >= kMaxPlane) return SFOC_E_UNSUPPORTED;
        if (q.n > 0 && (!q.ips || !q.cps)) return SFOC_E_INVALID_ARG;
        if (q.fft_side != 0 && form_index(q.fft_side) < 0) return SFOC_E_INVALID_ARG;
        if (q.fft_side != 0 && match_plan_L(q.n, q.m, q.r, q.fft_side).L == 0) return SFOC_E_UNSUPPORTED;
        if (q.fft_side == kDirectSide && !direct_ok(q.m, q.r, p->desc_dtype)) return SFOC_E_UNSUPPORTED;
    }
    hipStream_t st = (hipStream_t)stream;
    sfoc_plan* P = new sfoc_plan;
    P->p = *p;
    build_describe_consts(p, &P->c);
    P->z = z;
    P->dtype = p->desc_dtype;
    P->flags = flags;
    P->pairs.assign(pairs, pairs + n_pairs);
    hipError_t e = hipGetDevice(&P->device);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        free_plan(P);
        return hip_status(e);
    }

    // ---- host copies of the IPs (sparse describe tiles, autotuning) ----
    std::vector<std::vector<int32_t>> hips(n_pairs), hprior(n_pairs);
    if (sparse || tune) {
        for (int k = 0; k < n_pairs && e == hipSuccess; ++k) {
            const sfoc_pair& q = pairs[k];
            if (q.n == 0) continue;
            hips[k].resize(2 * (size_t)q.n);
            e = hipMemcpy(hips[k].data(), q.ips, hips[k].size() * sizeof(int32_t), hipMemcpyDeviceToHost);
            if (e == hipSuccess && q.prior) {
                hprior[k].resize(2 * (size_t)q.n);
                e = hipMemcpy(hprior[k].data(), q.prior, hprior[k].size() * sizeof(int32_t), hipMemcpyDeviceToHost);
            }
        }
        if (e != hipSuccess) {
            free_plan(P);
            return hip_status(e);
        }
    }

    // ---- describe tiles ----
    const int T = kDescribeTile;
    std::vector<DescribeJob> djobs(2 * (size_t)n_pairs);
    std::vector<int4> dtiles;
    std::vector<std::pair<int, int>> sens;
    // Reference tiles first.  Sparse: the tiles the search windows read are
    // described; the others only get zero aggregates (entries with w = 1,
    // after the rest), so that the integral images stay exact wherever a
    // window reads them, and only the read tiles get integral-image passes.
    std::vector<std::vector<uint8_t>> rmask(n_pairs);
    std::vector<int4> rzero, rread;
    for (int k = 0; k < n_pairs; ++k) {
        const sfoc_pair& q = pairs[k];
        const int ntyr = (int)((q.Hr + T - 1) / T), ntxr = (int)((q.Wr + T - 1) / T);
        if (sparse) {
            rmask[k].assign((size_t)ntyr * ntxr, 0);
            if (q.n > 0)
                window_tile_mask(hips[k].data(), q.prior ? hprior[k].data() : nullptr, q.n, q.m, q.r, q.Hs, q.Ws,
                                 q.Hr, q.Wr, T, rmask[k].data());
        }
        for (int a = 0; a < ntyr; ++a)
            for (int b = 0; b < ntxr; ++b) {
                const bool read = !sparse || rmask[k][(size_t)a * ntxr + b];
                (read ? rread : rzero).push_back(make_int4(2 * k, a * T, b * T, read ? 0 : 1));
            }
    }
    // The describe kernel deals its entries to the eight XCDs as eight
    // contiguous runs; each run gets an eighth of the described tiles.
    {
        const size_t N = rread.size() + rzero.size(), R = N / 8, nc = rread.size();
        size_t ic = 0, iz = 0;
        for (size_t x = 0; x < 8; ++x) {
            const size_t want = (x + 1) * nc / 8 - x * nc / 8;
            for (size_t j = 0; j < R; ++j)
                dtiles.push_back(((j < want && ic < nc) || iz == rzero.size()) ? rread[ic++] : rzero[iz++]);
        }
        while (ic < nc) dtiles.push_back(rread[ic++]);
        while (iz < rzero.size()) dtiles.push_back(rzero[iz++]);
    }
    const int nref_tiles = (int)dtiles.size();
    for (int k = 0; k < n_pairs; ++k) {
        const sfoc_pair& q = pairs[k];
        if (sparse) {   // the tiles over the templates of in-bounds IPs
            if (q.n > 0)
                sensed_tiles(hips[k].data(), q.prior ? hprior[k].data() : nullptr, q.n, q.m, q.r, q.Hs, q.Ws, q.Hr,
                             q.Wr, T, kCoverSmaller, sens);
            else
                sens.clear();
            for (const auto& o : sens) dtiles.push_back(make_int4(2 * k + 1, o.first, o.second, 0));
            continue;
        }
        const int ntys = (int)((q.Hs + T - 1) / T), ntxs = (int)((q.Ws + T - 1) / T);
        for (int a = 0; a < ntys; ++a)
            for (int b = 0; b < ntxs; ++b) dtiles.push_back(make_int4(2 * k + 1, a * T, b * T, 0));
    }

    // ---- memory: per pair descriptors, integrals, scan scratch, match scratch ----
    std::vector<PairMem> pm(n_pairs);
    Cursor cur;
    std::vector<std::vector<int>> cands(n_pairs);
    for (int k = 0; k < n_pairs; ++k) {
        const sfoc_pair& q = pairs[k];
        int Ls[kNumForms];
        int nc = 0;
        if (q.fft_side) {
            Ls[nc++] = q.fft_side;
        } else if (tune) {
            nc = plan_candidates(q.m, q.r, p->desc_dtype, Ls);
        } else {
            Ls[nc++] = match_plan_dt(q.n, q.m, q.r, p->desc_dtype).L;
        }
        cands[k].assign(Ls, Ls + nc);
        size_t ws = 0;
        for (int L : cands[k]) ws = std::max(ws, match_plan_L(q.n, q.m, q.r, L).ws_bytes);
        pm[k].dref = cur.take((size_t)z * q.Hr * q.Wr * es);
        pm[k].dsen = cur.take((size_t)z * q.Hs * q.Ws * es);
        pm[k].i1 = cur.take((size_t)(q.Hr + 1) * (q.Wr + 1) * sizeof(double));
        pm[k].i2 = cur.take((size_t)(q.Hr + 1) * (q.Wr + 1) * sizeof(double));
        pm[k].scan = cur.take(describe_ws_bytes(q.Hr, q.Wr));
        pm[k].ws = cur.take(ws);
    }
    // integral-image work lists: prefix items, then the reference tiles the
    // windows read (every tile when dense)
    std::vector<IntegJob> ijobs(n_pairs);
    std::vector<int4> ipre, itiles;
    size_t max_items[kNumForms] = {}, max_peak = 0;
    DirLaunch dir{3, 1};
    for (int k = 0; k < n_pairs; ++k) {
        const sfoc_pair& q = pairs[k];
        integral_prefix_items(k, (int)q.Hr, (int)q.Wr, ipre);
        const IntegAgg ag = integ_agg(q.Hr, q.Wr);
        for (int a = 0; a < ag.nty; ++a)
            for (int b = 0; b < ag.ntx; ++b)
                if (!sparse || rmask[k][(size_t)a * ag.ntx + b]) itiles.push_back(make_int4(k, a, b, 0));
        for (int L : cands[k]) {
            const MatchPlan m = match_plan_L(q.n, q.m, q.r, L);
            max_items[bucket_of(L)] += (size_t)q.n * m.nb * m.nb;
            if (L == kDirectSide) {
                const DirLaunch d = direct_launch_of(q.m, q.r);
                dir.m = std::max(dir.m, d.m);
                dir.nkb = std::max(dir.nkb, d.nkb);
            }
        }
        max_peak += ((size_t)q.n + 255) / 256;
    }
    const size_t o_djobs = cur.take(djobs.size() * sizeof(DescribeJob));
    const size_t o_dtiles = cur.take(dtiles.size() * sizeof(int4));
    const size_t o_ijobs = cur.take(ijobs.size() * sizeof(IntegJob));
    const size_t o_ipre = cur.take(ipre.size() * sizeof(int4));
    const size_t o_itiles = cur.take(itiles.size() * sizeof(int4));
    const size_t o_margs = cur.take((size_t)n_pairs * sizeof(MatchArgs));
    size_t o_items[kNumForms];
    for (int b = 0; b < kNumForms; ++b) o_items[b] = cur.take(max_items[b] * sizeof(int4));
    const size_t o_peak = cur.take(max_peak * sizeof(int4));
    const size_t o_counters = cur.take(kNumForms * sizeof(int));
    P->bytes = cur.off;
    e = hipMalloc((void**)&P->mem, P->bytes);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&P->side_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&P->ev_fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&P->ev_join, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&P->ev_fork2, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&P->ev_join2, hipEventDisableTiming);
    if (e != hipSuccess) {
        free_plan(P);
        return hip_status(e);
    }
    char* mem = P->mem;
    for (int k = 0; k < n_pairs; ++k) {
        const sfoc_pair& q = pairs[k];
        double* agg = (double*)(mem + pm[k].scan);
        djobs[2 * k] = DescribeJob{q.ref, mem + pm[k].dref, (double*)(mem + pm[k].i1), (double*)(mem + pm[k].i2),
                                   agg, q.ldr, (int)q.Hr, (int)q.Wr};
        djobs[2 * k + 1] = DescribeJob{q.sen, mem + pm[k].dsen, nullptr, nullptr, nullptr, q.lds, (int)q.Hs, (int)q.Ws};
        ijobs[k] = IntegJob{(double*)(mem + pm[k].i1), (double*)(mem + pm[k].i2), agg, (int)q.Hr, (int)q.Wr};
    }
    P->djobs = (DescribeJob*)(mem + o_djobs);
    P->dtiles = (int4*)(mem + o_dtiles);
    P->ndt = (int)dtiles.size();
    P->ndt_ref = nref_tiles;
    P->ijobs = (IntegJob*)(mem + o_ijobs);
    P->ipre = (int4*)(mem + o_ipre);
    P->itiles = (int4*)(mem + o_itiles);
    P->npre = (int)ipre.size();
    P->nitiles = (int)itiles.size();
    P->margs = (MatchArgs*)(mem + o_margs);
    for (int b = 0; b < kNumForms; ++b) P->items[b] = (int4*)(mem + o_items[b]);
    P->dir = dir;
    P->peak = (int4*)(mem + o_peak);
    P->counters = (int*)(mem + o_counters);
    {
        int cus = 0;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, P->device);
        P->grid = cus > 0 ? cus : 1;
    }
    auto up = [&](void* dst, const void* src, size_t n) {
        if (e == hipSuccess && n) e = hipMemcpy(dst, src, n, hipMemcpyHostToDevice);
    };
    up(P->djobs, djobs.data(), djobs.size() * sizeof(DescribeJob));
    up(P->dtiles, dtiles.data(), dtiles.size() * sizeof(int4));
    up(P->ijobs, ijobs.data(), ijobs.size() * sizeof(IntegJob));
    up(P->ipre, ipre.data(), ipre.size() * sizeof(int4));
    up(P->itiles, itiles.data(), itiles.size() * sizeof(int4));
    if (e != hipSuccess) {
        free_plan(P);
        return hip_status(e);
    }

    // ---- describe launch configuration: asked for, or the faster of the
    //      two on this plan's tiles (both give the same descriptors) ----
    const bool two_configs = describe_configs(P->c) == 2;
    P->dvar = two_configs && (flags & SFOC_PLAN_DESCRIBE_ALT) ? 1 : 0;
    if (tune && two_configs && P->ndt > 0) {
        const float t0 = time_describe(P, 0, st, 3, &e);
        const float t1 = e == hipSuccess ? time_describe(P, 1, st, 3, &e) : 0.f;
        if (e != hipSuccess) {
            free_plan(P);
            return hip_status(e);
        }
        P->dvar = t1 < t0 ? 1 : 0;
    }

    // ---- transform side per pair ----
    P->side.assign(n_pairs, 0);
    std::map<std::pair<int, int>, std::vector<int>> classes;   // (m, r) -> pairs still open
    for (int k = 0; k < n_pairs; ++k) {
        if (cands[k].size() == 1) P->side[k] = cands[k][0];
        else classes[{pairs[k].m, pairs[k].r}].push_back(k);
    }
    if (!classes.empty()) {
        const std::string dev = device_key(P->device);
        TuneCache cache = tune_cache_read(tune_cache);
        bool wrote = false;
        bool described = false;
        for (auto& cl : classes) {
            const int m = cl.first.first, r = cl.first.second;
            const TuneKey key(dev, z, P->dtype, m, r);
            int best = tune_cache_lookup(cache, dev, z, P->dtype, m, r);
            if (best != 0) {
                ++P->cached;
            } else {
                if (!described) {   // the candidates are timed on this plan's own descriptors
                    e = launch_describe_batched(P->djobs, P->dtiles, P->ndt, P->c, st, P->dvar);
                    if (e == hipSuccess)
                        e = launch_integral_batched(P->ijobs, P->ipre, P->npre, P->itiles, P->nitiles, st);
                    described = true;
                }
                // at most ~2048 IPs of the class are timed
                float tbest = 0.f;
                int Ls[kNumForms];
                const int nc = plan_candidates(m, r, P->dtype, Ls);
                for (int c = 0; c < nc && e == hipSuccess; ++c) {
                    const int L = Ls[c];
                    std::vector<MatchArgs> margs(n_pairs);
                    std::vector<int4> items;
                    int budget = 2048;
                    for (int k : cl.second) {
                        if (budget <= 0) break;
                        const MatchPlan mpl = match_plan_L(pairs[k].n, m, r, L);
                        margs[k] = make_args(pairs[k], mem, pm[k], z, P->dtype, mpl);
                        append_items(items, k, std::min(pairs[k].n, budget), mpl.nb);
                        budget -= pairs[k].n;
                    }
                    if (items.empty()) break;
                    up(P->margs, margs.data(), margs.size() * sizeof(MatchArgs));
                    int4* dit = P->items[bucket_of(L)];
                    up(dit, items.data(), items.size() * sizeof(int4));
                    if (e != hipSuccess) break;
                    const float t = time_items(L, P->dtype, P->margs, dit, (int)items.size(), nullptr, 0, P->dir, st,
                                               3, &e);
                    if (c == 0 || t < tbest) {
                        tbest = t;
                        best = L;
                    }
                }
                if (e != hipSuccess) break;
                if (best == 0) {
                    best = Ls[0];   // nothing to time (no IPs): the default, not remembered
                } else {
                    cache[key] = best;
                    wrote = true;
                    ++P->tuned;
                }
            }
            for (int k : cl.second) P->side[k] = best;
        }
        if (e != hipSuccess) {
            free_plan(P);
            return hip_status(e);
        }
        if (wrote) (void)tune_cache_write(tune_cache, cache);
    }

    // ---- match work lists; costlier items first ----
    P->mp.resize(n_pairs);
    std::vector<MatchArgs> margs(n_pairs);
    for (int k = 0; k < n_pairs; ++k) {
        P->mp[k] = match_plan_L(pairs[k].n, pairs[k].m, pairs[k].r, P->side[k]);
        margs[k] = make_args(pairs[k], mem, pm[k], z, P->dtype, P->mp[k]);
    }
    std::vector<int> order(n_pairs);
    for (int k = 0; k < n_pairs; ++k) order[k] = k;
    auto cost = [&](int k) {   // rows transformed per item: search block + template
        const MatchPlan& m = P->mp[k];
        return pairs[k].m + std::min(m.Vb, 2 * pairs[k].r + 1) - 1 + pairs[k].m;
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
    std::vector<int4> items[kNumForms], peak;
    for (int k : order) {
        append_items(items[bucket_of(P->side[k])], k, pairs[k].n, P->mp[k].nb);
        if (P->mp[k].nb > 1)
            for (int i = 0; i < pairs[k].n; i += 256) peak.push_back(make_int4(k, i, 0, 0));
    }
    up(P->margs, margs.data(), margs.size() * sizeof(MatchArgs));
    for (int b = 0; b < kNumForms; ++b) {
        up(P->items[b], items[b].data(), items[b].size() * sizeof(int4));
        P->nitems[b] = (int)items[b].size();
    }
    up(P->peak, peak.data(), peak.size() * sizeof(int4));
    P->npeak = (int)peak.size();
    // launch form per side: persistent when asked; with autotuning the
    // faster of the two on this plan's items
    for (int b = 0; b < kNumSides && e == hipSuccess; ++b) {   // the direct form has one launch form
        P->persist[b] = (flags & SFOC_PLAN_PERSISTENT) != 0;
        if (tune && P->nitems[b] > 0) {
            const int L = kSides[b];
            const float tg = time_items(L, P->dtype, P->margs, P->items[b], P->nitems[b], nullptr, 0, P->dir, st, 3,
                                        &e);
            if (e != hipSuccess) break;
            const float tp = time_items(L, P->dtype, P->margs, P->items[b], P->nitems[b], P->counters + b, P->grid,
                                        P->dir, st, 3, &e);
            P->persist[b] = tp < tg;
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        free_plan(P);
        return hip_status(e);
    }
    *plan = P;
    return SFOC_OK;
}

int sfoc_register_cps_batched(sfoc_plan* P, void* stream) {
    if (!P) return SFOC_E_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    if (!(P->flags & SFOC_PLAN_GRAPH)) return hip_status(enqueue_all(P, st));
    hipError_t e = hipSuccess;
    if (!P->exec) {
        // One eager pass first, so that kernel attributes are set outside the
        // capture; then the sequence is captured on the plan's own stream
        // and the graph is launched on the caller's.
        e = enqueue_all(P, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e == hipSuccess) e = hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_status(e);
        const hipError_t ee = enqueue_all(P, P->cap_stream);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(P->cap_stream, &g);
        if (ee != hipSuccess || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return hip_status(ee != hipSuccess ? ee : e);
        }
        e = hipGraphInstantiate(&P->exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g);
            P->exec = nullptr;
            return hip_status(e);
        }
        P->graph = g;
    }
    return hip_status(hipGraphLaunch(P->exec, st));
}

int sfoc_plan_destroy(sfoc_plan* P) {
    if (!P) return SFOC_E_INVALID_ARG;
    // the plan's memory may still be in use by work enqueued on any stream
    (void)hipDeviceSynchronize();
    free_plan(P);
    return SFOC_OK;
}

int sfoc_plan_get_info(const sfoc_plan* P, sfoc_plan_info* info, int32_t* fft_side, int32_t* blocks, int32_t cap) {
    if (!P || !info || cap < 0) return SFOC_E_INVALID_ARG;
    info->n_pairs = (int32_t)P->pairs.size();
    info->describe_tiles = P->ndt;
    for (int b = 0; b < kNumSides; ++b) {
        info->match_items[b] = P->nitems[b];
        info->persistent[b] = P->persist[b];
    }
    info->peak_items = P->npeak;
    info->tuned_classes = P->tuned;
    info->cached_classes = P->cached;
    info->graph = P->exec != nullptr;
    info->describe_config = P->dvar;
    info->direct_items = P->nitems[form_index(kDirectSide)];
    info->device_bytes = (int64_t)P->bytes;
    const int n = std::min<int>(cap, (int)P->pairs.size());
    for (int k = 0; k < n; ++k) {
        if (fft_side) fft_side[k] = P->side[k];
        if (blocks) blocks[k] = P->mp[k].nb;
    }
    return SFOC_OK;
}

}  // extern "C"
