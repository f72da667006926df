// Per-kernel HIP-event timing (sfoc_trace_enable / sfoc_trace_collect).
#include "sfoc_trace.h"

#include <vector>

#include "sfoc.h"

namespace sfoc {

struct TraceRec {
    hipEvent_t a, b;
    int kid;
};

static bool g_on = false;
static std::vector<hipEvent_t> g_pool;     // created lazily, reused
static std::vector<TraceRec> g_recs;
static size_t g_next = 0;                   // next free pool event
static int g_open = -1;                     // index of the record awaiting its end

static hipEvent_t take_event() {
    if (g_next < g_pool.size()) return g_pool[g_next++];
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    g_pool.push_back(e);
    ++g_next;
    return e;
}

// Launches recorded into a graph under stream capture are not timed.
static bool capturing(hipStream_t st) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

void trace_begin(hipStream_t st, int kid) {
    if (!g_on || g_recs.size() >= SFOC_TRACE_MAX || capturing(st)) return;
    hipEvent_t a = take_event(), b = take_event();
    if (!a || !b) return;
    hipEventRecord(a, st);
    g_recs.push_back({a, b, kid});
    g_open = (int)g_recs.size() - 1;
}

void trace_end(hipStream_t st, int kid) {
    if (!g_on || g_open < 0 || g_recs[g_open].kid != kid || capturing(st)) return;
    hipEventRecord(g_recs[g_open].b, st);
    g_open = -1;
}

}  // namespace sfoc

using namespace sfoc;

extern "C" int sfoc_trace_enable(int on) {
    g_on = on != 0;
    return SFOC_OK;
}

extern "C" int sfoc_trace_collect(double* ms, int64_t* counts, int n) {
    if (n < 0 || (n > 0 && (!ms || !counts))) return SFOC_E_INVALID_ARG;
    for (int k = 0; k < n; ++k) {
        ms[k] = 0.0;
        counts[k] = 0;
    }
    int rc = SFOC_OK;
    for (const TraceRec& r : g_recs) {
        if (hipEventSynchronize(r.b) != hipSuccess) {
            rc = SFOC_E_HIP;
            continue;
        }
        float t = 0.f;
        if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) {
            rc = SFOC_E_HIP;
            continue;
        }
        if (r.kid >= 0 && r.kid < n) {
            ms[r.kid] += t;
            counts[r.kid] += 1;
        }
    }
    g_recs.clear();
    g_next = 0;
    g_open = -1;
    return rc == SFOC_OK ? (n < SFOC_K_COUNT ? n : SFOC_K_COUNT) : rc;
}
