// Per-launch HIP-event timing of the library's kernels (instrumentation for
// measuring each kernel class against its roofline while the real loop runs).
#include <algorithm>
#include <utility>
#include <vector>

#include "flame_internal.h"

namespace flame {

namespace {

struct Rec {
    int kclass;
    hipEvent_t a, b;
    double flops, bytes;
};

struct TraceState {
    bool on = false;
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
};

thread_local TraceState g_tr;

hipEvent_t pool_event() {
    if (g_tr.used == g_tr.pool.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        g_tr.pool.push_back(e);
    }
    return g_tr.pool[g_tr.used++];
}

}  // namespace

int trace_begin(int kclass, hipStream_t s) {
    if (!g_tr.on) return -1;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return -1;
    Rec r{kclass, pool_event(), pool_event(), 0.0, 0.0};
    if (r.a == nullptr || r.b == nullptr) return -1;
    if (hipEventRecord(r.a, s) != hipSuccess) return -1;
    g_tr.recs.push_back(r);
    return (int)g_tr.recs.size() - 1;
}

void trace_end(int id, hipStream_t s, double flops, double bytes) {
    if (id < 0) return;
    Rec &r = g_tr.recs[id];
    r.flops = flops;
    r.bytes = bytes;
    (void)hipEventRecord(r.b, s);
}

}  // namespace flame

using namespace flame;

extern "C" int flame_trace_enable(int32_t on) {
    g_tr.on = (on != 0);
    g_tr.recs.clear();
    g_tr.used = 0;
    return FLAME_OK;
}

extern "C" int flame_trace_collect(int64_t *launches, double *ms, double *flops, double *bytes) {
    int64_t L[FLAME_KC_COUNT] = {0, 0, 0, 0};
    double T[FLAME_KC_COUNT] = {0, 0, 0, 0}, F[FLAME_KC_COUNT] = {0, 0, 0, 0}, B[FLAME_KC_COUNT] = {0, 0, 0, 0};
    for (const Rec &r : g_tr.recs) {
        FLAME_HIP(hipEventSynchronize(r.b));
        float t = 0.f;
        FLAME_HIP(hipEventElapsedTime(&t, r.a, r.b));
        L[r.kclass] += 1;
        T[r.kclass] += t;
        F[r.kclass] += r.flops;
        B[r.kclass] += r.bytes;
    }
    for (int k = 0; k < FLAME_KC_COUNT; ++k) {
        if (launches) launches[k] = L[k];
        if (ms) ms[k] = T[k];
        if (flops) flops[k] = F[k];
        if (bytes) bytes[k] = B[k];
    }
    return FLAME_OK;
}

extern "C" int flame_trace_busy(double *busy_ms, double *span_ms) {
    double B[FLAME_KC_COUNT] = {0, 0, 0, 0};
    double span = 0.0;
    if (!g_tr.recs.empty()) {
        // every interval on one clock: milliseconds since the first record's start
        const hipEvent_t ref = g_tr.recs.front().a;
        std::vector<std::pair<double, double>> iv[FLAME_KC_COUNT];
        for (const Rec &r : g_tr.recs) {
            FLAME_HIP(hipEventSynchronize(r.b));
            float t0 = 0.f, t1 = 0.f;
            FLAME_HIP(hipEventElapsedTime(&t0, ref, r.a));
            FLAME_HIP(hipEventElapsedTime(&t1, ref, r.b));
            iv[r.kclass].emplace_back((double)t0, (double)t1);
            span = std::max(span, (double)t1);
        }
        for (int k = 0; k < FLAME_KC_COUNT; ++k) {
            auto &v = iv[k];
            std::sort(v.begin(), v.end());
            double cur0 = 0.0, cur1 = -1.0, sum = 0.0;
            for (const auto &p : v) {
                if (p.first > cur1) {
                    if (cur1 > cur0) sum += cur1 - cur0;
                    cur0 = p.first;
                    cur1 = p.second;
                } else {
                    cur1 = std::max(cur1, p.second);
                }
            }
            if (cur1 > cur0) sum += cur1 - cur0;
            B[k] = sum;
        }
    }
    for (int k = 0; k < FLAME_KC_COUNT; ++k)
        if (busy_ms) busy_ms[k] = B[k];
    if (span_ms) *span_ms = span;
    return FLAME_OK;
}
