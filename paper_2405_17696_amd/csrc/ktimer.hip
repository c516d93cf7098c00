// Per-kernel event timer and algorithmic-work counter (diagnostics).
#include <algorithm>
#include <string>
#include <utility>
#include <vector>

#include "common.h"

namespace helm {

namespace {
struct TimerState {
    std::string name;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;   // eager launches
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    unsigned long long* dcount = nullptr;
    hipEvent_t pending = nullptr;
    hipEvent_t ref = nullptr;  // recorded at the start: the origin of the launch intervals
    int period = 1;            // every period-th launch is sampled
    long long launches = 0;    // launches of the named kernel since the start
    bool sample = true;        // whether the next launch is sampled
    bool by_step = false;      // sample whole restart cycles, not single launches
    long long steps = 0;       // restart cycles since the start
};
TimerState g_t;

// Fence-free events (no system-scope release): the timestamps stay exact and
// the packets cost far less than default events between back-to-back kernels.
hipEvent_t take_event() {
    if (g_t.used < g_t.pool.size()) return g_t.pool[g_t.used++];
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    g_t.pool.push_back(e);
    g_t.used++;
    return e;
}
}  // namespace

static bool named(const char* name) { return !g_t.name.empty() && g_t.name == name; }
bool KTimer::armed(const char* name) const { return named(name) && g_t.sample; }
unsigned long long* KTimer::counter() const { return g_t.dcount; }
static bool stream_capturing(hipStream_t s) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(s, &cs) == hipSuccess && cs == hipStreamCaptureStatusActive;
}
bool KTimer::capturing(hipStream_t s) const { return stream_capturing(s); }
// Launches inside a stream capture are not timed: a replayed graph has no
// per-launch events (the timed measurements launch eagerly).
void KTimer::begin(hipStream_t s) {
    g_t.pending = nullptr;
    if (stream_capturing(s)) return;
    hipEvent_t e = take_event();
    if (e && hipEventRecord(e, s) == hipSuccess) g_t.pending = e;
}
void KTimer::end(hipStream_t s) {
    if (!g_t.pending) return;
    hipEvent_t e = take_event();
    if (e && hipEventRecord(e, s) == hipSuccess) g_t.ev.push_back({g_t.pending, e});
    g_t.pending = nullptr;
}
// A launch is sampled when a multiplicative hash of its index falls in the
// lowest 1/period of the 32-bit range: on average every period-th launch, but
// not in step with the number of launches per network application (a fixed
// stride would sample the same few layers whenever the two share a factor).
void KTimer::next(const char* name, hipStream_t s) {
    if (!named(name) || stream_capturing(s)) return;
    ++g_t.launches;
    if (g_t.by_step) return;
    const unsigned h = (unsigned)g_t.launches * 2654435761u;
    g_t.sample = g_t.period <= 1 || h < 0xFFFFFFFFu / (unsigned)g_t.period;
}
// The same hash over the index of the restart cycle: every launch of the
// family inside a sampled cycle is timed, on whichever stream it runs, so that
// the union of their intervals is the family's busy time in that cycle even
// when two streams overlap (they join at the end of every cycle).
void KTimer::step(hipStream_t s) {
    if (!g_t.by_step || g_t.name.empty() || stream_capturing(s)) return;
    ++g_t.steps;
    const unsigned h = (unsigned)g_t.steps * 2654435761u;
    g_t.sample = g_t.period <= 1 || h < 0xFFFFFFFFu / (unsigned)g_t.period;
}
void KTimer::replayed() {}
void KTimer::harvest() {}
void KTimer::new_capture() {}
KTimer& ktimer() {
    static KTimer t;
    return t;
}

}  // namespace helm

using namespace helm;

extern "C" int helm_ktimer_start(const char* kernel) {
    if (hipDeviceSynchronize() != hipSuccess) return fail(HELM_EHIP, "helm_ktimer_start: device sync failed");
    g_t.ev.clear();
    g_t.used = 0;
    g_t.name = kernel ? kernel : "";
    g_t.launches = 0;
    g_t.steps = 0;
    g_t.sample = true;
    if (!g_t.ref && hipEventCreateWithFlags(&g_t.ref, hipEventDisableSystemFence) != hipSuccess) {
        g_t.ref = nullptr;
        return fail(HELM_EHIP, "helm_ktimer_start: event creation failed");
    }
    if (hipEventRecord(g_t.ref, nullptr) != hipSuccess) return fail(HELM_EHIP, "helm_ktimer_start: event record failed");
    if (kernel) {
        const size_t bytes = sizeof(unsigned long long) * WORK_SLOTS * WORK_SLOT_STRIDE;
        if (!g_t.dcount && hipMalloc(&g_t.dcount, bytes) != hipSuccess)
            return fail(HELM_ENOMEM, "helm_ktimer_start: counter allocation failed");
        if (hipMemset(g_t.dcount, 0, bytes) != hipSuccess)
            return fail(HELM_EHIP, "helm_ktimer_start: counter reset failed");
    }
    return HELM_OK;
}

extern "C" int helm_ktimer_sample(int every) {
    if (every < 1) return fail(HELM_EINVAL, "helm_ktimer_sample: every must be >= 1, got %d", every);
    g_t.period = every;
    g_t.by_step = false;
    return HELM_OK;
}

extern "C" int helm_ktimer_sample_steps(int every) {
    if (every < 1) return fail(HELM_EINVAL, "helm_ktimer_sample_steps: every must be >= 1, got %d", every);
    g_t.period = every;
    g_t.by_step = true;
    return HELM_OK;
}

extern "C" int helm_ktimer_count(long long* launches) {
    if (!launches) return fail(HELM_EINVAL, "helm_ktimer_count: NULL output");
    *launches = g_t.launches;
    return HELM_OK;
}

extern "C" int helm_ktimer_read(int* launches, double* total_ms, double* total_work) {
    if (hipDeviceSynchronize() != hipSuccess) return fail(HELM_EHIP, "helm_ktimer_read: device sync failed");
    double ms = 0;
    for (auto& p : g_t.ev) {
        float t = 0;
        if (hipEventElapsedTime(&t, p.first, p.second) != hipSuccess)
            return fail(HELM_EHIP, "helm_ktimer_read: elapsed time failed");
        ms += t;
    }
    unsigned long long w = 0;
    if (g_t.dcount) {
        std::vector<unsigned long long> slots(WORK_SLOTS * WORK_SLOT_STRIDE);
        if (hipMemcpy(slots.data(), g_t.dcount, sizeof(unsigned long long) * slots.size(), hipMemcpyDeviceToHost) !=
            hipSuccess)
            return fail(HELM_EHIP, "helm_ktimer_read: counter read failed");
        for (int i = 0; i < WORK_SLOTS; ++i) w += slots[(size_t)i * WORK_SLOT_STRIDE];
    }
    if (launches) *launches = (int)g_t.ev.size();
    if (total_ms) *total_ms = ms;
    if (total_work) *total_work = (double)w;
    return HELM_OK;
}

extern "C" int helm_ktimer_busy(double* busy_ms) {
    if (!busy_ms) return fail(HELM_EINVAL, "helm_ktimer_busy: NULL output");
    if (hipDeviceSynchronize() != hipSuccess) return fail(HELM_EHIP, "helm_ktimer_busy: device sync failed");
    std::vector<std::pair<float, float>> iv;
    iv.reserve(g_t.ev.size());
    for (auto& p : g_t.ev) {
        float a = 0, b = 0;
        if (!g_t.ref || hipEventElapsedTime(&a, g_t.ref, p.first) != hipSuccess ||
            hipEventElapsedTime(&b, g_t.ref, p.second) != hipSuccess)
            return fail(HELM_EHIP, "helm_ktimer_busy: elapsed time failed");
        iv.push_back({a, b});
    }
    std::sort(iv.begin(), iv.end());
    double busy = 0, lo = 0, hi = -1;
    for (auto& x : iv) {
        if (x.first > hi) {
            if (hi > lo) busy += hi - lo;
            lo = x.first;
            hi = x.second;
        } else if (x.second > hi) {
            hi = x.second;
        }
    }
    if (hi > lo) busy += hi - lo;
    *busy_ms = busy;
    return HELM_OK;
}
