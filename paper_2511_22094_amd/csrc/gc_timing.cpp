// Kernel timing registry (see gacelle.h: gc_timing_*).
#include "gc_timing.hpp"

#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>

#include "../../include/gacelle.h"

namespace gc {

namespace {
std::atomic<int> g_on{0};
std::mutex g_mu;
struct Tot {
    double ms = 0.0;
    int64_t n = 0;
};
std::map<std::string, Tot> g_tot;

// GACELLE_TRACE=<file>: every launch of the timed families is recorded (name,
// device, stream, start and duration from its HIP events) and the list is
// written at process exit as a Chrome trace-event JSON file.  Start times
// are measured from a reference event recorded once per device, after a
// device synchronisation, when the device's first traced launch begins.
struct TraceEv {
    std::string name;
    int dev;
    uintptr_t stream;
    double ts_us, dur_us;
};
struct Trace {
    std::string path;
    std::vector<TraceEv> ev;
    std::map<int, hipEvent_t> ref;
    Trace() {
        const char* p = std::getenv("GACELLE_TRACE");
        if (p && *p) {
            path = p;
            g_on.store(1);
        }
    }
    ~Trace() {
        // host data only: the HIP runtime may already be gone at exit
        if (path.empty()) return;
        FILE* f = std::fopen(path.c_str(), "w");
        if (!f) return;
        std::fprintf(f, "{\"displayTimeUnit\": \"ms\", \"traceEvents\": [\n");
        for (size_t i = 0; i < ev.size(); ++i) {
            const TraceEv& e = ev[i];
            std::fprintf(f,
                         "{\"name\": \"%s\", \"ph\": \"X\", \"pid\": %d, \"tid\": %llu, "
                         "\"ts\": %.3f, \"dur\": %.3f}%s\n",
                         e.name.c_str(), e.dev, (unsigned long long)e.stream, e.ts_us, e.dur_us,
                         i + 1 < ev.size() ? "," : "");
        }
        std::fprintf(f, "]}\n");
        std::fclose(f);
    }
};
Trace g_trace;

bool tracing() { return !g_trace.path.empty(); }

// The current device's reference event (created on first use).
hipEvent_t trace_ref(int* dev_out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    *dev_out = dev;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_trace.ref.find(dev);
    if (it != g_trace.ref.end()) return it->second;
    hipEvent_t e = nullptr;
    if (hipDeviceSynchronize() != hipSuccess || hipEventCreate(&e) != hipSuccess) return nullptr;
    if (hipEventRecord(e, nullptr) != hipSuccess || hipEventSynchronize(e) != hipSuccess) {
        (void)hipEventDestroy(e);
        return nullptr;
    }
    g_trace.ref.emplace(dev, e);
    return e;
}
}  // namespace

bool timing_on() { return g_on.load() != 0; }
int timing_every() { const int k = g_on.load(); return k > 0 ? k : 1; }

DispatchEvents& dispatch_events() {
    thread_local DispatchEvents slot;
    return slot;
}

void LaunchTimer::begin() {
    if (!timing_on()) return;
    if (count++ % timing_every() != 0) return;
    if (tracing() && !ref) ref = trace_ref(&dev);
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return;
    }
    pending = a;
    pending_stop = b;
    dispatch_events() = DispatchEvents{a, b, false};
}

void LaunchTimer::end() {
    if (!pending) return;
    DispatchEvents& de = dispatch_events();
    if (de.start == pending && de.taken) {
        ev.emplace_back(pending, pending_stop);
    } else {
        // the launch did not take the events (it failed before its dispatch):
        // it stays untimed
        (void)hipEventDestroy(pending);
        (void)hipEventDestroy(pending_stop);
    }
    de = DispatchEvents{};
    pending = pending_stop = nullptr;
}

void LaunchTimer::flush() {
    if (ev.empty()) return;
    double tot = 0.0;
    std::vector<TraceEv> tr;
    for (auto& pr : ev) {
        float ms = 0.f;
        if (hipEventSynchronize(pr.second) == hipSuccess &&
            hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) {
            tot += ms;
            float t0 = 0.f;
            if (ref && hipEventElapsedTime(&t0, (hipEvent_t)ref, pr.first) == hipSuccess)
                tr.push_back(TraceEv{family, dev, (uintptr_t)s, 1e3 * t0, 1e3 * ms});
        }
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    std::lock_guard<std::mutex> lk(g_mu);
    g_tot[family].ms += tot;
    g_tot[family].n += (int64_t)ev.size();
    if (tracing()) g_trace.ev.insert(g_trace.ev.end(), tr.begin(), tr.end());
    ev.clear();
}

LaunchTimer::~LaunchTimer() {
    for (auto& pr : ev) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    if (pending) {
        (void)hipEventDestroy(pending);
        (void)hipEventDestroy(pending_stop);
        if (dispatch_events().start == pending) dispatch_events() = DispatchEvents{};
    }
}

}  // namespace gc

extern "C" {

int gc_timing_enable(int on) {
    gc::g_on.store(on > 0 ? on : 0);
    return GC_OK;
}

int gc_timing_get(const char* family, double* total_ms, int64_t* launches) {
    if (!family) return GC_E_INVAL;
    std::lock_guard<std::mutex> lk(gc::g_mu);
    auto it = gc::g_tot.find(family);
    if (total_ms) *total_ms = it == gc::g_tot.end() ? 0.0 : it->second.ms;
    if (launches) *launches = it == gc::g_tot.end() ? 0 : it->second.n;
    return GC_OK;
}

int gc_timing_reset(void) {
    std::lock_guard<std::mutex> lk(gc::g_mu);
    gc::g_tot.clear();
    return GC_OK;
}

}  // extern "C"
