// Kernel timing registry (see gacelle.h: gc_timing_*).
#include "gc_timing.hpp"

#include <atomic>
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
}  // namespace

bool timing_on() { return g_on.load() != 0; }
int timing_every() { const int k = g_on.load(); return k > 0 ? k : 1; }

void LaunchTimer::begin() {
    if (!timing_on()) return;
    if (count++ % timing_every() != 0) return;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    (void)hipEventRecord(e, s);
    pending = e;
}

void LaunchTimer::end() {
    if (!pending) return;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipEventDestroy(pending);
        pending = nullptr;
        return;
    }
    (void)hipEventRecord(e, s);
    ev.emplace_back(pending, e);
    pending = nullptr;
}

void LaunchTimer::flush() {
    if (ev.empty()) return;
    double tot = 0.0;
    for (auto& pr : ev) {
        float ms = 0.f;
        if (hipEventSynchronize(pr.second) == hipSuccess &&
            hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess)
            tot += ms;
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    std::lock_guard<std::mutex> lk(g_mu);
    g_tot[family].ms += tot;
    g_tot[family].n += (int64_t)ev.size();
    ev.clear();
}

LaunchTimer::~LaunchTimer() {
    for (auto& pr : ev) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    if (pending) (void)hipEventDestroy(pending);
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
