// Per-family kernel timing with HIP events (enabled by gc_timing_enable).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

namespace gc {

bool timing_on();
int timing_every();   // time every k-th launch (k >= 1) while on
// Brackets launches: begin() before, end() after; flush() after the stream
// has been synchronised adds the elapsed times to the family's total.
struct LaunchTimer {
    std::string family;
    hipStream_t s;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    hipEvent_t pending = nullptr;
    int64_t count = 0;       // launches seen (timed or not)
    void* ref = nullptr;     // the device's trace reference event (GACELLE_TRACE)
    int dev = 0;
    LaunchTimer(const char* fam, hipStream_t st) : family(fam), s(st) {}
    void begin();
    void end();
    void flush();
    ~LaunchTimer();
};

}  // namespace gc
