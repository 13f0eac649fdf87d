// Per-family kernel timing with HIP events (enabled by gc_timing_enable).
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

namespace gc {

bool timing_on();
int timing_every();   // time every k-th launch (k >= 1) while on

// The events of a launch being timed.  LaunchTimer::begin() puts a pair in
// this thread's slot and end() empties it; a launcher that launches through
// GC_LAUNCH attaches the pair to its dispatch (hipExtLaunchKernelGGL), so
// that their elapsed time is the kernel's own execution, as a kernel trace
// reports it, without the event packets a stream would run around it.
struct DispatchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
    bool taken = false;
};
DispatchEvents& dispatch_events();

#define GC_LAUNCH(kernel, grid, block, shmem, stream, ...)                                   \
    do {                                                                                      \
        ::gc::DispatchEvents& gc_de_ = ::gc::dispatch_events();                               \
        if (gc_de_.start && !gc_de_.taken) {                                                  \
            gc_de_.taken = true;                                                              \
            hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, gc_de_.start,           \
                                  gc_de_.stop, 0, __VA_ARGS__);                               \
        } else {                                                                              \
            hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);              \
        }                                                                                     \
    } while (0)
// Brackets launches: begin() before, end() after; flush() after the stream
// has been synchronised adds the elapsed times to the family's total.
struct LaunchTimer {
    std::string family;
    hipStream_t s;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    hipEvent_t pending = nullptr, pending_stop = nullptr;
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
