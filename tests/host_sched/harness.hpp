// Host-only stand-in for the GPU, used to test the library's host code (the
// continuous-batching scheduler, the staging and the arena) on the CPU.
//
// fake_hip.cpp implements the subset of the HIP runtime the host code calls:
// device memory is host memory, every stream is a worker thread that runs its
// queue in order (with random delays, so the host runs ahead of the "GPU" by
// varying amounts), events and stream waits keep their HIP meaning.
// stub_kernels.cpp replaces every kernel launcher: a launch is queued like a
// real one and, when it runs, checks every address range the real kernel
// would touch (from its own indexing) against the allocations live at that
// moment -- including that the memory was allocated before the launch was
// enqueued, which catches a block freed and handed to another job while work
// that uses it is still queued.  The stubs compute nothing of the method;
// they only do the index bookkeeping the host reads back (mask compaction
// counts, fills of flags).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <functional>

namespace hh {

// Queues fn on stream s; fn receives the sequence number the launch was
// enqueued with (every allocation and launch draws from one counter).
void enqueue(hipStream_t s, const char* name, std::function<void(uint64_t)> fn);

// True if [p, p + bytes) lies inside one live device allocation (an arena
// block if the address is in an arena chunk) that was allocated before the
// operation with sequence number seq was enqueued, and, when base != nullptr,
// inside the same allocation as base.  Records a violation otherwise.
bool dev_ok(const void* base, const void* p, size_t bytes, uint64_t seq, const char* kern,
            const char* what);

// Records a violation (printed at once, counted).
void violation(const char* fmt, ...);
size_t violations();

// Operation counters (launches, copies) for the replay's report.
void count_launch(const char* name);

}  // namespace hh
