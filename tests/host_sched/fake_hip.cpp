// Host-only stand-in for the HIP runtime subset used by the library's host
// code (see harness.hpp).  Device memory is reserved host memory; a stream
// is a worker thread running its queue in order after a random delay per
// operation; events complete when the worker reaches their record.
#include <sys/mman.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <random>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "harness.hpp"

struct ihipStream_t {
    std::mutex mu;
    std::condition_variable cv;
    struct Item {
        uint64_t seq;
        const char* name;
        std::function<void(uint64_t)> fn;
    };
    std::deque<Item> q;
    bool stop = false;
    int running = 0;
    std::thread th;
    unsigned seed = 0;
};

struct ihipEvent_t {
    std::mutex mu;
    std::condition_variable cv;
    uint64_t recorded = 0, done = 0;
    double t_done = 0.0;
};

namespace hh {
namespace {

std::atomic<uint64_t> g_seq{1};

enum { K_DEV = 0, K_ASYNC = 1, K_CHUNK = 2 };
struct Blk {
    char* base;
    size_t size;
    uint64_t seq;
    int kind;
};
std::mutex g_mem_mu;
std::map<char*, Blk> g_dev;   // hipMalloc / hipMallocAsync regions (arena chunks marked)
std::map<char*, Blk> g_sub;   // arena blocks
std::map<char*, Blk> g_pin;   // pinned host memory

std::mutex g_vmu;
size_t g_nviol = 0;
std::map<std::string, uint64_t> g_launch;

std::mutex g_reg_mu;
std::map<ihipEvent_t*, std::shared_ptr<ihipEvent_t>> g_events;
std::set<ihipStream_t*> g_streams;
ihipStream_t* g_null = nullptr;

size_t env_size(const char* k, size_t dflt) {
    const char* v = std::getenv(k);
    return v ? (size_t)std::strtoull(v, nullptr, 10) : dflt;
}
// copies up to this size move their bytes (every descriptor upload of a round
// among them: the kernel stubs read the descriptors); larger ones, bulk data
// the stubs never read, are checked by range only
const size_t kCopyCap = env_size("HH_COPY_CAP", (size_t)64 << 20);
const unsigned kDelayUs = (unsigned)env_size("HH_DELAY_US", 100);

double now() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

const Blk* find_in(std::map<char*, Blk>& m, const void* p) {
    auto it = m.upper_bound((char*)p);
    if (it == m.begin()) return nullptr;
    --it;
    return (char*)p < it->second.base + it->second.size ? &it->second : nullptr;
}

// the live block holding address p (arena block inside a chunk, or a region)
const Blk* dev_block(const void* p, bool* in_chunk) {
    *in_chunk = false;
    if (const Blk* b = find_in(g_sub, p)) return b;
    const Blk* r = find_in(g_dev, p);
    if (r && r->kind == K_CHUNK) {
        *in_chunk = true;
        return nullptr;
    }
    return r;
}

bool pinned_ok(const void* p, size_t bytes) {
    std::lock_guard<std::mutex> lk(g_mem_mu);
    const Blk* b = find_in(g_pin, p);
    return b && (char*)p + bytes <= b->base + b->size;
}

bool is_pinned(const void* p) {
    std::lock_guard<std::mutex> lk(g_mem_mu);
    return find_in(g_pin, p) != nullptr;
}

bool is_device(const void* p) {
    std::lock_guard<std::mutex> lk(g_mem_mu);
    return find_in(g_dev, p) != nullptr;
}

void worker(ihipStream_t* s) {
    std::mt19937 rng(s->seed);
    for (;;) {
        ihipStream_t::Item it;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv.wait(lk, [&] { return s->stop || !s->q.empty(); });
            if (s->q.empty()) return;
            it = std::move(s->q.front());
            s->q.pop_front();
            s->running = 1;
        }
        if (kDelayUs) std::this_thread::sleep_for(std::chrono::microseconds(rng() % (kDelayUs + 1)));
        it.fn(it.seq);
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->running = 0;
        }
        s->cv.notify_all();
    }
}

ihipStream_t* new_stream() {
    auto* s = new ihipStream_t();
    static std::atomic<unsigned> n{0};
    s->seed = 1234567u + 7919u * n.fetch_add(1);
    s->th = std::thread(worker, s);
    std::lock_guard<std::mutex> lk(g_reg_mu);
    g_streams.insert(s);
    return s;
}

ihipStream_t* stream_of(hipStream_t s) {
    if (s) return s;
    std::lock_guard<std::mutex> lk(g_reg_mu);
    if (!g_null) {
        g_null = new ihipStream_t();
        g_null->seed = 99u;
        g_null->th = std::thread(worker, g_null);
        g_streams.insert(g_null);
    }
    return g_null;
}

void drain(ihipStream_t* s) {
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv.wait(lk, [&] { return s->q.empty() && s->running == 0; });
}

void drain_all() {
    std::vector<ihipStream_t*> all;
    {
        std::lock_guard<std::mutex> lk(g_reg_mu);
        all.assign(g_streams.begin(), g_streams.end());
    }
    for (auto* s : all) drain(s);
}

std::shared_ptr<ihipEvent_t> event_of(hipEvent_t e, const char* what) {
    std::lock_guard<std::mutex> lk(g_reg_mu);
    auto it = g_events.find(e);
    if (it == g_events.end()) {
        violation("%s: event %p is not a live event", what, (void*)e);
        return nullptr;
    }
    return it->second;
}

void* reserve(size_t bytes) {
    const size_t pg = 4096;
    size_t sz = (bytes + pg - 1) / pg * pg;
    void* p = mmap(nullptr, sz, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE,
                   -1, 0);
    return p == MAP_FAILED ? nullptr : p;
}

void unreserve(void* p, size_t bytes) {
    const size_t pg = 4096;
    munmap(p, (bytes + pg - 1) / pg * pg);
}

}  // namespace

void enqueue(hipStream_t st, const char* name, std::function<void(uint64_t)> fn) {
    ihipStream_t* s = stream_of(st);
    const uint64_t seq = g_seq.fetch_add(1);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->q.push_back(ihipStream_t::Item{seq, name, std::move(fn)});
    }
    s->cv.notify_all();
}

void violation(const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    std::lock_guard<std::mutex> lk(g_vmu);
    ++g_nviol;
    if (g_nviol <= 50) std::fprintf(stderr, "VIOLATION: %s\n", buf);
}

size_t violations() {
    std::lock_guard<std::mutex> lk(g_vmu);
    return g_nviol;
}

void count_launch(const char* name) {
    std::lock_guard<std::mutex> lk(g_vmu);
    g_launch[name]++;
}

bool dev_ok(const void* base, const void* p, size_t bytes, uint64_t seq, const char* kern,
            const char* what) {
    if (bytes == 0) return true;
    if (!p) {
        violation("%s: %s is null (%zu bytes accessed)", kern, what, bytes);
        return false;
    }
    std::lock_guard<std::mutex> lk(g_mem_mu);
    bool in_chunk = false;
    const Blk* b = dev_block(p, &in_chunk);
    if (!b) {
        violation("%s: %s at %p (%zu bytes) is %s", kern, what, p, bytes,
                  in_chunk ? "freed arena memory" : "not in any live device allocation");
        return false;
    }
    if ((char*)p + bytes > b->base + b->size) {
        violation("%s: %s [%p, +%zu) overruns its allocation [%p, +%zu) by %zu bytes", kern, what,
                  p, bytes, (void*)b->base, b->size,
                  (size_t)((char*)p + bytes - (b->base + b->size)));
        return false;
    }
    if (b->seq >= seq) {
        violation("%s: %s at %p lies in an allocation made after the launch was enqueued "
                  "(its memory was freed and handed out again while the launch was queued)",
                  kern, what, p);
        return false;
    }
    if (base && base != p) {
        bool c2 = false;
        const Blk* bb = dev_block(base, &c2);
        if (bb != b) {
            violation("%s: %s at %p is not in the allocation of its base %p", kern, what, p, base);
            return false;
        }
    }
    return true;
}

}  // namespace hh

// ------------------------------------------------------------------ arena hook
extern "C" void gc_harness_arena_event(int op, void* p, size_t bytes) {
    using namespace hh;
    std::lock_guard<std::mutex> lk(g_mem_mu);
    if (op == 0) {   // chunk: its memory is used only through blocks
        auto it = g_dev.find((char*)p);
        if (it == g_dev.end()) violation("arena chunk %p is not a device allocation", p);
        else it->second.kind = K_CHUNK;
    } else if (op == 1) {
        if (find_in(g_sub, p)) violation("arena block %p handed out twice", p);
        g_sub[(char*)p] = Blk{(char*)p, bytes, g_seq.fetch_add(1), K_DEV};
    } else {
        auto it = g_sub.find((char*)p);
        if (it == g_sub.end()) {
            violation("arena free of %p, which is not a live block", p);
            return;
        }
        if (it->second.size <= ((size_t)1 << 20)) std::memset(p, 0xDB, it->second.size);
        g_sub.erase(it);
    }
}

// ------------------------------------------------------------------ HIP API
using namespace hh;

extern "C" {

const char* hipGetErrorString(hipError_t e) {
    switch (e) {
        case hipSuccess: return "hipSuccess";
        case hipErrorNotReady: return "hipErrorNotReady";
        case hipErrorOutOfMemory: return "hipErrorOutOfMemory";
        case hipErrorInvalidValue: return "hipErrorInvalidValue";
        default: return "hipError(fake)";
    }
}

hipError_t hipGetLastError(void) { return hipSuccess; }
hipError_t hipGetDevice(int* d) {
    *d = 0;
    return hipSuccess;
}
hipError_t hipSetDevice(int d) { return d == 0 ? hipSuccess : hipErrorInvalidDevice; }
hipError_t hipGetDeviceCount(int* n) {
    *n = 1;
    return hipSuccess;
}
hipError_t hipMemGetInfo(size_t* fr, size_t* tot) {
    *fr = env_size("HH_FREE_BYTES", (size_t)64 << 30);
    *tot = 2 * *fr;
    return hipSuccess;
}
hipError_t hipDeviceGetDefaultMemPool(hipMemPool_t* pool, int) {
    *pool = (hipMemPool_t)0x1;
    return hipSuccess;
}
hipError_t hipMemPoolSetAttribute(hipMemPool_t, hipMemPoolAttr, void*) { return hipSuccess; }

hipError_t hipMalloc(void** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) return hipSuccess;
    void* m = reserve(bytes);
    if (!m) return hipErrorOutOfMemory;
    std::lock_guard<std::mutex> lk(g_mem_mu);
    g_dev[(char*)m] = Blk{(char*)m, bytes, g_seq.fetch_add(1), K_DEV};
    *p = m;
    return hipSuccess;
}

hipError_t hipFree(void* p) {
    if (!p) return hipSuccess;
    drain_all();   // hipFree waits for the device
    std::lock_guard<std::mutex> lk(g_mem_mu);
    auto it = g_dev.find((char*)p);
    if (it == g_dev.end()) {
        violation("hipFree(%p): not a live allocation", p);
        return hipErrorInvalidValue;
    }
    unreserve(p, it->second.size);
    g_dev.erase(it);
    return hipSuccess;
}

hipError_t hipMallocAsync(void** p, size_t bytes, hipStream_t) {
    *p = nullptr;
    if (bytes == 0) return hipSuccess;
    void* m = reserve(bytes);
    if (!m) return hipErrorOutOfMemory;
    std::lock_guard<std::mutex> lk(g_mem_mu);
    g_dev[(char*)m] = Blk{(char*)m, bytes, g_seq.fetch_add(1), K_ASYNC};
    *p = m;
    return hipSuccess;
}

hipError_t hipFreeAsync(void* p, hipStream_t s) {
    if (!p) return hipSuccess;
    enqueue(s, "hipFreeAsync", [p](uint64_t) {
        std::lock_guard<std::mutex> lk(g_mem_mu);
        auto it = g_dev.find((char*)p);
        if (it == g_dev.end()) {
            violation("hipFreeAsync(%p): not a live allocation", p);
            return;
        }
        unreserve(p, it->second.size);
        g_dev.erase(it);
    });
    return hipSuccess;
}

hipError_t hipHostMalloc(void** p, size_t bytes, unsigned int) {
    *p = std::malloc(bytes ? bytes : 1);
    if (!*p) return hipErrorOutOfMemory;
    std::lock_guard<std::mutex> lk(g_mem_mu);
    g_pin[(char*)*p] = Blk{(char*)*p, bytes ? bytes : 1, g_seq.fetch_add(1), K_DEV};
    return hipSuccess;
}

hipError_t hipHostFree(void* p) {
    if (!p) return hipSuccess;
    {
        std::lock_guard<std::mutex> lk(g_mem_mu);
        auto it = g_pin.find((char*)p);
        if (it == g_pin.end()) {
            violation("hipHostFree(%p): not pinned memory", p);
            return hipErrorInvalidValue;
        }
        g_pin.erase(it);
    }
    std::free(p);
    return hipSuccess;
}

hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind,
                          hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    const bool dd = is_device(dst), sd = is_device(src);
    const bool dp = !dd && is_pinned(dst), sp = !sd && is_pinned(src);
    const bool data = bytes <= kCopyCap;
    if ((kind == hipMemcpyHostToDevice && (!dd || sd)) ||
        (kind == hipMemcpyDeviceToHost && (dd || !sd)) ||
        (kind == hipMemcpyDeviceToDevice && (!dd || !sd))) {
        violation("hipMemcpyAsync kind %d does not match its pointers (dst %s, src %s)", (int)kind,
                  dd ? "device" : "host", sd ? "device" : "host");
        return hipErrorInvalidValue;
    }
    std::shared_ptr<std::vector<char>> snap;
    if (!sd && !sp && data) {   // pageable source: staged when the call is made
        snap = std::make_shared<std::vector<char>>((const char*)src, (const char*)src + bytes);
    }
    enqueue(s, "memcpy", [=](uint64_t seq) {
        if (dd && !dev_ok(nullptr, dst, bytes, seq, "memcpy", "destination")) return;
        if (sd && !dev_ok(nullptr, src, bytes, seq, "memcpy", "source")) return;
        if (dp && !pinned_ok(dst, bytes)) {
            violation("memcpy: pinned destination %p (%zu bytes) was freed or is too small", dst, bytes);
            return;
        }
        if (sp && !pinned_ok(src, bytes)) {
            violation("memcpy: pinned source %p (%zu bytes) was freed or is too small", src, bytes);
            return;
        }
        if (!data) return;
        std::memcpy(dst, snap ? snap->data() : (const char*)src, bytes);
    });
    return hipSuccess;
}

hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind kind) {
    hipError_t e = hipMemcpyAsync(dst, src, bytes, kind, nullptr);
    if (e != hipSuccess) return e;
    drain(stream_of(nullptr));
    return hipSuccess;
}

hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int) {
    *s = new_stream();
    return hipSuccess;
}

hipError_t hipStreamDestroy(hipStream_t s) {
    if (!s) return hipSuccess;
    drain(s);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    s->th.join();
    {
        std::lock_guard<std::mutex> lk(g_reg_mu);
        g_streams.erase(s);
    }
    delete s;
    return hipSuccess;
}

hipError_t hipStreamSynchronize(hipStream_t s) {
    drain(stream_of(s));
    return hipSuccess;
}

hipError_t hipDeviceSynchronize(void) {
    drain_all();
    return hipSuccess;
}

hipError_t hipEventCreate(hipEvent_t* e) {
    auto ev = std::make_shared<ihipEvent_t>();
    std::lock_guard<std::mutex> lk(g_reg_mu);
    g_events[ev.get()] = ev;
    *e = ev.get();
    return hipSuccess;
}

hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }

hipError_t hipEventDestroy(hipEvent_t e) {
    std::lock_guard<std::mutex> lk(g_reg_mu);
    if (!g_events.erase(e)) {
        violation("hipEventDestroy(%p): not a live event", (void*)e);
        return hipErrorInvalidValue;
    }
    return hipSuccess;
}

hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
    auto ev = event_of(e, "hipEventRecord");
    if (!ev) return hipErrorInvalidValue;
    uint64_t g;
    {
        std::lock_guard<std::mutex> lk(ev->mu);
        g = ++ev->recorded;
    }
    enqueue(s, "event", [ev, g](uint64_t) {
        {
            std::lock_guard<std::mutex> lk(ev->mu);
            if (ev->done < g) ev->done = g;
            ev->t_done = now();
        }
        ev->cv.notify_all();
    });
    return hipSuccess;
}

hipError_t hipEventQuery(hipEvent_t e) {
    auto ev = event_of(e, "hipEventQuery");
    if (!ev) return hipErrorInvalidValue;
    std::lock_guard<std::mutex> lk(ev->mu);
    return ev->done >= ev->recorded ? hipSuccess : hipErrorNotReady;
}

hipError_t hipEventSynchronize(hipEvent_t e) {
    auto ev = event_of(e, "hipEventSynchronize");
    if (!ev) return hipErrorInvalidValue;
    std::unique_lock<std::mutex> lk(ev->mu);
    const uint64_t r = ev->recorded;
    ev->cv.wait(lk, [&] { return ev->done >= r; });
    return hipSuccess;
}

hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
    auto ea = event_of(a, "hipEventElapsedTime"), eb = event_of(b, "hipEventElapsedTime");
    if (!ea || !eb) return hipErrorInvalidValue;
    *ms = (float)((eb->t_done - ea->t_done) * 1e3);
    return hipSuccess;
}

hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned int) {
    auto ev = event_of(e, "hipStreamWaitEvent");
    if (!ev) return hipErrorInvalidValue;
    uint64_t r;
    {
        std::lock_guard<std::mutex> lk(ev->mu);
        r = ev->recorded;
    }
    enqueue(s, "wait", [ev, r](uint64_t) {
        std::unique_lock<std::mutex> lk(ev->mu);
        ev->cv.wait(lk, [&] { return ev->done >= r; });
    });
    return hipSuccess;
}

}  // extern "C"
