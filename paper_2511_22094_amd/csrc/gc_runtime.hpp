// Host runtime shared by the synchronous C ABI and the server: the model
// object, error reporting, device / stream selection, stream-ordered
// scratch memory, and the staging + compaction of one problem.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/gacelle.h"
#include "gc_internal.hpp"

struct gc_model {
    int kind = 0;
    int P = 0;
    int M = 0;
    int Meff = 0;
    bool complex_ = false;
    std::string name;
    std::vector<std::string> pnames;
    std::vector<double> te, bval, bvec;   // host copies (bval in s/mm^2)
    bool uniform = false;
    double te0 = 0.0, dte = 0.0;
    struct DevAcq {
        void* buf = nullptr;              // one allocation holding all arrays
        gc::AcqDev acq{};
    };
    mutable std::mutex mu;
    mutable std::map<int, DevAcq> dev;    // per device ordinal
    // references: the creator's (dropped by gc_model_destroy) plus one per
    // server job that has not finished; the last one frees the model
    mutable std::atomic<int> refs{1};
};

namespace gc {

void set_error(const char* fmt, ...);
void clear_error();

#define GC_TRY_HIP(expr)                                                           \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess) {                                                    \
            ::gc::set_error("%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                            __LINE__);                                             \
            return GC_E_DEVICE;                                                    \
        }                                                                          \
    } while (0)

#define GC_REQUIRE(cond, code, ...)      \
    do {                                 \
        if (!(cond)) {                   \
            ::gc::set_error(__VA_ARGS__); \
            return (code);               \
        }                                \
    } while (0)

// Selects the device for the duration of a call and restores the previous one.
struct DeviceScope {
    int prev = -1;
    int dev = 0;
    hipStream_t stream = nullptr;
    int mem_kind = GC_MEM_HOST;
    int open(const gc_exec* ex);
    ~DeviceScope();
};

// Device memory owned by the host: chunks from hipMalloc, sub-allocated
// first-fit.  A block is returned only when the host knows the GPU has
// finished with it (after observing an event), so no stream-ordering
// assumption is involved; the server draws all its memory from one arena.
struct DevArena {
    std::mutex mu;
    struct Chunk {
        char* base = nullptr;
        size_t size = 0;
        std::map<size_t, size_t> free_;   // offset -> length
    };
    std::vector<Chunk> chunks;
    std::map<char*, std::pair<size_t, size_t>> used;   // ptr -> (chunk, length)
    size_t chunk_bytes = (size_t)256 << 20;
    size_t in_use = 0;
    hipError_t alloc(void** p, size_t bytes);
    void free(void* p);
    // true if [p, p + bytes) lies inside one block handed out and not freed
    bool owns(const void* p, size_t bytes);
    ~DevArena();
};

// Scratch allocations released at scope exit: stream-ordered on `s`
// (synchronous entry points, one stream), from an arena (server), or carved
// in order from a fixed region the caller owns (allocation-free entry
// points: nothing is allocated or released; a request past the region's end
// fails with hipErrorOutOfMemory and is remembered in `short_by`).
struct Scratch {
    hipStream_t s = nullptr;
    DevArena* arena = nullptr;
    std::vector<void*> ptrs;
    char* fixed = nullptr;
    size_t cap = 0, used = 0, short_by = 0;
    explicit Scratch(hipStream_t st, DevArena* a = nullptr) : s(st), arena(a) {}
    ~Scratch();
    hipError_t alloc(void** p, size_t bytes);
    template <typename T> hipError_t alloc_n(T** p, size_t n) {
        return alloc((void**)p, n * sizeof(T));
    }
};

// Model references (server jobs keep their model alive until they finish).
void model_retain(const gc_model* m);
void model_release(const gc_model* m);

// Device-side acquisition of a model on the current device.
int model_acq(const gc_model* m, int device, AcqDev* out);

// A bulk argument in exec memory: returns a device pointer, staging host data.
int stage_in(Scratch& sc, const void* p, size_t bytes, int mem_kind, const void** dptr);

// Compaction of one volume (mask -> index maps, gathered rows).
struct Packed {
    int64_t G = 0, n = 0;
    int32_t* g2c = nullptr;
    int32_t* c2g = nullptr;
    float* y = nullptr;      // [Meff][n]
    float* w = nullptr;      // [n] or null
    float* x0 = nullptr;     // [P][n] or null
};
int pack_problem(Scratch& sc, const gc_model* m, const gc_volume* data, const uint8_t* mask,
                 const float* weights, const float* x0map, int mem_kind, Packed* out);

// Prior maps (Eq. 6) of a fit, gathered to [P][n] over the mask; sigma must be
// finite and > 0, mu finite (GC_E_INVAL / GC_E_NONFINITE otherwise).  Both
// stay nullptr when the prior is off.
int pack_prior(Scratch& sc, const gc_model* m, const gc_adam_hyper* h, const Packed& pk,
               int mem_kind, float** mu, float** sigma);
// Graph adjacency of a fit with graph TV, in device memory and checked
// (GC_E_INVAL unless it is a valid CSR over the n masked voxels): sets the
// descriptor's g_rowptr, g_col and g_nnz (null and 0 without graph TV).
int pack_graph(Scratch& sc, const gc_adam_hyper* h, int64_t n, int mem_kind, FitJob* J);
int validate_graph(Scratch& sc, int64_t n, int64_t nnz, const int64_t* rowptr,
                   const int32_t* col, hipStream_t s);

int validate_bounds(const gc_model* m, const gc_bounds* b);
int validate_adam(const gc_model* m, const gc_adam_hyper* h);
int validate_volume(const gc_model* m, const gc_volume* v);

// descriptor builders shared by the synchronous calls and the server
int fill_mh_job(const gc_model* m, const gc_bounds* b, const gc_mcmc_hyper* h, int n_chains,
                int n_iter, int burnin, int thin, const AcqDev& acq, MhJob* job);
int fill_fit_job(const gc_model* m, const gc_bounds* b, const gc_adam_hyper* h, int64_t n,
                 const AcqDev& acq, FitJob* job);

void mempool_setup(int device);
double now_seconds();

// MCMC (gc_mcmc and its allocation-free variant): argument checks, then the
// whole call with every device allocation drawn from `sc`.
int mcmc_validate(const gc_model* model, const gc_volume* data, const gc_bounds* bounds,
                  int* n_chains, int n_iter, int burnin, int thin, const gc_mcmc_hyper* hyper,
                  const double* out_mean, const double* out_std, const float* out_samples);
int mcmc_impl(const gc_model* model, const gc_volume* data, const uint8_t* mask,
              const gc_bounds* bounds, int n_chains, int n_iter, int burnin, int thin,
              const gc_mcmc_hyper* hyper, double* out_mean, double* out_std, float* out_samples,
              int32_t* out_accept, DeviceScope& ds, Scratch& sc, bool noalloc);

}  // namespace gc
