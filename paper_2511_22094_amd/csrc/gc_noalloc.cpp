// gc_mcmc_noalloc: gc_mcmc for callers that cannot allocate device memory
// (code under stream capture, tight serving loops, harnesses that forbid
// hipMalloc).  Every piece of device scratch -- compacted data, index maps,
// chain state, Welford moments, descriptors, work-lists, the model's
// acquisition tables -- is carved from one fixed device array per GPU.
#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <mutex>

#include "gc_runtime.hpp"

// Size of the scratch array: 128 MiB per GPU.
#ifndef GC_NOALLOC_SCRATCH_BYTES
#define GC_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
#endif
constexpr size_t kNoAllocScratchBytes = GC_NOALLOC_SCRATCH_BYTES;

// The scratch array of the allocation-free entry point.  Each GPU the
// library runs on holds one copy until the process ends.  In host code its
// name is only a stand-in for the symbol: the device address of a GPU's copy
// comes from hipGetSymbolAddress with that GPU current (scratch_on below).
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace gc {
namespace {

struct DevScratch {
    void* ptr = nullptr;
    std::mutex mu;   // the array is shared: one call at a time per GPU
};
std::mutex g_mu;
std::map<int, std::unique_ptr<DevScratch>> g_dev;

// The device address of `scratch` on `dev` (which must be current): looked
// up once per device and kept.
int scratch_on(int dev, DevScratch** out) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_dev.find(dev);
    if (it == g_dev.end()) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        GC_REQUIRE(e == hipSuccess && p != nullptr, GC_E_DEVICE,
                   "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        auto ds = std::make_unique<DevScratch>();
        ds->ptr = p;
        it = g_dev.emplace(dev, std::move(ds)).first;
    }
    *out = it->second.get();
    return GC_OK;
}

}  // namespace
}  // namespace gc

using namespace gc;

extern "C" {

size_t gc_noalloc_scratch_bytes(void) { return kNoAllocScratchBytes; }

int gc_mcmc_noalloc(const gc_model* model, const gc_volume* data, const uint8_t* mask,
                    const gc_bounds* bounds, int n_chains, int n_iter, int burnin, int thin,
                    const gc_mcmc_hyper* hyper, double* out_mean, double* out_std,
                    float* out_samples, int32_t* out_accept, const gc_exec* exec) {
    try {
        clear_error();
        int rc;
        if ((rc = mcmc_validate(model, data, bounds, &n_chains, n_iter, burnin, thin, hyper,
                                out_mean, out_std, out_samples)))
            return rc;
        GC_REQUIRE(exec && exec->mem_kind == GC_MEM_DEVICE, GC_E_INVAL,
                   "gc_mcmc_noalloc takes device-memory arguments only (exec->mem_kind = "
                   "GC_MEM_DEVICE)");
        GC_REQUIRE(!hyper->sample_sink, GC_E_INVAL,
                   "gc_mcmc_noalloc has no sample sink (it would need host staging)");
        DeviceScope ds;
        if ((rc = ds.open(exec))) return rc;
        DevScratch* dsc = nullptr;
        if ((rc = scratch_on(ds.dev, &dsc))) return rc;
        std::lock_guard<std::mutex> lk(dsc->mu);
        Scratch sc(ds.stream);
        sc.fixed = (char*)dsc->ptr;
        sc.cap = kNoAllocScratchBytes;
        rc = mcmc_impl(model, data, mask, bounds, n_chains, n_iter, burnin, thin, hyper, out_mean,
                       out_std, out_samples, out_accept, ds, sc, true);
        if (sc.short_by > 0) {
            // nothing that depends on the missing memory was launched; let the
            // work already queued finish before the next call reuses the array
            (void)hipStreamSynchronize(ds.stream);
            set_error("gc_mcmc_noalloc: the problem needs more than the %zu bytes of scratch "
                      "this entry point holds per GPU (short by at least %zu bytes); use gc_mcmc",
                      kNoAllocScratchBytes, sc.short_by);
            return GC_E_NOMEM;
        }
        if (rc != GC_OK) (void)hipStreamSynchronize(ds.stream);
        return rc;
    } catch (...) {
        set_error("internal error");
        return GC_E_DEVICE;
    }
}

}  // extern "C"
