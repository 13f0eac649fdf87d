// Synchronous C ABI: model registry, validation, staging, and the drivers of
// the fit and MCMC kernels.  Every entry point catches every C++ exception.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <new>

#include "gc_runtime.hpp"
#include "gc_sense.hpp"
#include "gc_timing.hpp"

namespace gc {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}
void clear_error() { g_err.clear(); }

double now_seconds() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

void mempool_setup(int device) {
    static std::mutex mu;
    static std::map<int, bool> done;
    std::lock_guard<std::mutex> lk(mu);
    if (done[device]) return;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
        uint64_t thr = UINT64_MAX;   // keep freed blocks for reuse by later calls
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
    done[device] = true;
}

int DeviceScope::open(const gc_exec* ex) {
    GC_TRY_HIP(hipGetDevice(&prev));
    dev = (ex && ex->device >= 0) ? ex->device : prev;
    int count = 0;
    GC_TRY_HIP(hipGetDeviceCount(&count));
    GC_REQUIRE(dev >= 0 && dev < count, GC_E_INVAL, "device %d out of range (%d devices)", dev,
               count);
    if (dev != prev) GC_TRY_HIP(hipSetDevice(dev));
    stream = ex ? (hipStream_t)ex->stream : nullptr;
    mem_kind = ex ? ex->mem_kind : GC_MEM_HOST;
    GC_REQUIRE(mem_kind == GC_MEM_HOST || mem_kind == GC_MEM_DEVICE, GC_E_INVAL,
               "exec->mem_kind must be GC_MEM_HOST or GC_MEM_DEVICE");
    mempool_setup(dev);
    return GC_OK;
}

DeviceScope::~DeviceScope() {
    if (prev >= 0 && prev != dev) (void)hipSetDevice(prev);
}

Scratch::~Scratch() {
    for (void* p : ptrs) {
        if (arena) arena->free(p);
        else (void)hipFreeAsync(p, s);
    }
}

hipError_t Scratch::alloc(void** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) bytes = 256;
    if (fixed) {
        const size_t b = (bytes + 255) / 256 * 256;
        if (used + b > cap) {
            short_by += used + b - cap;
            return hipErrorOutOfMemory;
        }
        *p = fixed + used;
        used += b;
        return hipSuccess;
    }
    hipError_t e = arena ? arena->alloc(p, bytes) : hipMallocAsync(p, bytes, s);
    if (e == hipSuccess) ptrs.push_back(*p);
    return e;
}

// The host-only test build of the scheduler (a stand-in runtime on the CPU)
// observes the arena's chunks and blocks to check every access of the
// stand-in kernels against the blocks live at that moment.
#ifdef GC_HOST_HARNESS
extern "C" void gc_harness_arena_event(int op, void* p, size_t bytes);
#define GC_ARENA_EVENT(op, p, b) gc_harness_arena_event(op, p, b)
#else
#define GC_ARENA_EVENT(op, p, b) ((void)0)
#endif

hipError_t DevArena::alloc(void** p, size_t bytes) {
    std::lock_guard<std::mutex> lk(mu);
    bytes = (bytes + 255) / 256 * 256;
    for (size_t ci = 0;; ++ci) {
        if (ci == chunks.size()) {
            Chunk c;
            c.size = std::max(bytes, chunk_bytes);
            hipError_t e = hipMalloc((void**)&c.base, c.size);
            if (e != hipSuccess) return e;
            GC_ARENA_EVENT(0, c.base, c.size);
            c.free_[0] = c.size;
            chunks.push_back(std::move(c));
        }
        Chunk& c = chunks[ci];
        for (auto it = c.free_.begin(); it != c.free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, len = it->second;
            c.free_.erase(it);
            if (len > bytes) c.free_[off + bytes] = len - bytes;
            *p = c.base + off;
            used[c.base + off] = {ci, bytes};
            in_use += bytes;
            GC_ARENA_EVENT(1, *p, bytes);
            return hipSuccess;
        }
    }
}

void DevArena::free(void* p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(mu);
    auto it = used.find((char*)p);
    if (it == used.end()) return;
    Chunk& c = chunks[it->second.first];
    size_t off = (size_t)((char*)p - c.base), len = it->second.second;
    GC_ARENA_EVENT(2, p, len);
    used.erase(it);
    in_use -= len;
    // coalesce with the free neighbours inside the chunk
    auto nx = c.free_.lower_bound(off);
    if (nx != c.free_.end() && nx->first == off + len) {
        len += nx->second;
        nx = c.free_.erase(nx);
    }
    if (nx != c.free_.begin()) {
        auto pv = std::prev(nx);
        if (pv->first + pv->second == off) {
            pv->second += len;
            return;
        }
    }
    c.free_[off] = len;
}

bool DevArena::owns(const void* p, size_t bytes) {
    std::lock_guard<std::mutex> lk(mu);
    auto it = used.upper_bound((char*)p);
    if (it == used.begin()) return false;
    --it;
    return (const char*)p + bytes <= it->first + it->second.second;
}

DevArena::~DevArena() {
    for (auto& c : chunks) (void)hipFree(c.base);
}

void model_retain(const gc_model* m) {
    if (m) m->refs.fetch_add(1);
}

void model_release(const gc_model* m) {
    if (!m || m->refs.fetch_sub(1) != 1) return;
    for (auto& kv : m->dev) {
        int prev = 0;
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(kv.first);
        (void)hipFree(kv.second.buf);
        (void)hipSetDevice(prev);
    }
    delete m;
}

int stage_in(Scratch& sc, const void* p, size_t bytes, int mem_kind, const void** dptr) {
    if (p == nullptr || mem_kind == GC_MEM_DEVICE) {
        *dptr = p;
        return GC_OK;
    }
    void* d = nullptr;
    hipError_t e = sc.alloc(&d, bytes);
    GC_REQUIRE(e == hipSuccess, GC_E_NOMEM, "device allocation of %zu bytes failed", bytes);
    GC_TRY_HIP(hipMemcpyAsync(d, p, bytes, hipMemcpyHostToDevice, sc.s));
    *dptr = d;
    return GC_OK;
}

int model_acq(const gc_model* m, int device, AcqDev* out) {
    std::lock_guard<std::mutex> lk(m->mu);
    auto it = m->dev.find(device);
    if (it != m->dev.end()) {
        *out = it->second.acq;
        return GC_OK;
    }
    const int M = m->M;
    // layout: te f32[M] | b f32[M] | g f32[3M] | te f64[M] | b f64[M] | g f64[3M]
    std::vector<float> f(5 * M, 0.f);
    std::vector<double> d(5 * M, 0.0);
    for (int j = 0; j < M; ++j) {
        if (!m->te.empty()) {
            f[j] = (float)m->te[j];
            d[j] = m->te[j];
        }
        if (!m->bval.empty()) {
            f[M + j] = (float)(m->bval[j] * 1e-3);
            d[M + j] = m->bval[j] * 1e-3;
            for (int k = 0; k < 3; ++k) {
                f[2 * M + 3 * j + k] = (float)m->bvec[3 * j + k];
                d[2 * M + 3 * j + k] = m->bvec[3 * j + k];
            }
        }
    }
    // runs of consecutive equal b values (shells in acquisition order)
    std::vector<int32_t> run_end;
    for (int j = 1; j < M; ++j)
        if (!m->bval.empty() && m->bval[j] != m->bval[j - 1]) run_end.push_back(j);
    run_end.push_back(M);
    const size_t fb = f.size() * sizeof(float), db = d.size() * sizeof(double);
    const size_t rb = run_end.size() * sizeof(int32_t);
    const size_t off = (fb + 255) / 256 * 256;
    const size_t off2 = off + (db + 255) / 256 * 256;
    void* buf = nullptr;
    GC_TRY_HIP(hipMalloc(&buf, off2 + rb));
    GC_TRY_HIP(hipMemcpy(buf, f.data(), fb, hipMemcpyHostToDevice));
    GC_TRY_HIP(hipMemcpy((char*)buf + off, d.data(), db, hipMemcpyHostToDevice));
    GC_TRY_HIP(hipMemcpy((char*)buf + off2, run_end.data(), rb, hipMemcpyHostToDevice));
    AcqDev a{};
    float* fp = (float*)buf;
    double* dp = (double*)((char*)buf + off);
    a.te = fp;
    a.bval = fp + M;
    a.bvec = fp + 2 * M;
    a.te_d = dp;
    a.bval_d = dp + M;
    a.bvec_d = dp + 2 * M;
    a.M = M;
    a.uniform = m->uniform ? 1 : 0;
    a.te0 = (float)m->te0;
    a.dte = (float)m->dte;
    a.te0_d = m->te0;
    a.dte_d = m->dte;
    a.run_end = (const int32_t*)((char*)buf + off2);
    a.nrun = (int)run_end.size();
    m->dev[device] = gc_model::DevAcq{buf, a};
    *out = a;
    return GC_OK;
}

int validate_volume(const gc_model* m, const gc_volume* v) {
    GC_REQUIRE(v != nullptr && v->y != nullptr, GC_E_INVAL, "data volume missing");
    GC_REQUIRE(v->nx >= 1 && v->ny >= 1 && v->nz >= 1, GC_E_INVAL, "grid dims must be >= 1");
    const int64_t G = (int64_t)v->nx * v->ny * v->nz;
    GC_REQUIRE(G < ((int64_t)1 << 31), GC_E_INVAL, "grid of %lld voxels exceeds 2^31", (long long)G);
    (void)m;
    return GC_OK;
}

int validate_bounds(const gc_model* m, const gc_bounds* b) {
    GC_REQUIRE(b && b->lb && b->ub, GC_E_INVAL, "bounds lb/ub missing");
    for (int p = 0; p < m->P; ++p) {
        GC_REQUIRE(std::isfinite(b->lb[p]) && std::isfinite(b->ub[p]) && b->lb[p] < b->ub[p],
                   GC_E_INVAL, "bounds of parameter %d must be finite with lb < ub", p);
        if (b->x0) {
            GC_REQUIRE(b->x0[p] >= b->lb[p] && b->x0[p] <= b->ub[p], GC_E_INVAL,
                       "x0 of parameter %d is outside its bounds", p);
        }
    }
    return GC_OK;
}

int pack_problem(Scratch& sc, const gc_model* m, const gc_volume* data, const uint8_t* mask,
                 const float* weights, const float* x0map, int mem_kind, Packed* out) {
    const int64_t G = (int64_t)data->nx * data->ny * data->nz;
    const hipStream_t s = sc.s;
    const void *dy, *dmask, *dw, *dx0;
    int rc;
    if ((rc = stage_in(sc, data->y, (size_t)G * m->Meff * sizeof(float), mem_kind, &dy))) return rc;
    if ((rc = stage_in(sc, mask, (size_t)G, mem_kind, &dmask))) return rc;
    if ((rc = stage_in(sc, weights, (size_t)G * sizeof(float), mem_kind, &dw))) return rc;
    if ((rc = stage_in(sc, x0map, (size_t)G * m->P * sizeof(float), mem_kind, &dx0))) return rc;
    PackPlan plan{};
    plan.n_grid = G;
    plan.n_tiles = (G + kTile - 1) / kTile;
    GC_TRY_HIP(sc.alloc_n(&plan.tile_count, plan.n_tiles));
    GC_TRY_HIP(sc.alloc_n(&plan.tile_offset, plan.n_tiles + 1));
    GC_TRY_HIP(sc.alloc_n(&plan.g2c, G));
    GC_TRY_HIP(sc.alloc_n(&plan.c2g, G));
    GC_TRY_HIP(pack_index((const uint8_t*)dmask, plan, s));
    int64_t n = 0;
    GC_TRY_HIP(hipMemcpyAsync(&n, plan.tile_offset + plan.n_tiles, sizeof(int64_t),
                              hipMemcpyDeviceToHost, s));
    GC_TRY_HIP(hipStreamSynchronize(s));
    out->G = G;
    out->n = n;
    out->g2c = plan.g2c;
    out->c2g = plan.c2g;
    int* flag = nullptr;
    GC_TRY_HIP(sc.alloc_n(&flag, 1));
    GC_TRY_HIP(fill_i32(flag, 1, 0, s));
    GC_TRY_HIP(sc.alloc_n(&out->y, (size_t)std::max<int64_t>(n, 1) * m->Meff));
    {
        // the pack step's data gather; timed like the hot kernels, except on
        // the allocation-free path (whose scratch is fixed), as there
        LaunchTimer tm("gather_rows", s);
        if (!sc.fixed) tm.begin();
        GC_TRY_HIP(gather_rows((const float*)dy, m->Meff, G, plan.c2g, n, out->y, flag, s));
        tm.end();
        if (!tm.ev.empty()) {   // timed: read it out here (a profiling mode)
            GC_TRY_HIP(hipStreamSynchronize(s));
            tm.flush();
        }
    }
    out->w = nullptr;
    if (dw) {
        GC_TRY_HIP(sc.alloc_n(&out->w, (size_t)std::max<int64_t>(n, 1)));
        GC_TRY_HIP(gather_rows((const float*)dw, 1, G, plan.c2g, n, out->w, flag, s));
    }
    out->x0 = nullptr;
    if (dx0) {
        GC_TRY_HIP(sc.alloc_n(&out->x0, (size_t)std::max<int64_t>(n, 1) * m->P));
        GC_TRY_HIP(gather_rows((const float*)dx0, m->P, G, plan.c2g, n, out->x0, flag, s));
    }
    int hflag = 0;
    GC_TRY_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    GC_TRY_HIP(hipStreamSynchronize(s));
    GC_REQUIRE(hflag == 0, GC_E_NONFINITE, "non-finite data, weight or start value inside the mask");
    return GC_OK;
}

int pack_prior(Scratch& sc, const gc_model* m, const gc_adam_hyper* h, const Packed& pk,
               int mem_kind, float** mu, float** sigma) {
    *mu = nullptr;
    *sigma = nullptr;
    if (!(h->prior_lambda > 0) || h->prior_mask == 0) return GC_OK;
    const hipStream_t s = sc.s;
    const int64_t G = pk.G, n = pk.n;
    const size_t bytes = (size_t)G * m->P * sizeof(float);
    const void *dmu, *dsg;
    int rc;
    if ((rc = stage_in(sc, h->prior_mu, bytes, mem_kind, &dmu))) return rc;
    if ((rc = stage_in(sc, h->prior_sigma, bytes, mem_kind, &dsg))) return rc;
    int* flag = nullptr;
    GC_TRY_HIP(sc.alloc_n(&flag, 2));
    GC_TRY_HIP(fill_i32(flag, 2, 0, s));
    const size_t np = (size_t)std::max<int64_t>(n, 1) * m->P;
    GC_TRY_HIP(sc.alloc_n(mu, np));
    GC_TRY_HIP(sc.alloc_n(sigma, np));
    GC_TRY_HIP(gather_rows((const float*)dmu, m->P, G, pk.c2g, n, *mu, flag, s));
    GC_TRY_HIP(gather_rows((const float*)dsg, m->P, G, pk.c2g, n, *sigma, flag, s));
    GC_TRY_HIP(check_positive(*sigma, n * m->P, flag + 1, s));
    int hf[2] = {0, 0};
    GC_TRY_HIP(hipMemcpyAsync(hf, flag, sizeof(hf), hipMemcpyDeviceToHost, s));
    GC_TRY_HIP(hipStreamSynchronize(s));
    GC_REQUIRE(hf[0] == 0, GC_E_NONFINITE, "non-finite prior mean or SD inside the mask");
    GC_REQUIRE(hf[1] == 0, GC_E_INVAL, "prior SDs must be > 0 inside the mask");
    return GC_OK;
}

int validate_graph(Scratch& sc, int64_t n, int64_t nnz, const int64_t* rowptr,
                   const int32_t* col, hipStream_t s) {
    int* flag = nullptr;
    GC_TRY_HIP(sc.alloc_n(&flag, 1));
    GC_TRY_HIP(fill_i32(flag, 1, 0, s));
    GC_TRY_HIP(check_graph(n, nnz, rowptr, col, flag, s));
    int h = 0;
    GC_TRY_HIP(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    GC_TRY_HIP(hipStreamSynchronize(s));
    GC_REQUIRE(h == 0, GC_E_INVAL,
               "graph adjacency: rowptr must start at 0, not decrease and end at nnz; "
               "neighbour indices must lie in [0, n)");
    return GC_OK;
}

int pack_graph(Scratch& sc, const gc_adam_hyper* h, int64_t n, int mem_kind, FitJob* J) {
    J->g_rowptr = nullptr;
    J->g_col = nullptr;
    J->g_nnz = 0;
    if (!(h->lambda > 0) || h->tv_mask == 0 || h->tv_kind != GC_TV_GRAPH) return GC_OK;
    GC_REQUIRE(h->graph_n == n, GC_E_INVAL,
               "graph_n (%lld) must equal the number of masked voxels (%lld)",
               (long long)h->graph_n, (long long)n);
    if (n == 0) return GC_OK;
    const void *drp, *dcol = nullptr;
    int rc;
    if ((rc = stage_in(sc, h->graph_rowptr, (size_t)(n + 1) * 8, mem_kind, &drp))) return rc;
    if (h->graph_nnz > 0 &&
        (rc = stage_in(sc, h->graph_col, (size_t)h->graph_nnz * 4, mem_kind, &dcol)))
        return rc;
    if ((rc = validate_graph(sc, n, h->graph_nnz, (const int64_t*)drp, (const int32_t*)dcol,
                             sc.s)))
        return rc;
    J->g_rowptr = (const int64_t*)drp;
    J->g_col = (const int32_t*)dcol;
    J->g_nnz = h->graph_nnz;
    return GC_OK;
}

int fill_mh_job(const gc_model* m, const gc_bounds* b, const gc_mcmc_hyper* h, int n_chains,
                int n_iter, int burnin, int thin, const AcqDev& acq, MhJob* J) {
    std::memset((void*)J, 0, sizeof(MhJob));
    GC_REQUIRE(h->sigma > 0 && std::isfinite(h->sigma), GC_E_INVAL, "sigma must be > 0");
    J->C = n_chains;
    J->P = m->P;
    J->k0 = (uint32_t)h->seed;
    J->k1 = (uint32_t)(h->seed >> 32);
    J->burnin = burnin;
    J->thin = thin;
    // retained steps t >= burnin with (t - burnin + 1) % thin == 0: those
    // before step T number max(0, T - burnin) / thin
    auto kept_before = [&](int T) { return T > burnin ? (T - burnin) / thin : 0; };
    J->k_base = kept_before(h->t_start);
    J->K = kept_before(n_iter) - J->k_base;
    J->s_base = J->k_base;   // a sample buffer holds all of this call's draws
    J->s_K = J->K;
    J->x0_mode = h->x0_mode;
    for (int p = 0; p < m->P; ++p) {
        const double lo = b->lb[p], hi = b->ub[p];
        const double st = h->step ? h->step[p] : 0.02 * (hi - lo);
        GC_REQUIRE(std::isfinite(st) && st > 0, GC_E_INVAL, "step of parameter %d must be > 0", p);
        const double x0 = b->x0 ? b->x0[p] : 0.5 * (lo + hi);
        J->lb[p] = (float)lo;
        J->ub[p] = (float)hi;
        J->step[p] = (float)st;
        J->x0c[p] = (float)x0;
        J->lbd[p] = lo;
        J->ubd[p] = hi;
        J->stepd[p] = st;
        J->x0cd[p] = x0;
        J->balld[p] = 0.01 * (hi - lo);
        J->ball[p] = (float)J->balld[p];
    }
    const double inv = 1.0 / (2.0 * h->sigma * h->sigma);
    J->inv2s2 = (float)inv;
    J->inv2s2d = inv;
    J->stretch = (float)(h->stretch > 1.0 ? h->stretch : 2.0);
    J->stretchd = h->stretch > 1.0 ? h->stretch : 2.0;
    J->acq = acq;
    return GC_OK;
}

int fill_fit_job(const gc_model* m, const gc_bounds* b, const gc_adam_hyper* h, int64_t n,
                 const AcqDev& acq, FitJob* J) {
    std::memset((void*)J, 0, sizeof(FitJob));
    J->n = n;
    J->P = m->P;
    J->loss_p = h->loss;
    J->optimizer = h->optimizer;
    J->tv_mask = h->lambda > 0 ? h->tv_mask : 0u;
    J->tv_kind = h->tv_kind;
    J->prior_mask = h->prior_lambda > 0 ? h->prior_mask : 0u;
    for (int p = 0; p < m->P; ++p) {
        const double lo = b->lb[p], hi = b->ub[p];
        J->lb[p] = (float)lo;
        J->rng[p] = (float)(hi - lo);
        const double x0 = b->x0 ? b->x0[p] : 0.5 * (lo + hi);
        J->u0[p] = (float)((x0 - lo) / (hi - lo));
    }
    J->lr = (float)h->lr;
    J->beta1 = (float)h->beta1;
    J->beta2 = (float)h->beta2;
    J->beta1d = h->beta1;
    J->beta2d = h->beta2;
    J->eps = (float)h->eps;
    J->momentum = (float)h->momentum;
    J->rho = (float)h->rho;
    J->omb1 = (float)(1.0 - h->beta1);
    J->omb2 = (float)(1.0 - h->beta2);
    J->omrho = (float)(1.0 - h->rho);
    const double N = (double)(n > 0 ? n : 1);
    J->scale_data = (float)(1.0 / (N * m->Meff));
    J->scale_tv = (float)(h->lambda / N);
    J->scale_prior = (float)(h->prior_lambda / N);
    // the same constants unrounded, for the FP64 instantiation
    for (int p = 0; p < m->P; ++p) {
        const double lo = b->lb[p], hi = b->ub[p];
        J->lbd[p] = lo;
        J->rngd[p] = hi - lo;
        const double x0 = b->x0 ? b->x0[p] : 0.5 * (lo + hi);
        J->u0d[p] = (x0 - lo) / (hi - lo);
    }
    J->lrd = h->lr;
    J->epsd = h->eps;
    J->momentumd = h->momentum;
    J->rhod = h->rho;
    J->omb1d = 1.0 - h->beta1;
    J->omb2d = 1.0 - h->beta2;
    J->omrhod = 1.0 - h->rho;
    J->scale_datad = 1.0 / (N * m->Meff);
    J->scale_tvd = h->lambda / N;
    J->scale_priord = h->prior_lambda / N;
    J->active = 1;
    J->acq = acq;
    return GC_OK;
}

int validate_adam(const gc_model* m, const gc_adam_hyper* h) {
    GC_REQUIRE(h, GC_E_INVAL, "hyper missing");
    GC_REQUIRE(h->n_iter >= 1, GC_E_INVAL, "n_iter must be >= 1");
    GC_REQUIRE(h->loss == 1 || h->loss == 2, GC_E_INVAL, "loss must be 1 or 2");
    GC_REQUIRE(h->optimizer >= 0 && h->optimizer <= 2, GC_E_INVAL, "unknown optimizer");
    GC_REQUIRE(h->lr > 0 && std::isfinite(h->lr), GC_E_INVAL, "lr must be > 0");
    GC_REQUIRE(h->beta1 >= 0 && h->beta1 < 1 && h->beta2 >= 0 && h->beta2 < 1, GC_E_INVAL,
               "beta1, beta2 must be in [0,1)");
    GC_REQUIRE(h->eps >= 0 && h->rho >= 0 && h->rho < 1 && h->momentum >= 0, GC_E_INVAL,
               "eps, rho, momentum out of range");
    GC_REQUIRE(h->lambda >= 0 && std::isfinite(h->lambda), GC_E_INVAL, "lambda must be >= 0");
    GC_REQUIRE(h->tv_dim == 2 || h->tv_dim == 3, GC_E_INVAL, "tv_dim must be 2 or 3");
    GC_REQUIRE((h->tv_mask >> m->P) == 0, GC_E_INVAL, "tv_mask names a parameter >= P");
    GC_REQUIRE(h->tv_kind >= GC_TV_ANISO && h->tv_kind <= GC_TV_GRAPH, GC_E_INVAL,
               "unknown tv_kind");
    if (h->lambda > 0 && h->tv_mask && h->tv_kind == GC_TV_GRAPH) {
        GC_REQUIRE(h->graph_rowptr && h->graph_nnz >= 0 && (h->graph_col || h->graph_nnz == 0),
                   GC_E_INVAL, "graph TV needs graph_rowptr, graph_col and graph_nnz >= 0");
        GC_REQUIRE(h->graph_n < INT32_MAX, GC_E_INVAL, "graph too large (n >= 2^31)");
    }
    GC_REQUIRE(h->prior_lambda >= 0 && std::isfinite(h->prior_lambda), GC_E_INVAL,
               "prior_lambda must be >= 0");
    GC_REQUIRE((h->prior_mask >> m->P) == 0, GC_E_INVAL, "prior_mask names a parameter >= P");
    GC_REQUIRE(!(h->prior_lambda > 0 && h->prior_mask) || (h->prior_mu && h->prior_sigma),
               GC_E_INVAL, "the prior needs prior_mu and prior_sigma");
    GC_REQUIRE(!(h->conv_value > 0) || h->conv_window > 1, GC_E_INVAL,
               "conv_window must be > 1");
    GC_REQUIRE(h->t_start >= 0 && h->t_start < h->n_iter, GC_E_INVAL,
               "t_start must be in [0, n_iter)");
    GC_REQUIRE(h->t_start == 0 || h->init_state, GC_E_INVAL,
               "resume (t_start > 0) needs init_state");
    GC_REQUIRE(h->t_start == 0 || !(h->conv_value > 0) || h->loss_history, GC_E_INVAL,
               "resume with a convergence window needs loss_history holding the first "
               "t_start losses");
    GC_REQUIRE(h->precision == GC_PREC_FP32 || h->precision == GC_PREC_FP64, GC_E_INVAL,
               "precision must be GC_PREC_FP32 or GC_PREC_FP64");
    GC_REQUIRE(h->precision == GC_PREC_FP32 || (h->t_start == 0 && !h->init_state &&
                                                !h->final_state),
               GC_E_INVAL, "checkpoint / resume is an FP32 option");
    return GC_OK;
}

}  // namespace gc

using namespace gc;

#define GC_GUARD_BEGIN try {
#define GC_GUARD_END                                              \
    }                                                             \
    catch (const std::bad_alloc&) {                               \
        set_error("host allocation failed");                      \
        return GC_E_NOMEM;                                        \
    }                                                             \
    catch (const std::exception& e) {                             \
        set_error("internal error: %s", e.what());                \
        return GC_E_DEVICE;                                       \
    }                                                             \
    catch (...) {                                                 \
        set_error("internal error");                              \
        return GC_E_DEVICE;                                       \
    }

extern "C" {

const char* gc_last_error(void) { return g_err.c_str(); }
#ifndef GC_SOURCE_HASH
#define GC_SOURCE_HASH "unknown"
#endif
const char* gc_version(void) { return "gacelle-mi355x 0.2 (gfx950) src " GC_SOURCE_HASH; }

int gc_model_create(const char* name, const gc_acq* acq, gc_model** out) {
    GC_GUARD_BEGIN
    clear_error();
    GC_REQUIRE(name && acq && out, GC_E_INVAL, "null argument");
    std::string nm(name);
    int kind;
    std::vector<std::string> pn;
    if (nm == "monoexp_t2s") { kind = MONOEXP_T2S; pn = {"S0", "T2star"}; }
    else if (nm == "monoexp_r2s") { kind = MONOEXP_R2S; pn = {"S0", "R2star"}; }
    else if (nm == "gre3") { kind = GRE3; pn = {"A1", "A2", "A3", "T2s1", "T2s2", "T2s3", "df1", "df2", "df3"}; }
    else if (nm == "dwi2") { kind = DWI2; pn = {"f", "Da", "De", "theta", "phi"}; }
    else if (nm == "linear3") { kind = LINEAR3; pn = {"A1", "A2", "A3"}; }
    else {
        set_error("unknown model '%s'", name);
        return GC_E_NOMODEL;
    }
    const int M = acq->n_meas;
    GC_REQUIRE(M >= 1 && M <= 4096, GC_E_INVAL, "n_meas must be in 1..4096");
    auto* m = new gc_model();
    m->kind = kind;
    m->P = (int)pn.size();
    m->M = M;
    m->complex_ = kind == GRE3;
    m->Meff = m->complex_ ? 2 * M : M;
    m->name = nm;
    m->pnames = pn;
    if (kind == DWI2) {
        if (!acq->bval || !acq->bvec) {
            delete m;
            set_error("dwi2 needs bval and bvec");
            return GC_E_INVAL;
        }
        m->bval.assign(acq->bval, acq->bval + M);
        m->bvec.assign(acq->bvec, acq->bvec + 3 * M);
        for (double x : m->bval) if (!std::isfinite(x) || x < 0) { delete m; set_error("bad bval"); return GC_E_INVAL; }
        for (double x : m->bvec) if (!std::isfinite(x)) { delete m; set_error("bad bvec"); return GC_E_INVAL; }
    } else {
        if (!acq->te) {
            delete m;
            set_error("model '%s' needs te", name);
            return GC_E_INVAL;
        }
        m->te.assign(acq->te, acq->te + M);
        for (double x : m->te) if (!std::isfinite(x) || x < 0) { delete m; set_error("bad te"); return GC_E_INVAL; }
        m->te0 = m->te[0];
        m->dte = M > 1 ? m->te[1] - m->te[0] : 0.0;
        bool uni = M > 1 && m->dte > 0;
        for (int j = 0; j < M && uni; ++j)
            uni = std::fabs(m->te[j] - (m->te0 + j * m->dte)) <= 1e-9 * std::max(1.0, std::fabs(m->te[j]));
        m->uniform = uni;
    }
    *out = m;
    return GC_OK;
    GC_GUARD_END
}

int gc_model_info(const gc_model* m, int* n_params, int* n_meas_eff, int* is_complex) {
    GC_REQUIRE(m, GC_E_INVAL, "null model");
    if (n_params) *n_params = m->P;
    if (n_meas_eff) *n_meas_eff = m->Meff;
    if (is_complex) *is_complex = m->complex_ ? 1 : 0;
    return GC_OK;
}

const char* gc_model_param_name(const gc_model* m, int p) {
    if (!m || p < 0 || p >= m->P) return nullptr;
    return m->pnames[p].c_str();
}

int gc_model_destroy(gc_model* m) {
    model_release(m);
    return GC_OK;
}

int gc_count_mask(const uint8_t* mask, int64_t n_grid, int64_t* n_masked, const gc_exec* exec) {
    GC_GUARD_BEGIN
    GC_REQUIRE(n_masked && n_grid >= 0, GC_E_INVAL, "bad arguments");
    if (!mask) { *n_masked = n_grid; return GC_OK; }
    std::vector<uint8_t> h;
    const uint8_t* p = mask;
    if (exec && exec->mem_kind == GC_MEM_DEVICE) {
        DeviceScope ds;
        int rc = ds.open(exec);
        if (rc) return rc;
        h.resize((size_t)n_grid);
        GC_TRY_HIP(hipMemcpyAsync(h.data(), mask, (size_t)n_grid, hipMemcpyDeviceToHost, ds.stream));
        GC_TRY_HIP(hipStreamSynchronize(ds.stream));
        p = h.data();
    }
    int64_t c = 0;
    for (int64_t i = 0; i < n_grid; ++i) c += p[i] ? 1 : 0;
    *n_masked = c;
    return GC_OK;
    GC_GUARD_END
}

void gc_adam_defaults(gc_adam_hyper* h) {
    std::memset(h, 0, sizeof(*h));
    h->optimizer = GC_OPT_ADAM;
    h->lr = 0.01;
    h->beta1 = 0.9;
    h->beta2 = 0.999;
    h->eps = 1e-8;
    h->momentum = 0.9;
    h->rho = 0.9;
    h->n_iter = 200;
    h->loss = 2;
    h->tv_dim = 3;
    h->conv_window = 20;
}

void gc_mcmc_defaults(gc_mcmc_hyper* h) {
    std::memset(h, 0, sizeof(*h));
    h->sigma = 1.0;
    h->precision = GC_PREC_FP32;
    h->sampler = GC_SAMPLER_MH;
    h->n_walkers = 50;
    h->stretch = 2.0;
}

int gc_burnin_from_ratio(double ratio, int n_iter) {
    if (!(ratio >= 0) || n_iter < 0) return 0;
    return (int)std::floor(ratio * (double)n_iter);
}

// ------------------------------------------------------------------ askadam
}  // extern "C"

namespace gc {
// The optimiser state [3][P][n] (u, m, v) of a fit: in = caller's state into
// the iterate buffer u and the moments m, v; out = the reverse.  The caller's
// array is exec memory (host or device), the copies are ordered on s.
static hipError_t copy_state(const void* st, float* u, float* m, float* v, size_t np, bool in,
                             hipStream_t s) {
    float* bufs[3] = {u, m, v};
    for (int k = 0; k < 3; ++k) {
        float* ext = (float*)st + (size_t)k * np;
        hipError_t e = in ? hipMemcpyAsync(bufs[k], ext, np * sizeof(float), hipMemcpyDefault, s)
                          : hipMemcpyAsync(ext, bufs[k], np * sizeof(float), hipMemcpyDefault, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
}  // namespace gc

extern "C" {

int gc_fit_askadam(const gc_model* model, const gc_volume* data, const uint8_t* mask,
                   const gc_bounds* bounds, const gc_adam_hyper* hyper, float* out_maps,
                   gc_fit_report* report, const gc_exec* exec) {
    GC_GUARD_BEGIN
    clear_error();
    int rc;
    GC_REQUIRE(model && out_maps, GC_E_INVAL, "null model or output");
    if ((rc = validate_volume(model, data))) return rc;
    if ((rc = validate_bounds(model, bounds))) return rc;
    if ((rc = validate_adam(model, hyper))) return rc;
    DeviceScope ds;
    if ((rc = ds.open(exec))) return rc;
    const hipStream_t s = ds.stream;
    Scratch sc(s);
    AcqDev acq;
    if ((rc = model_acq(model, ds.dev, &acq))) return rc;
    Packed pk;
    if ((rc = pack_problem(sc, model, data, mask, hyper->weights, bounds->x0_map, ds.mem_kind, &pk)))
        return rc;
    const int P = model->P;
    const int64_t n = pk.n, G = pk.G;
    const int T = hyper->n_iter;
    const int t_start = hyper->t_start;
    FitJob J;
    if ((rc = fill_fit_job(model, bounds, hyper, n, acq, &J))) return rc;
    J.y = pk.y;
    J.w = pk.w;
    J.x0map = pk.x0;
    float *pmu = nullptr, *psg = nullptr;
    if ((rc = pack_prior(sc, model, hyper, pk, ds.mem_kind, &pmu, &psg))) return rc;
    J.mu = pmu;
    J.sigma = psg;
    if ((rc = pack_graph(sc, hyper, n, ds.mem_kind, &J))) return rc;
    float *u0 = nullptr, *u1 = nullptr, *m = nullptr, *v = nullptr;
    const size_t np = (size_t)std::max<int64_t>(n, 1) * P;
    GC_TRY_HIP(sc.alloc_n(&u0, np));
    GC_TRY_HIP(sc.alloc_n(&u1, np));
    GC_TRY_HIP(sc.alloc_n(&m, np));
    GC_TRY_HIP(sc.alloc_n(&v, np));
    J.u = u0;
    J.m = m;
    J.v = v;
    const int64_t nblk = (n + kBlock - 1) / kBlock;
    std::vector<BlkMap> hmap((size_t)std::max<int64_t>(nblk, 1));
    for (int64_t b = 0; b < nblk; ++b) hmap[b] = BlkMap{0, 0, b * kBlock};
    BlkMap* dmap = nullptr;
    GC_TRY_HIP(sc.alloc_n(&dmap, hmap.size()));
    GC_TRY_HIP(hipMemcpyAsync(dmap, hmap.data(), hmap.size() * sizeof(BlkMap), hipMemcpyHostToDevice, s));

    int iters = T, reason = 0;
    double final_loss = 0.0;
    // host descriptors stay alive until the stream has consumed them
    std::vector<FitJob> jobs;
    float* theta_c = nullptr;
    GC_TRY_HIP(sc.alloc_n(&theta_c, np));
    if (n > 0) {
        const bool tv = J.tv_mask != 0;
        const bool stopping = hyper->tol > 0 || hyper->conv_value > 0;
        const bool history = hyper->loss_history != nullptr;
        FitJob* djob = nullptr;
        const bool f64 = hyper->precision == GC_PREC_FP64;
        if (!f64 && !tv && !stopping && !history) {
            // fused path: the whole loop in registers, chunks of <= 1000 iterations
            const int chunk = 1000;
            const int nck = (T - t_start + chunk - 1) / chunk;
            jobs.assign(nck, J);
            float* lossv = nullptr;
            GC_TRY_HIP(sc.alloc_n(&lossv, (size_t)n));
            // bias-correction powers after t_start iterations, multiplied in
            // the order the kernel multiplies them
            double b1 = 1.0, b2 = 1.0;
            for (int t = 1; t <= t_start; ++t) {
                b1 *= hyper->beta1;
                b2 *= hyper->beta2;
            }
            for (int c = 0; c < nck; ++c) {
                jobs[c].t0 = t_start + c * chunk + 1;
                jobs[c].t1 = std::min(T, t_start + (c + 1) * chunk);
                jobs[c].b1pow = b1;
                jobs[c].b2pow = b2;
                for (int t = jobs[c].t0; t <= jobs[c].t1; ++t) {
                    b1 *= hyper->beta1;
                    b2 *= hyper->beta2;
                }
                jobs[c].t_rec = T;
                jobs[c].loss_v = lossv;
            }
            GC_TRY_HIP(sc.alloc_n(&djob, (size_t)nck));
            GC_TRY_HIP(hipMemcpyAsync(djob, jobs.data(), nck * sizeof(FitJob), hipMemcpyHostToDevice, s));
            if (t_start == 0) GC_TRY_HIP(fit_init(djob, dmap, (int)nblk, s));
            else GC_TRY_HIP(copy_state(hyper->init_state, u0, m, v, np, true, s));
            const int maxm = fit_pick_maxm(model->kind, model->M);
            LaunchTimer tm("fit_fused", s);
            for (int c = 0; c < nck; ++c) {
                tm.begin();
                GC_TRY_HIP(fit_fused(model->kind, maxm, djob + c, dmap, (int)nblk, s));
                tm.end();
            }
            if (timing_on()) {
                GC_TRY_HIP(hipStreamSynchronize(s));
                tm.flush();
            }
            double* dl = nullptr;
            GC_TRY_HIP(sc.alloc_n(&dl, 1));
            GC_TRY_HIP(sum_partials(lossv, n, dl, s));
            GC_TRY_HIP(hipMemcpyAsync(&final_loss, dl, sizeof(double), hipMemcpyDeviceToHost, s));
            GC_TRY_HIP(fit_theta(P, J.lb, J.rng, u0, n, theta_c, s));
            if (hyper->final_state)
                GC_TRY_HIP(copy_state(hyper->final_state, u0, m, v, np, false, s));
        } else {
            // step path: one launch per iteration, double-buffered iterate
            int32_t* nbr = nullptr;
            if (tv && hyper->tv_kind != GC_TV_GRAPH) {
                GC_TRY_HIP(sc.alloc_n(&nbr, (size_t)n * 6));
                GC_TRY_HIP(build_neighbours(pk.c2g, pk.g2c, n, data->nx, data->ny, data->nz,
                                            hyper->tv_dim, nbr, s));
            }
            float* partial = nullptr;
            double* hist = nullptr;
            int* stop = nullptr;
            // the loss is reduced on every iteration only when a stopping rule or
            // the history needs it, else once, on the last iteration
            const bool each = stopping || history;
            // FP64 instantiation: its own iterate, moments and loss partials
            double *u0d = nullptr, *u1d = nullptr, *md = nullptr, *vd = nullptr,
                   *partiald = nullptr;
            if (f64) {
                GC_TRY_HIP(sc.alloc_n(&u0d, np));
                GC_TRY_HIP(sc.alloc_n(&u1d, np));
                GC_TRY_HIP(sc.alloc_n(&md, np));
                GC_TRY_HIP(sc.alloc_n(&vd, np));
                GC_TRY_HIP(sc.alloc_n(&partiald, (size_t)nblk * (each ? T : 1)));
            }
            GC_TRY_HIP(sc.alloc_n(&partial, (size_t)nblk * (each ? T : 1)));
            GC_TRY_HIP(sc.alloc_n(&hist, (size_t)T));
            GC_TRY_HIP(sc.alloc_n(&stop, 2));
            GC_TRY_HIP(fill_i32(stop, 2, 0, s));
            jobs.assign(T, J);
            double b1 = 1.0, b2 = 1.0;
            for (int t = 1; t <= T; ++t) {
                FitJob& q = jobs[t - 1];
                b1 *= hyper->beta1;
                b2 *= hyper->beta2;
                q.c1 = (float)(1.0 / (1.0 - b1));
                q.c2 = (float)(1.0 / (1.0 - b2));
                q.c1d = 1.0 / (1.0 - b1);
                q.c2d = 1.0 / (1.0 - b2);
                q.u = u0;   // fit_init writes here
                q.u_in = (t % 2 == 1) ? u0 : u1;
                q.u_out = (t % 2 == 1) ? u1 : u0;
                q.ud = u0d;
                q.u_ind = (t % 2 == 1) ? u0d : u1d;
                q.u_outd = (t % 2 == 1) ? u1d : u0d;
                q.md = md;
                q.vd = vd;
                q.nbr = nbr;
                q.record = (each || t == T) ? 1 : 0;
                q.partial = partial + (each ? (size_t)(t - 1) * nblk : 0);
                q.partiald = f64 ? partiald + (each ? (size_t)(t - 1) * nblk : 0) : nullptr;
                q.blk0 = 0;
                q.stop = stop;
            }
            GC_TRY_HIP(sc.alloc_n(&djob, (size_t)T));
            GC_TRY_HIP(hipMemcpyAsync(djob, jobs.data(), T * sizeof(FitJob), hipMemcpyHostToDevice, s));
            if (f64) {
                GC_TRY_HIP(fit_init_f64(djob, dmap, (int)nblk, s));
            } else if (t_start == 0) {
                GC_TRY_HIP(fit_init(djob, dmap, (int)nblk, s));
            } else {
                // iteration t_start + 1 reads the iterate from its u_in buffer;
                // the convergence window sees the earlier losses
                float* uin = ((t_start + 1) % 2 == 1) ? u0 : u1;
                GC_TRY_HIP(copy_state(hyper->init_state, uin, m, v, np, true, s));
                if (history)
                    GC_TRY_HIP(hipMemcpyAsync(hist, hyper->loss_history, t_start * sizeof(double),
                                              hipMemcpyHostToDevice, s));
            }
            const double tol = hyper->tol > 0 ? hyper->tol : -INFINITY;
            const int poll = 32;
            int hstop[2] = {0, 0};
            LaunchTimer tm("fit_step", s);
            for (int t = t_start + 1; t <= T; ++t) {
                tm.begin();
                if (f64) GC_TRY_HIP(fit_step_f64(model->kind, djob + (t - 1), dmap, (int)nblk, 1, s));
                else GC_TRY_HIP(fit_step(model->kind, djob + (t - 1), dmap, (int)nblk, 1, s));
                tm.end();
                if (jobs[t - 1].record && f64)
                    GC_TRY_HIP(fit_loss_stop_f64(jobs[t - 1].partiald, nblk, hist, t, tol,
                                                 hyper->conv_value, hyper->conv_window, stop, s));
                else if (jobs[t - 1].record)
                    GC_TRY_HIP(fit_loss_stop(jobs[t - 1].partial, nblk, hist, t, tol,
                                             hyper->conv_value, hyper->conv_window, stop, s));
                if (stopping && t % poll == 0 && t < T) {
                    GC_TRY_HIP(hipMemcpyAsync(hstop, stop, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
                    GC_TRY_HIP(hipStreamSynchronize(s));
                    if (hstop[0] != 0) break;
                }
            }
            GC_TRY_HIP(hipMemcpyAsync(hstop, stop, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
            GC_TRY_HIP(hipStreamSynchronize(s));
            tm.flush();
            if (hstop[0] != 0) {
                iters = hstop[0];
                reason = hstop[1];
            }
            if (history) {
                GC_TRY_HIP(hipMemcpyAsync(hyper->loss_history, hist, iters * sizeof(double),
                                          hipMemcpyDeviceToHost, s));
                GC_TRY_HIP(hipStreamSynchronize(s));
                final_loss = hyper->loss_history[iters - 1];
            } else {
                GC_TRY_HIP(hipMemcpyAsync(&final_loss, hist + (iters - 1), sizeof(double),
                                          hipMemcpyDeviceToHost, s));
                GC_TRY_HIP(hipStreamSynchronize(s));
            }
            float* ufin = (iters % 2 == 1) ? u1 : u0;
            if (f64)
                GC_TRY_HIP(fit_theta_f64(P, J.lbd, J.rngd, (iters % 2 == 1) ? u1d : u0d, n,
                                         theta_c, s));
            else
                GC_TRY_HIP(fit_theta(P, J.lb, J.rng, ufin, n, theta_c, s));
            if (hyper->final_state)
                GC_TRY_HIP(copy_state(hyper->final_state, ufin, m, v, np, false, s));
        }
    }
    // scatter to the grid (0 outside the mask)
    float* dout = out_maps;
    if (ds.mem_kind == GC_MEM_HOST) GC_TRY_HIP(sc.alloc_n(&dout, (size_t)G * P));
    GC_TRY_HIP(scatter_rows_f32(theta_c, P, n, pk.g2c, G, dout, s));
    if (ds.mem_kind == GC_MEM_HOST)
        GC_TRY_HIP(hipMemcpyAsync(out_maps, dout, (size_t)G * P * sizeof(float), hipMemcpyDeviceToHost, s));
    GC_TRY_HIP(hipStreamSynchronize(s));
    if (report) {
        report->iters_run = n > 0 ? iters : 0;
        report->final_loss = final_loss;
        report->stop_reason = reason;
    }
    return GC_OK;
    GC_GUARD_END
}

}  // extern "C"

namespace gc {

// ------------------------------------------------------------------ MCMC
// Model acquisition tables copied into a caller-provided scratch region (the
// allocation-free entry point), with the same layout as model_acq's.
static int model_acq_into(const gc_model* m, Scratch& sc, AcqDev* out) {
    const int M = m->M;
    std::vector<float> f(5 * M, 0.f);
    std::vector<double> d(5 * M, 0.0);
    for (int j = 0; j < M; ++j) {
        if (!m->te.empty()) {
            f[j] = (float)m->te[j];
            d[j] = m->te[j];
        }
        if (!m->bval.empty()) {
            f[M + j] = (float)(m->bval[j] * 1e-3);
            d[M + j] = m->bval[j] * 1e-3;
            for (int k = 0; k < 3; ++k) {
                f[2 * M + 3 * j + k] = (float)m->bvec[3 * j + k];
                d[2 * M + 3 * j + k] = m->bvec[3 * j + k];
            }
        }
    }
    std::vector<int32_t> run_end;
    for (int j = 1; j < M; ++j)
        if (!m->bval.empty() && m->bval[j] != m->bval[j - 1]) run_end.push_back(j);
    run_end.push_back(M);
    float* fp = nullptr;
    double* dp = nullptr;
    int32_t* rp = nullptr;
    GC_TRY_HIP(sc.alloc_n(&fp, f.size()));
    GC_TRY_HIP(sc.alloc_n(&dp, d.size()));
    GC_TRY_HIP(sc.alloc_n(&rp, run_end.size()));
    GC_TRY_HIP(hipMemcpyAsync(fp, f.data(), f.size() * 4, hipMemcpyHostToDevice, sc.s));
    GC_TRY_HIP(hipMemcpyAsync(dp, d.data(), d.size() * 8, hipMemcpyHostToDevice, sc.s));
    GC_TRY_HIP(hipMemcpyAsync(rp, run_end.data(), run_end.size() * 4, hipMemcpyHostToDevice, sc.s));
    GC_TRY_HIP(hipStreamSynchronize(sc.s));   // the host vectors go out of scope
    AcqDev a{};
    a.te = fp;
    a.bval = fp + M;
    a.bvec = fp + 2 * M;
    a.te_d = dp;
    a.bval_d = dp + M;
    a.bvec_d = dp + 2 * M;
    a.M = M;
    a.uniform = m->uniform ? 1 : 0;
    a.te0 = (float)m->te0;
    a.dte = (float)m->dte;
    a.te0_d = m->te0;
    a.dte_d = m->dte;
    a.run_end = rp;
    a.nrun = (int)run_end.size();
    *out = a;
    return GC_OK;
}

int mcmc_validate(const gc_model* model, const gc_volume* data, const gc_bounds* bounds,
                  int* n_chains, int n_iter, int burnin, int thin, const gc_mcmc_hyper* hyper,
                  const double* out_mean, const double* out_std, const float* out_samples) {
    int rc;
    GC_REQUIRE(model && hyper && out_mean && out_std, GC_E_INVAL, "null argument");
    if ((rc = validate_volume(model, data))) return rc;
    if ((rc = validate_bounds(model, bounds))) return rc;
    const bool ens = hyper->sampler == GC_SAMPLER_ENSEMBLE;
    GC_REQUIRE(hyper->sampler == GC_SAMPLER_MH || ens, GC_E_INVAL, "unknown sampler");
    if (ens) {
        GC_REQUIRE(hyper->n_walkers >= 4 && hyper->n_walkers % 2 == 0 && hyper->n_walkers <= 512,
                   GC_E_INVAL, "n_walkers must be even, in 4..512");
        *n_chains = hyper->n_walkers;
    }
    GC_REQUIRE(*n_chains >= 1 && *n_chains <= 65535, GC_E_INVAL, "n_chains must be in 1..65535");
    GC_REQUIRE(n_iter >= 1 && burnin >= 0 && burnin < n_iter && thin >= 1, GC_E_INVAL,
               "need n_iter >= 1, 0 <= burnin < n_iter, thin >= 1");
    GC_REQUIRE(hyper->t_start >= 0 && hyper->t_start < n_iter, GC_E_INVAL,
               "t_start must be in [0, n_iter)");
    GC_REQUIRE(hyper->t_start == 0 || hyper->init_state, GC_E_INVAL,
               "resuming at t_start > 0 needs init_state");
    GC_REQUIRE(!ens || (hyper->t_start == 0 && !hyper->init_state), GC_E_INVAL,
               "resume (t_start, init_state) is for the MH sampler");
    {
        const int k_all = (n_iter - burnin) / thin;
        const int k_before = hyper->t_start > burnin ? (hyper->t_start - burnin) / thin : 0;
        GC_REQUIRE(k_all - k_before >= 2, GC_E_INVAL,
                   "fewer than 2 retained samples per chain in this call");
    }
    GC_REQUIRE(hyper->precision == GC_PREC_FP32 || hyper->precision == GC_PREC_FP64, GC_E_INVAL,
               "precision must be GC_PREC_FP32 or GC_PREC_FP64");
    GC_REQUIRE(hyper->x0_mode >= 0 && hyper->x0_mode <= 2, GC_E_INVAL, "bad x0_mode");
    GC_REQUIRE(!(hyper->sample_sink && out_samples), GC_E_INVAL,
               "give either out_samples or a sample sink, not both");
    return GC_OK;
}

namespace {

// Pinned host staging, copy stream and events of a sample sink; released by
// the destructor (after the streams have been synchronised by the caller).
struct SinkRes {
    void* pin[2] = {nullptr, nullptr};
    hipEvent_t done[2] = {nullptr, nullptr}, copied[2] = {nullptr, nullptr};
    hipStream_t cs = nullptr;
    ~SinkRes() {
        if (cs) {
            (void)hipStreamSynchronize(cs);
            (void)hipStreamDestroy(cs);
        }
        for (int i = 0; i < 2; ++i) {
            if (pin[i]) (void)hipHostFree(pin[i]);
            if (done[i]) (void)hipEventDestroy(done[i]);
            if (copied[i]) (void)hipEventDestroy(copied[i]);
        }
    }
};

}  // namespace

// The body of gc_mcmc and of its allocation-free variant: all device memory
// comes from `sc`; with noalloc the model tables are staged into it too and
// nothing else is allocated (no free-memory query, no timing events).
int mcmc_impl(const gc_model* model, const gc_volume* data, const uint8_t* mask,
              const gc_bounds* bounds, int n_chains, int n_iter, int burnin, int thin,
              const gc_mcmc_hyper* hyper, double* out_mean, double* out_std, float* out_samples,
              int32_t* out_accept, DeviceScope& ds, Scratch& sc, bool noalloc) {
    int rc;
    const bool ens = hyper->sampler == GC_SAMPLER_ENSEMBLE;
    const bool fp64 = hyper->precision == GC_PREC_FP64;
    const hipStream_t s = ds.stream;
    AcqDev acq;
    if (noalloc) {
        if ((rc = model_acq_into(model, sc, &acq))) return rc;
    } else if ((rc = model_acq(model, ds.dev, &acq))) {
        return rc;
    }
    Packed pk;
    const float* x0map = hyper->x0_mode == GC_X0_GIVEN ? bounds->x0_map : nullptr;
    if ((rc = pack_problem(sc, model, data, mask, hyper->weights, x0map, ds.mem_kind, &pk)))
        return rc;
    const int P = model->P, C = n_chains;
    const int64_t n = pk.n, G = pk.G, NL = n * C;
    MhJob J;
    if ((rc = fill_mh_job(model, bounds, hyper, C, n_iter, burnin, thin, acq, &J))) return rc;
    const int K = J.K;
    J.y = pk.y;
    J.w = pk.w;
    J.x0map = pk.x0;
    J.n = n;
    if (hyper->init_state && n > 0) {
        const void *dis = nullptr, *dil = nullptr;
        if ((rc = stage_in(sc, hyper->init_state, (size_t)P * C * n * sizeof(double), ds.mem_kind,
                           &dis)))
            return rc;
        if ((rc = stage_in(sc, hyper->init_logl, (size_t)C * n * sizeof(double), ds.mem_kind,
                           &dil)))
            return rc;
        J.init_state = (const double*)dis;
        J.init_logl = (const double*)dil;
    }
    const size_t rs = fp64 ? sizeof(double) : sizeof(float);
    const size_t nl1 = (size_t)std::max<int64_t>(NL, 1);
    if (!noalloc) {   // footprint check against free device memory
        size_t freeb = 0, totalb = 0;
        GC_TRY_HIP(hipMemGetInfo(&freeb, &totalb));
        const size_t need = nl1 * (P * rs + rs + 4 + 2 * P * sizeof(double));
        GC_REQUIRE(need < freeb, GC_E_NOMEM, "chain state needs %zu bytes, %zu free", need, freeb);
    }
    GC_TRY_HIP(sc.alloc(&J.th, nl1 * P * rs));
    GC_TRY_HIP(sc.alloc(&J.ll, nl1 * rs));
    GC_TRY_HIP(sc.alloc_n(&J.acc, nl1));
    GC_TRY_HIP(sc.alloc_n(&J.mean, nl1 * P));
    GC_TRY_HIP(sc.alloc_n(&J.m2, nl1 * P));
    float* dsamp = out_samples;
    const size_t nsamp = (size_t)C * K * P * (size_t)n;
    if (out_samples && ds.mem_kind == GC_MEM_HOST) GC_TRY_HIP(sc.alloc_n(&dsamp, std::max<size_t>(nsamp, 1)));
    J.samples = dsamp;
    std::vector<MhJob> jobs;
    std::vector<BlkMap> hmap, emap;
    std::vector<int> delivery;   // sink: delivery index of each launch (-1 = none)
    double *mean_c = nullptr, *std_c = nullptr;
    GC_TRY_HIP(sc.alloc_n(&mean_c, (size_t)std::max<int64_t>(n, 1) * P));
    GC_TRY_HIP(sc.alloc_n(&std_c, (size_t)std::max<int64_t>(n, 1) * P));
    SinkRes sink;
    const bool streaming = hyper->sample_sink != nullptr && n > 0;
    int kc = 0;                  // retained draws per chain per delivery
    float* sbuf[2] = {nullptr, nullptr};
    if (n > 0) {
        const int chunk = hyper->chunk_iters > 0 ? hyper->chunk_iters : 1000;
        const int t_first = hyper->t_start;
        if (!streaming) {
            const int nck = (n_iter - t_first + chunk - 1) / chunk;
            jobs.assign(nck, J);
            for (int c = 0; c < nck; ++c) {
                jobs[c].t0 = t_first + c * chunk;
                jobs[c].t1 = std::min(n_iter, t_first + (c + 1) * chunk);
            }
        } else {
            // Deliveries of kc retained draws per chain ([C][kc][P][n] FP32, at
            // most sink_bytes, at least one draw); delivery j holds the draws
            // k_base + j kc + 1 .. of this call, retained at steps
            // t = burnin - 1 + k thin.  Its launches end right after its last
            // draw (at most chunk steps each), and it is written into one of two
            // device buffers while the other is copied to the host.
            const size_t per_draw = (size_t)C * P * (size_t)n * sizeof(float);
            const size_t cap = hyper->sink_bytes > 0 ? hyper->sink_bytes : ((size_t)256 << 20);
            kc = (int)std::max<size_t>(1, std::min<size_t>((size_t)K, cap / per_draw));
            const int nd = (K + kc - 1) / kc;
            int t = t_first;
            for (int j = 0; j < nd; ++j) {
                const int k_lo = J.k_base + j * kc;                 // draws before this delivery
                const int k_hi = J.k_base + std::min(K, (j + 1) * kc);
                const int t_end = j == nd - 1 ? n_iter : burnin - 1 + k_hi * thin + 1;
                for (; t < t_end; t = std::min(t_end, t + chunk)) {
                    MhJob q = J;
                    q.t0 = t;
                    q.t1 = std::min(t_end, t + chunk);
                    q.s_base = k_lo;
                    q.s_K = k_hi - k_lo;
                    jobs.push_back(q);
                    delivery.push_back(j);
                }
            }
            for (int b = 0; b < 2 && b < nd; ++b) {
                GC_TRY_HIP(sc.alloc_n(&sbuf[b], (size_t)C * kc * P * (size_t)n));
                GC_TRY_HIP(hipHostMalloc(&sink.pin[b], per_draw * kc, hipHostMallocDefault));
                GC_TRY_HIP(hipEventCreateWithFlags(&sink.done[b], hipEventDisableTiming));
                GC_TRY_HIP(hipEventCreateWithFlags(&sink.copied[b], hipEventDisableTiming));
            }
            GC_TRY_HIP(hipStreamCreateWithFlags(&sink.cs, hipStreamNonBlocking));
            for (size_t i = 0; i < jobs.size(); ++i) jobs[i].samples = sbuf[delivery[i] % 2];
        }
        const int nck = (int)jobs.size();
        MhJob* djob = nullptr;
        GC_TRY_HIP(sc.alloc_n(&djob, (size_t)nck));
        GC_TRY_HIP(hipMemcpyAsync(djob, jobs.data(), nck * sizeof(MhJob), hipMemcpyHostToDevice, s));
        const int64_t nblk = (NL + kBlock - 1) / kBlock;
        const int64_t vblk = (n + kBlock - 1) / kBlock;
        GC_REQUIRE(nblk < (1LL << 31), GC_E_INVAL, "too many chains x voxels");
        hmap.resize((size_t)nblk + (size_t)vblk);
        for (int64_t b = 0; b < nblk; ++b) hmap[b] = BlkMap{0, 0, b * kBlock};
        for (int64_t b = 0; b < vblk; ++b) hmap[nblk + b] = BlkMap{0, 0, b * kBlock};
        BlkMap* dmap = nullptr;
        GC_TRY_HIP(sc.alloc_n(&dmap, hmap.size()));
        GC_TRY_HIP(hipMemcpyAsync(dmap, hmap.data(), hmap.size() * sizeof(BlkMap), hipMemcpyHostToDevice, s));
        const BlkMap* cmap = dmap;   // chunk launches: lanes, or voxel groups for the ensemble
        int cblk = (int)nblk;
        if (ens) {
            GC_TRY_HIP(ens_init(model->kind, fp64, djob, dmap, (int)nblk, s));
            // chunks: blocks cover groups of vpb voxels with all their walkers
            const int vpb = kBlock / (C / 2);
            const int64_t eblk = (n + vpb - 1) / vpb;
            emap.resize((size_t)eblk);
            for (int64_t b = 0; b < eblk; ++b) emap[b] = BlkMap{0, 0, b * vpb};
            BlkMap* demap = nullptr;
            GC_TRY_HIP(sc.alloc_n(&demap, emap.size()));
            GC_TRY_HIP(hipMemcpyAsync(demap, emap.data(), emap.size() * sizeof(BlkMap),
                                      hipMemcpyHostToDevice, s));
            cmap = demap;
            cblk = (int)eblk;
        } else {
            GC_TRY_HIP(mh_init(model->kind, fp64, djob, dmap, (int)nblk, s));
        }
        const int maxm = mh_pick_variant(model->kind, model->M, model->uniform ? 1 : 0);
        LaunchTimer tm(ens ? "ens_chunk" : "mh_chunk", s);
        const bool timed = !noalloc && timing_on();
        auto launch = [&](int c) -> int {
            if (timed) tm.begin();
            if (ens)
                GC_TRY_HIP(ens_chunk_walkers(model->kind, fp64, djob + c, cmap, cblk, C,
                                             model->Meff, s));
            else
                GC_TRY_HIP(mh_chunk(model->kind, fp64, maxm, djob + c, cmap, cblk, C, model->Meff, s));
            if (timed) tm.end();
            return GC_OK;
        };
        if (!streaming) {
            for (int c = 0; c < nck; ++c)
                if ((rc = launch(c))) return rc;
        } else {
            // delivery j: launches into buffer j % 2 (after the copy of delivery
            // j - 2 has read it), then an event; the host hands delivery j - 2
            // to the sink (its pinned slot is then free) and queues the copy of
            // delivery j on the copy stream
            const size_t per_draw = (size_t)C * P * (size_t)n * sizeof(float);
            const int nd = delivery.back() + 1;
            auto deliver = [&](int j) -> int {
                const int b = j % 2;
                GC_TRY_HIP(hipEventSynchronize(sink.copied[b]));
                const int k_first = j * kc;
                const int k_cnt = std::min(K, (j + 1) * kc) - k_first;
                const int r = hyper->sample_sink(hyper->sink_user, k_first, k_cnt,
                                                 (const float*)sink.pin[b], n, C, P);
                GC_REQUIRE(r == 0, GC_E_CANCELLED, "the sample sink stopped the run (%d)", r);
                return GC_OK;
            };
            int c = 0;
            for (int j = 0; j < nd; ++j) {
                const int b = j % 2;
                if (j >= 2) GC_TRY_HIP(hipStreamWaitEvent(s, sink.copied[b], 0));
                for (; c < nck && delivery[c] == j; ++c)
                    if ((rc = launch(c))) return rc;
                GC_TRY_HIP(hipEventRecord(sink.done[b], s));
                if (j >= 2 && (rc = deliver(j - 2))) {
                    (void)hipStreamSynchronize(s);
                    return rc;
                }
                const int k_cnt = std::min(K, (j + 1) * kc) - j * kc;
                GC_TRY_HIP(hipStreamWaitEvent(sink.cs, sink.done[b], 0));
                GC_TRY_HIP(hipMemcpyAsync(sink.pin[b], sbuf[b], per_draw * k_cnt,
                                          hipMemcpyDeviceToHost, sink.cs));
                GC_TRY_HIP(hipEventRecord(sink.copied[b], sink.cs));
            }
            for (int j = std::max(0, nd - 2); j < nd; ++j)
                if ((rc = deliver(j))) {
                    (void)hipStreamSynchronize(s);
                    return rc;
                }
        }
        if (timed) {
            GC_TRY_HIP(hipStreamSynchronize(s));
            tm.flush();
        }
        GC_TRY_HIP(mh_finalize(fp64, djob, dmap + nblk, (int)vblk, mean_c, std_c, s));
    }
    // outputs
    double* dmean = out_mean;
    double* dstd = out_std;
    int32_t* dacc = out_accept;
    if (ds.mem_kind == GC_MEM_HOST) {
        GC_TRY_HIP(sc.alloc_n(&dmean, (size_t)G * P));
        GC_TRY_HIP(sc.alloc_n(&dstd, (size_t)G * P));
        if (out_accept) GC_TRY_HIP(sc.alloc_n(&dacc, (size_t)G * C));
    }
    GC_TRY_HIP(scatter_rows_f64(mean_c, P, n, pk.g2c, G, dmean, s));
    GC_TRY_HIP(scatter_rows_f64(std_c, P, n, pk.g2c, G, dstd, s));
    if (out_accept) GC_TRY_HIP(scatter_rows_i32(J.acc, C, n, pk.g2c, G, dacc, s));
    if (hyper->final_state && n > 0) {
        double* dfs = hyper->final_state;
        if (ds.mem_kind == GC_MEM_HOST) GC_TRY_HIP(sc.alloc_n(&dfs, (size_t)NL * P));
        if (fp64) GC_TRY_HIP(hipMemcpyAsync(dfs, J.th, (size_t)NL * P * sizeof(double), hipMemcpyDeviceToDevice, s));
        else GC_TRY_HIP(f32_to_f64((const float*)J.th, dfs, NL * P, s));
        if (ds.mem_kind == GC_MEM_HOST)
            GC_TRY_HIP(hipMemcpyAsync(hyper->final_state, dfs, (size_t)NL * P * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    if (hyper->final_logl && n > 0) {
        double* dfl = hyper->final_logl;
        if (ds.mem_kind == GC_MEM_HOST) GC_TRY_HIP(sc.alloc_n(&dfl, (size_t)NL));
        if (fp64) GC_TRY_HIP(hipMemcpyAsync(dfl, J.ll, (size_t)NL * sizeof(double), hipMemcpyDeviceToDevice, s));
        else GC_TRY_HIP(f32_to_f64((const float*)J.ll, dfl, NL, s));
        if (ds.mem_kind == GC_MEM_HOST)
            GC_TRY_HIP(hipMemcpyAsync(hyper->final_logl, dfl, (size_t)NL * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    if (ds.mem_kind == GC_MEM_HOST) {
        GC_TRY_HIP(hipMemcpyAsync(out_mean, dmean, (size_t)G * P * sizeof(double), hipMemcpyDeviceToHost, s));
        GC_TRY_HIP(hipMemcpyAsync(out_std, dstd, (size_t)G * P * sizeof(double), hipMemcpyDeviceToHost, s));
        if (out_accept)
            GC_TRY_HIP(hipMemcpyAsync(out_accept, dacc, (size_t)G * C * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        if (out_samples && nsamp)
            GC_TRY_HIP(hipMemcpyAsync(out_samples, dsamp, nsamp * sizeof(float), hipMemcpyDeviceToHost, s));
    }
    GC_TRY_HIP(hipStreamSynchronize(s));
    return GC_OK;
}

}  // namespace gc

extern "C" {

int gc_mcmc(const gc_model* model, const gc_volume* data, const uint8_t* mask,
            const gc_bounds* bounds, int n_chains, int n_iter, int burnin, int thin,
            const gc_mcmc_hyper* hyper, double* out_mean, double* out_std, float* out_samples,
            int32_t* out_accept, const gc_exec* exec) {
    GC_GUARD_BEGIN
    clear_error();
    int rc;
    if ((rc = mcmc_validate(model, data, bounds, &n_chains, n_iter, burnin, thin, hyper, out_mean,
                            out_std, out_samples)))
        return rc;
    DeviceScope ds;
    if ((rc = ds.open(exec))) return rc;
    Scratch sc(ds.stream);
    return mcmc_impl(model, data, mask, bounds, n_chains, n_iter, burnin, thin, hyper, out_mean,
                     out_std, out_samples, out_accept, ds, sc, false);
    GC_GUARD_END
}

// ------------------------------------------------------------ autograd ops
static int stage_simple(Scratch& sc, int mem_kind, const void* p, size_t bytes, const void** d) {
    return stage_in(sc, p, bytes, mem_kind, d);
}

int gc_model_forward(const gc_model* m, const float* theta, int64_t n, float* s_out,
                     const gc_exec* exec) {
    GC_GUARD_BEGIN
    clear_error();
    GC_REQUIRE(m && theta && s_out && n >= 0, GC_E_INVAL, "bad arguments");
    DeviceScope ds;
    int rc;
    if ((rc = ds.open(exec))) return rc;
    Scratch sc(ds.stream);
    AcqDev a;
    if ((rc = model_acq(m, ds.dev, &a))) return rc;
    const void* dth;
    if ((rc = stage_simple(sc, ds.mem_kind, theta, (size_t)n * m->P * 4, &dth))) return rc;
    float* dout = s_out;
    if (ds.mem_kind == GC_MEM_HOST) GC_TRY_HIP(sc.alloc_n(&dout, (size_t)std::max<int64_t>(n, 1) * m->Meff));
    GC_TRY_HIP(model_forward(m->kind, a, (const float*)dth, n, dout, ds.stream));
    if (ds.mem_kind == GC_MEM_HOST && n)
        GC_TRY_HIP(hipMemcpyAsync(s_out, dout, (size_t)n * m->Meff * 4, hipMemcpyDeviceToHost, ds.stream));
    GC_TRY_HIP(hipStreamSynchronize(ds.stream));
    return GC_OK;
    GC_GUARD_END
}

int gc_model_vjp(const gc_model* m, const float* theta, int64_t n, const float* ds_in,
                 float* dtheta, const gc_exec* exec) {
    GC_GUARD_BEGIN
    clear_error();
    GC_REQUIRE(m && theta && ds_in && dtheta && n >= 0, GC_E_INVAL, "bad arguments");
    DeviceScope ds;
    int rc;
    if ((rc = ds.open(exec))) return rc;
    Scratch sc(ds.stream);
    AcqDev a;
    if ((rc = model_acq(m, ds.dev, &a))) return rc;
    const void *dth, *dds;
    if ((rc = stage_simple(sc, ds.mem_kind, theta, (size_t)n * m->P * 4, &dth))) return rc;
    if ((rc = stage_simple(sc, ds.mem_kind, ds_in, (size_t)n * m->Meff * 4, &dds))) return rc;
    float* dout = dtheta;
    if (ds.mem_kind == GC_MEM_HOST) GC_TRY_HIP(sc.alloc_n(&dout, (size_t)std::max<int64_t>(n, 1) * m->P));
    GC_TRY_HIP(model_vjp(m->kind, a, (const float*)dth, n, (const float*)dds, dout, ds.stream));
    if (ds.mem_kind == GC_MEM_HOST && n)
        GC_TRY_HIP(hipMemcpyAsync(dtheta, dout, (size_t)n * m->P * 4, hipMemcpyDeviceToHost, ds.stream));
    GC_TRY_HIP(hipStreamSynchronize(ds.stream));
    return GC_OK;
    GC_GUARD_END
}

int gc_loss_vjp(const gc_model* m, const float* theta, const float* y, const float* w, int64_t n,
                int p, double scale, float* loss, float* dtheta, const gc_exec* exec) {
    GC_GUARD_BEGIN
    clear_error();
    GC_REQUIRE(m && theta && y && dtheta && n >= 0 && (p == 1 || p == 2), GC_E_INVAL,
               "bad arguments");
    DeviceScope ds;
    int rc;
    if ((rc = ds.open(exec))) return rc;
    Scratch sc(ds.stream);
    AcqDev a;
    if ((rc = model_acq(m, ds.dev, &a))) return rc;
    const void *dth, *dy, *dw;
    if ((rc = stage_simple(sc, ds.mem_kind, theta, (size_t)n * m->P * 4, &dth))) return rc;
    if ((rc = stage_simple(sc, ds.mem_kind, y, (size_t)n * m->Meff * 4, &dy))) return rc;
    if ((rc = stage_simple(sc, ds.mem_kind, w, (size_t)n * 4, &dw))) return rc;
    float* dg = dtheta;
    float* dl = loss;
    if (ds.mem_kind == GC_MEM_HOST) {
        GC_TRY_HIP(sc.alloc_n(&dg, (size_t)std::max<int64_t>(n, 1) * m->P));
        if (loss) GC_TRY_HIP(sc.alloc_n(&dl, (size_t)std::max<int64_t>(n, 1)));
    }
    GC_TRY_HIP(loss_vjp(m->kind, a, (const float*)dth, (const float*)dy, (const float*)dw, n, p,
                        (float)scale, dl, dg, ds.stream));
    if (ds.mem_kind == GC_MEM_HOST && n) {
        GC_TRY_HIP(hipMemcpyAsync(dtheta, dg, (size_t)n * m->P * 4, hipMemcpyDeviceToHost, ds.stream));
        if (loss) GC_TRY_HIP(hipMemcpyAsync(loss, dl, (size_t)n * 4, hipMemcpyDeviceToHost, ds.stream));
    }
    GC_TRY_HIP(hipStreamSynchronize(ds.stream));
    return GC_OK;
    GC_GUARD_END
}

static int tv_entry(int kind, int nx, int ny, int nz, const uint8_t* mask, const float* u,
                    int tv_dim, double scale, double* R, float* dR, const gc_exec* exec) {
    GC_GUARD_BEGIN
    clear_error();
    GC_REQUIRE(nx >= 1 && ny >= 1 && nz >= 1 && u && R && (tv_dim == 2 || tv_dim == 3),
               GC_E_INVAL, "bad arguments");
    DeviceScope ds;
    int rc;
    if ((rc = ds.open(exec))) return rc;
    Scratch sc(ds.stream);
    const int64_t G = (int64_t)nx * ny * nz;
    const void *dm, *du;
    if ((rc = stage_simple(sc, ds.mem_kind, mask, (size_t)G, &dm))) return rc;
    if ((rc = stage_simple(sc, ds.mem_kind, u, (size_t)G * 4, &du))) return rc;
    float* dd = dR;
    if (dR && ds.mem_kind == GC_MEM_HOST) GC_TRY_HIP(sc.alloc_n(&dd, (size_t)G));
    const int64_t nblk = (G + kBlock - 1) / kBlock;
    double *part = nullptr, *dsum = nullptr;
    GC_TRY_HIP(sc.alloc_n(&part, (size_t)nblk));
    GC_TRY_HIP(sc.alloc_n(&dsum, 1));
    if (kind == GC_TV_ISO)
        GC_TRY_HIP(tv_grid_iso(nx, ny, nz, (const uint8_t*)dm, (const float*)du, tv_dim,
                               (float)scale, part, nblk, dd, ds.stream));
    else
        GC_TRY_HIP(tv_grid(nx, ny, nz, (const uint8_t*)dm, (const float*)du, tv_dim, (float)scale,
                           part, nblk, dd, ds.stream));
    GC_TRY_HIP(sum_partials_f64(part, nblk, dsum, ds.stream));
    GC_TRY_HIP(hipMemcpyAsync(R, dsum, sizeof(double), hipMemcpyDeviceToHost, ds.stream));
    if (dR && ds.mem_kind == GC_MEM_HOST)
        GC_TRY_HIP(hipMemcpyAsync(dR, dd, (size_t)G * 4, hipMemcpyDeviceToHost, ds.stream));
    GC_TRY_HIP(hipStreamSynchronize(ds.stream));
    return GC_OK;
    GC_GUARD_END
}

int gc_tv(int nx, int ny, int nz, const uint8_t* mask, const float* u, int tv_dim, double scale,
          double* R, float* dR, const gc_exec* exec) {
    return tv_entry(GC_TV_ANISO, nx, ny, nz, mask, u, tv_dim, scale, R, dR, exec);
}

int gc_tv_iso(int nx, int ny, int nz, const uint8_t* mask, const float* u, int tv_dim,
              double scale, double* R, float* dR, const gc_exec* exec) {
    return tv_entry(GC_TV_ISO, nx, ny, nz, mask, u, tv_dim, scale, R, dR, exec);
}

int gc_tv_graph(int64_t n, const int64_t* rowptr, const int32_t* col, int64_t nnz,
                const float* u, double scale, double* R, float* dR, const gc_exec* exec) {
    GC_GUARD_BEGIN
    clear_error();
    GC_REQUIRE(n >= 1 && nnz >= 0 && rowptr && u && R && (col || nnz == 0), GC_E_INVAL,
               "bad arguments");
    GC_REQUIRE(n < INT32_MAX, GC_E_INVAL, "graph too large (n >= 2^31)");
    DeviceScope ds;
    int rc;
    if ((rc = ds.open(exec))) return rc;
    Scratch sc(ds.stream);
    const void *drp, *dcol = nullptr, *du;
    if ((rc = stage_simple(sc, ds.mem_kind, rowptr, (size_t)(n + 1) * 8, &drp))) return rc;
    if (nnz > 0 && (rc = stage_simple(sc, ds.mem_kind, col, (size_t)nnz * 4, &dcol))) return rc;
    if ((rc = stage_simple(sc, ds.mem_kind, u, (size_t)n * 4, &du))) return rc;
    if ((rc = validate_graph(sc, n, nnz, (const int64_t*)drp, (const int32_t*)dcol, ds.stream)))
        return rc;
    float* dd = dR;
    if (dR && ds.mem_kind == GC_MEM_HOST) GC_TRY_HIP(sc.alloc_n(&dd, (size_t)n));
    const int64_t nblk = (n + kBlock - 1) / kBlock;
    double *part = nullptr, *dsum = nullptr;
    GC_TRY_HIP(sc.alloc_n(&part, (size_t)nblk));
    GC_TRY_HIP(sc.alloc_n(&dsum, 1));
    GC_TRY_HIP(tv_graph(n, (const int64_t*)drp, (const int32_t*)dcol, (const float*)du,
                        (float)scale, part, nblk, dd, ds.stream));
    GC_TRY_HIP(sum_partials_f64(part, nblk, dsum, ds.stream));
    GC_TRY_HIP(hipMemcpyAsync(R, dsum, sizeof(double), hipMemcpyDeviceToHost, ds.stream));
    if (dR && ds.mem_kind == GC_MEM_HOST)
        GC_TRY_HIP(hipMemcpyAsync(dR, dd, (size_t)n * 4, hipMemcpyDeviceToHost, ds.stream));
    GC_TRY_HIP(hipStreamSynchronize(ds.stream));
    return GC_OK;
    GC_GUARD_END
}

int gc_philox(uint64_t seed, const uint32_t* ctr, int64_t n, uint32_t* out, const gc_exec* exec) {
    GC_GUARD_BEGIN
    clear_error();
    GC_REQUIRE(ctr && out && n >= 0, GC_E_INVAL, "bad arguments");
    DeviceScope ds;
    int rc;
    if ((rc = ds.open(exec))) return rc;
    Scratch sc(ds.stream);
    const void* dc;
    if ((rc = stage_simple(sc, ds.mem_kind, ctr, (size_t)n * 16, &dc))) return rc;
    uint32_t* dout = out;
    if (ds.mem_kind == GC_MEM_HOST) GC_TRY_HIP(sc.alloc_n(&dout, (size_t)std::max<int64_t>(n, 1) * 4));
    GC_TRY_HIP(philox_batch(seed, (const uint32_t*)dc, n, dout, ds.stream));
    if (ds.mem_kind == GC_MEM_HOST && n)
        GC_TRY_HIP(hipMemcpyAsync(out, dout, (size_t)n * 16, hipMemcpyDeviceToHost, ds.stream));
    GC_TRY_HIP(hipStreamSynchronize(ds.stream));
    return GC_OK;
    GC_GUARD_END
}

int gc_philox_uniform_normal(uint64_t seed, const uint32_t* ctr, int64_t n, int precision,
                             void* out_u, void* out_z, const gc_exec* exec) {
    GC_GUARD_BEGIN
    clear_error();
    GC_REQUIRE(ctr && out_u && out_z && n >= 0 && (precision == 0 || precision == 1), GC_E_INVAL,
               "bad arguments");
    DeviceScope ds;
    int rc;
    if ((rc = ds.open(exec))) return rc;
    Scratch sc(ds.stream);
    const void* dc;
    if ((rc = stage_simple(sc, ds.mem_kind, ctr, (size_t)n * 16, &dc))) return rc;
    const size_t es = precision ? 8 : 4;
    void *du = out_u, *dz = out_z;
    if (ds.mem_kind == GC_MEM_HOST) {
        GC_TRY_HIP(sc.alloc(&du, (size_t)std::max<int64_t>(n, 1) * 4 * es));
        GC_TRY_HIP(sc.alloc(&dz, (size_t)std::max<int64_t>(n, 1) * 4 * es));
    }
    GC_TRY_HIP(philox_uniform_normal(seed, (const uint32_t*)dc, n, precision == 1, du, dz, ds.stream));
    if (ds.mem_kind == GC_MEM_HOST && n) {
        GC_TRY_HIP(hipMemcpyAsync(out_u, du, (size_t)n * 4 * es, hipMemcpyDeviceToHost, ds.stream));
        GC_TRY_HIP(hipMemcpyAsync(out_z, dz, (size_t)n * 4 * es, hipMemcpyDeviceToHost, ds.stream));
    }
    GC_TRY_HIP(hipStreamSynchronize(ds.stream));
    return GC_OK;
    GC_GUARD_END
}

}  // extern "C"

// ------------------------------------------------------------ reconstruction
namespace {

bool pow2_in(int n, int lo, int hi) { return n >= lo && n <= hi && (n & (n - 1)) == 0; }
int ilog2(int n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

// Validates the problem, stages its arrays, builds the mask bit words and
// sample offsets and the twiddle tables, and (need_k) packs the measured
// samples; fills the kernel descriptor.
int sense_setup(Scratch& sc, const gc_sense_problem* pr, int mem_kind, bool need_k, SenseDev* S) {
    GC_REQUIRE(pr, GC_E_INVAL, "problem missing");
    GC_REQUIRE(pow2_in(pr->ny, 2, kSenseMaxN) && pow2_in(pr->nz, kSenseMinNz, kSenseMaxN),
               GC_E_INVAL, "ny must be a power of two in 2..%d, nz in %d..%d", kSenseMaxN,
               kSenseMinNz, kSenseMaxN);
    GC_REQUIRE(pr->n_echo >= 1 && pr->n_echo <= 1024 && pr->n_coil >= 1 && pr->n_coil <= 1024 &&
                   pr->coils && pr->mask,
               GC_E_INVAL, "need 1 <= n_echo, n_coil <= 1024, coils and mask");
    GC_REQUIRE(!need_k || pr->kspace, GC_E_INVAL, "kspace missing");
    const int E = pr->n_echo, Nc = pr->n_coil, Ny = pr->ny, Nz = pr->nz;
    const size_t pix = (size_t)Ny * Nz;
    const hipStream_t s = sc.s;
    const void *dc, *dm;
    int rc;
    if ((rc = stage_in(sc, pr->coils, (size_t)Nc * pix * 8, mem_kind, &dc))) return rc;
    if ((rc = stage_in(sc, pr->mask, (size_t)E * pix, mem_kind, &dm))) return rc;
    // the mask is small: per-tile row masks and sample offsets on the host
    std::vector<uint8_t> hm((size_t)E * pix);
    GC_TRY_HIP(hipMemcpyAsync(hm.data(), dm, hm.size(), hipMemcpyDeviceToHost, s));
    GC_TRY_HIP(hipStreamSynchronize(s));
    const int logNy = ilog2(Ny), G = sense_tile_cols(logNy), nzg = Nz / G;
    std::vector<uint32_t> tinfo((size_t)E * nzg * Ny, 0u);
    std::vector<int32_t> tbase((size_t)E * nzg, 0);
    int64_t cnt = 0;
    for (int e = 0; e < E; ++e) {
        for (int zg = 0; zg < nzg; ++zg) {
            GC_REQUIRE(cnt < INT32_MAX - 4096, GC_E_INVAL, "too many sampled entries");
            tbase[(size_t)e * nzg + zg] = (int32_t)cnt;
            uint32_t local = 0;
            for (int y = 0; y < Ny; ++y) {
                uint32_t m16 = 0;
                for (int j = 0; j < G; ++j)
                    if (hm[((size_t)e * Ny + y) * Nz + (size_t)zg * G + j]) m16 |= 1u << j;
                tinfo[((size_t)e * nzg + zg) * Ny + y] = (local << 16) | m16;
                local += (uint32_t)__builtin_popcount(m16);
            }
            cnt += local;
        }
    }
    // twiddles exp(-2 pi i k / N), k < N, in FP64 then rounded once
    std::vector<float> tw((size_t)(Ny + Nz) * 2);
    for (int k = 0; k < Ny; ++k) {
        const double a = -2.0 * M_PI * k / Ny;
        tw[2 * k] = (float)std::cos(a);
        tw[2 * k + 1] = (float)std::sin(a);
    }
    for (int k = 0; k < Nz; ++k) {
        const double a = -2.0 * M_PI * k / Nz;
        tw[2 * (Ny + k)] = (float)std::cos(a);
        tw[2 * (Ny + k) + 1] = (float)std::sin(a);
    }
    float* dtw = nullptr;
    uint32_t* dti = nullptr;
    int32_t* dtb = nullptr;
    GC_TRY_HIP(sc.alloc_n(&dtw, tw.size()));
    GC_TRY_HIP(sc.alloc_n(&dti, tinfo.size()));
    GC_TRY_HIP(sc.alloc_n(&dtb, tbase.size()));
    GC_TRY_HIP(hipMemcpyAsync(dtw, tw.data(), tw.size() * sizeof(float), hipMemcpyHostToDevice, s));
    GC_TRY_HIP(hipMemcpyAsync(dti, tinfo.data(), tinfo.size() * sizeof(uint32_t),
                              hipMemcpyHostToDevice, s));
    GC_TRY_HIP(hipMemcpyAsync(dtb, tbase.data(), tbase.size() * sizeof(int32_t),
                              hipMemcpyHostToDevice, s));
    SenseDev& D = *S;
    D = SenseDev{};
    D.E = E;
    D.Nc = Nc;
    D.Ny = Ny;
    D.Nz = Nz;
    D.logNy = logNy;
    D.logNz = ilog2(Nz);
    D.G = G;
    D.S = cnt;
    D.rsqrtNy = (float)(1.0 / std::sqrt((double)Ny));
    D.rsqrtNz = (float)(1.0 / std::sqrt((double)Nz));
    D.coils = (const float2*)dc;
    D.tinfo = dti;
    D.tbase = dtb;
    D.twy = (const float2*)dtw;
    D.twz = (const float2*)(dtw + 2 * Ny);
    D.scale_data = cnt > 0 ? (float)(1.0 / (2.0 * Nc * (double)cnt)) : 0.f;
    if (need_k && cnt > 0) {
        const void* dk;
        if ((rc = stage_in(sc, pr->kspace, (size_t)E * Nc * pix * 8, mem_kind, &dk))) return rc;
        float2* kc = nullptr;
        GC_TRY_HIP(sc.alloc_n(&kc, (size_t)Nc * cnt));
        GC_TRY_HIP(sense_pack_kspace(D, (const float2*)dk, kc, s));
        D.kc = kc;
    }
    return GC_OK;
}

}  // namespace

int gc_sense_recon(const gc_sense_problem* pr, const gc_adam_hyper* h, float* out_image,
                   gc_fit_report* report, const gc_exec* exec) {
    GC_GUARD_BEGIN
    clear_error();
    int rc;
    GC_REQUIRE(h && out_image, GC_E_INVAL, "null hyper or output");
    GC_REQUIRE(h->n_iter >= 1 && (h->loss == 1 || h->loss == 2) && h->optimizer >= 0 &&
                   h->optimizer <= 2 && h->lr > 0 && std::isfinite(h->lr) && h->lambda >= 0 &&
                   h->beta1 >= 0 && h->beta1 < 1 && h->beta2 >= 0 && h->beta2 < 1 &&
                   h->eps >= 0 && h->rho >= 0 && h->rho < 1 && h->momentum >= 0,
               GC_E_INVAL, "bad optimiser hyper-parameters");
    GC_REQUIRE(!(h->conv_value > 0) || h->conv_window > 1, GC_E_INVAL, "conv_window must be > 1");
    DeviceScope ds;
    if ((rc = ds.open(exec))) return rc;
    const hipStream_t s = ds.stream;
    Scratch sc(s);
    SenseDev S;
    if ((rc = sense_setup(sc, pr, ds.mem_kind, true, &S))) return rc;
    GC_REQUIRE(S.S > 0, GC_E_INVAL, "the mask samples nothing");
    S.loss_p = h->loss;
    const int T = h->n_iter;
    const int64_t npix = (int64_t)S.E * S.Ny * S.Nz;
    const size_t nbuf = (size_t)S.E * S.Nc * S.Ny * S.Nz;
    float2 *img0 = nullptr, *img1 = nullptr, *m = nullptr, *v = nullptr, *buf = nullptr;
    GC_TRY_HIP(sc.alloc_n(&img0, (size_t)npix));
    GC_TRY_HIP(sc.alloc_n(&img1, (size_t)npix));
    GC_TRY_HIP(sc.alloc_n(&m, (size_t)npix));
    GC_TRY_HIP(sc.alloc_n(&v, (size_t)npix));
    GC_TRY_HIP(sc.alloc_n(&buf, nbuf));
    GC_TRY_HIP(fill_f32((float*)m, npix * 2, 0.f, s));
    GC_TRY_HIP(fill_f32((float*)v, npix * 2, 0.f, s));
    if (pr->init) {
        const void* di;
        if ((rc = stage_in(sc, pr->init, (size_t)npix * 8, ds.mem_kind, &di))) return rc;
        GC_TRY_HIP(hipMemcpyAsync(img0, di, (size_t)npix * 8, hipMemcpyDeviceToDevice, s));
    } else {
        GC_TRY_HIP(fill_f32((float*)img0, npix * 2, 0.f, s));
    }
    const int64_t nparts = sense_partials(S);
    float* partial = nullptr;
    double* hist = nullptr;
    int* stop = nullptr;
    GC_TRY_HIP(sc.alloc_n(&partial, (size_t)nparts));
    GC_TRY_HIP(sc.alloc_n(&hist, (size_t)T));
    GC_TRY_HIP(sc.alloc_n(&stop, 2));
    GC_TRY_HIP(fill_i32(stop, 2, 0, s));
    SenseOpt O{};
    O.optimizer = h->optimizer;
    O.lr = (float)h->lr;
    O.beta1 = (float)h->beta1;
    O.beta2 = (float)h->beta2;
    O.eps = (float)h->eps;
    O.momentum = (float)h->momentum;
    O.rho = (float)h->rho;
    O.omb1 = (float)(1.0 - h->beta1);
    O.omb2 = (float)(1.0 - h->beta2);
    O.omrho = (float)(1.0 - h->rho);
    O.scale_tv = (float)(h->lambda / (double)npix);
    const bool stopping = h->tol > 0 || h->conv_value > 0;
    const bool each = stopping || h->loss_history != nullptr;
    const double tol = h->tol > 0 ? h->tol : -INFINITY;
    double b1 = 1.0, b2 = 1.0;
    int hstop[2] = {0, 0};
    LaunchTimer tm[kSenseStages] = {{"sense_ycols", s}, {"sense_zrows", s}};
    GC_TRY_HIP(sense_forward_rows(S, img0, buf, s));
    for (int t = 1; t <= T; ++t) {
        b1 *= h->beta1;
        b2 *= h->beta2;
        O.c1 = (float)(1.0 / (1.0 - b1));
        O.c2 = (float)(1.0 / (1.0 - b2));
        const bool rec = each || t == T;
        const float2* in = (t % 2 == 1) ? img0 : img1;
        float2* out = (t % 2 == 1) ? img1 : img0;
        for (int k = 0; k < kSenseStages; ++k) {
            tm[k].begin();
            GC_TRY_HIP(sense_stage(k, S, O, in, out, m, v, buf, rec ? partial : nullptr,
                                   stopping ? stop : nullptr, t < T ? 1 : 0, s));
            tm[k].end();
        }
        if (rec)
            GC_TRY_HIP(fit_loss_stop(partial, nparts, hist, t, tol, h->conv_value, h->conv_window,
                                     stop, s));
        if (stopping && t % 32 == 0 && t < T) {
            GC_TRY_HIP(hipMemcpyAsync(hstop, stop, sizeof(hstop), hipMemcpyDeviceToHost, s));
            GC_TRY_HIP(hipStreamSynchronize(s));
            if (hstop[0] != 0) break;
        }
    }
    GC_TRY_HIP(hipMemcpyAsync(hstop, stop, sizeof(hstop), hipMemcpyDeviceToHost, s));
    GC_TRY_HIP(hipStreamSynchronize(s));
    for (auto& x : tm) x.flush();
    const int iters = hstop[0] != 0 ? hstop[0] : T;
    double final_loss = 0.0;
    GC_TRY_HIP(hipMemcpyAsync(&final_loss, hist + (iters - 1), sizeof(double),
                              hipMemcpyDeviceToHost, s));
    if (h->loss_history)
        GC_TRY_HIP(hipMemcpyAsync(h->loss_history, hist, (size_t)iters * sizeof(double),
                                  hipMemcpyDeviceToHost, s));
    const float2* fin = (iters % 2 == 1) ? img1 : img0;
    GC_TRY_HIP(hipMemcpyAsync(out_image, fin, (size_t)npix * 8,
                              ds.mem_kind == GC_MEM_HOST ? hipMemcpyDeviceToHost
                                                         : hipMemcpyDeviceToDevice, s));
    GC_TRY_HIP(hipStreamSynchronize(s));
    if (report) {
        report->iters_run = iters;
        report->final_loss = final_loss;
        report->stop_reason = hstop[0] != 0 ? hstop[1] : 0;
    }
    return GC_OK;
    GC_GUARD_END
}

int gc_sense_forward(const gc_sense_problem* pr, const float* image, float* out,
                     const gc_exec* exec) {
    GC_GUARD_BEGIN
    clear_error();
    int rc;
    GC_REQUIRE(image && out, GC_E_INVAL, "null image or output");
    DeviceScope ds;
    if ((rc = ds.open(exec))) return rc;
    Scratch sc(ds.stream);
    SenseDev S;
    if ((rc = sense_setup(sc, pr, ds.mem_kind, false, &S))) return rc;
    const int64_t npix = (int64_t)S.E * S.Ny * S.Nz;
    const size_t nbuf = (size_t)S.E * S.Nc * S.Ny * S.Nz;
    const void* di;
    if ((rc = stage_in(sc, image, (size_t)npix * 8, ds.mem_kind, &di))) return rc;
    float2* buf = nullptr;
    GC_TRY_HIP(sc.alloc_n(&buf, nbuf));
    float2* dout = (float2*)out;
    if (ds.mem_kind == GC_MEM_HOST) GC_TRY_HIP(sc.alloc_n(&dout, nbuf));
    GC_TRY_HIP(sense_forward_op(S, (const float2*)di, buf, dout, ds.stream));
    if (ds.mem_kind == GC_MEM_HOST)
        GC_TRY_HIP(hipMemcpyAsync(out, dout, nbuf * 8, hipMemcpyDeviceToHost, ds.stream));
    GC_TRY_HIP(hipStreamSynchronize(ds.stream));
    return GC_OK;
    GC_GUARD_END
}

int gc_sense_adjoint(const gc_sense_problem* pr, const float* kspace, float* out,
                     const gc_exec* exec) {
    GC_GUARD_BEGIN
    clear_error();
    int rc;
    GC_REQUIRE(kspace && out, GC_E_INVAL, "null input or output");
    DeviceScope ds;
    if ((rc = ds.open(exec))) return rc;
    Scratch sc(ds.stream);
    SenseDev S;
    if ((rc = sense_setup(sc, pr, ds.mem_kind, false, &S))) return rc;
    const int64_t npix = (int64_t)S.E * S.Ny * S.Nz;
    const size_t nbuf = (size_t)S.E * S.Nc * S.Ny * S.Nz;
    const void* dk;
    if ((rc = stage_in(sc, kspace, nbuf * 8, ds.mem_kind, &dk))) return rc;
    float2* buf = nullptr;
    GC_TRY_HIP(sc.alloc_n(&buf, nbuf));
    float2* dout = (float2*)out;
    if (ds.mem_kind == GC_MEM_HOST) GC_TRY_HIP(sc.alloc_n(&dout, (size_t)npix));
    GC_TRY_HIP(sense_adjoint_op(S, (const float2*)dk, buf, dout, ds.stream));
    if (ds.mem_kind == GC_MEM_HOST)
        GC_TRY_HIP(hipMemcpyAsync(out, dout, (size_t)npix * 8, hipMemcpyDeviceToHost, ds.stream));
    GC_TRY_HIP(hipStreamSynchronize(ds.stream));
    return GC_OK;
    GC_GUARD_END
}
