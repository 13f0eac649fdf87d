// Continuous-batching server for fit and MCMC jobs (gc_server_* in gacelle.h).
//
// A scheduler thread owns three streams:
//   prep    -- staging, compaction and state initialisation of admitted jobs;
//   compute -- the shared launches: every round advances all resident jobs
//              by one chunk, one launch per (kernel, model, precision) group
//              whose block work-list concatenates the jobs' lanes;
//   copy    -- moment merges, scatters and result copies of finished jobs.
// Jobs are admitted in arrival order while a slot is free and their device
// footprint fits the HBM budget; they join at the next round boundary, and
// their memory and slot are released as soon as their results are on the
// host.  Each job keeps its own seed, descriptors and loss partials, so its
// arithmetic is exactly that of the synchronous call: results are the same
// alone and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <thread>
#include <unordered_map>

#include "gc_runtime.hpp"
#include "gc_timing.hpp"

namespace gc {

namespace {

// Pinned host staging memory, reused across jobs and rounds.
struct PinnedPool {
    std::mutex mu;
    std::multimap<size_t, void*> free_;
    std::vector<void*> all;
    void* get(size_t bytes) {
        std::lock_guard<std::mutex> lk(mu);
        auto it = free_.lower_bound(bytes);
        if (it != free_.end() && it->first <= 2 * bytes + (1 << 20)) {
            void* p = it->second;
            free_.erase(it);
            return p;
        }
        void* p = nullptr;
        size_t sz = std::max<size_t>(bytes, 4096);
        if (hipHostMalloc(&p, sz, hipHostMallocDefault) != hipSuccess) return nullptr;
        sizes[p] = sz;
        all.push_back(p);
        return p;
    }
    void put(void* p) {
        if (!p) return;
        std::lock_guard<std::mutex> lk(mu);
        free_.emplace(sizes[p], p);
    }
    std::unordered_map<void*, size_t> sizes;
    ~PinnedPool() {
        for (void* p : all) (void)hipHostFree(p);
    }
};

// Default admission: 64 resident jobs, or more (up to kMaxSlotsSmall) while
// the resident jobs hold fewer than kFillLanes lanes (voxel x chain pairs),
// about four rounds of waves of the whole GPU.
constexpr int kMaxSlotsSmall = 256;
constexpr int64_t kFillLanes = int64_t(1) << 21;

struct Job {
    uint64_t id = 0;
    gc_job spec{};
    std::vector<double> lb, ub, x0, step;   // owned copies of descriptor arrays
    int state = GC_JOB_QUEUED;
    int status = GC_OK;
    int fail_status = GC_OK;   // set when a shared launch failed for this job
    std::string err;
    bool cancel = false;
    double t_submit = 0, t_done = 0;
    size_t footprint = 0;
    int64_t lanes = 0;   // masked voxels x chains (walkers; 1 for a fit)
    int64_t G = 0, n = 0;
    // device residency
    std::unique_ptr<Scratch> mem;
    Packed pk;
    AcqDev acq{};
    int kind = 0, maxm = 0;
    bool fp64 = false, ens = false;
    // MCMC
    MhJob mh{};
    int C = 0;
    double* mean_c = nullptr;
    double* std_c = nullptr;
    // fit
    FitJob fit{};
    bool step_path = false;
    bool loss_each = false;   // stopping rules need the loss of every iteration
    float *u0 = nullptr, *u1 = nullptr, *theta_c = nullptr, *lossv = nullptr, *partial = nullptr;
    double* hist = nullptr;
    int* stop = nullptr;
    double b1 = 1.0, b2 = 1.0;   // beta^t after the iterations enqueued so far
    int64_t nblk = 0;
    // progress
    int t_next = 0;        // next iteration (MCMC: 0-based; fit: 1-based count done)
    int t_total = 0;
    int last_round = -1;   // round in which the job's last work was enqueued
    bool finishing = false;
    hipEvent_t ready = nullptr, done = nullptr;
    void* pin_out = nullptr;   // pinned result staging
    void* pin_aux = nullptr;   // pinned descriptor staging of the finalisation
    char* dout = nullptr;      // device result staging (arena)
    void* dj = nullptr;        // device descriptors of the finalisation (arena)
    int stage = 0;             // per-iteration fits: 1 = stop flag copied, 2 = maps copied
    size_t out_bytes = 0;
    int iters_run = 0, stop_reason = 0;
    double final_loss = 0.0;
    double voxel_iters = 0.0;
};

}  // namespace

}  // namespace gc

struct gc_server {
    gc_server_cfg cfg{};
    std::mutex mu;
    std::condition_variable cv;      // job state changes
    std::condition_variable wake;    // scheduler wake-up
    std::thread thr;
    bool stopping = false;
    uint64_t next_id = 1;
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, std::unique_ptr<gc::Job>> jobs;
    std::vector<gc::Job*> resident;
    size_t used = 0;
    int64_t resident_lanes = 0;   // lanes of the resident jobs
    int peak_resident = 0;
    hipStream_t prep = nullptr, compute = nullptr, copy = nullptr;
    // launch lanes of a round (batched mode): the groups of a round run on
    // these streams side by side, fenced by `lane_start` (after the round's
    // descriptor upload on `compute`) and `lane_end` (joined back into
    // `compute` before the round's completion event)
    static constexpr int kLanes = 8;
    hipStream_t lane[kLanes] = {};
    hipEvent_t lane_start = nullptr;
    hipEvent_t lane_end[kLanes] = {};
    gc::PinnedPool pinned;
    gc::DevArena arena;              // all device memory of resident jobs and rounds
    // statistics
    uint64_t n_sub = 0, n_done = 0, n_fail = 0, n_cancel = 0;
    double voxel_iters = 0.0, busy = 0.0, busy_since = -1.0;
    std::vector<double> latencies;
};

namespace gc {

namespace {

// iterations per round of per-iteration (TV / stopping-rule) fits: 25 when
// every launch of a round shares one stream; with launch lanes the steps run
// beside the round's other groups, and a fifth of the MCMC chunk keeps them
// from needing many more rounds than the chains they share the GPU with
constexpr int kFitStepRound = 25;

size_t footprint_of(const gc_model* m, const gc_job& j, int64_t G, int64_t n) {
    size_t b = (size_t)G * m->Meff * 4 + (size_t)G * 9 + (size_t)n * m->Meff * 4 +
               (size_t)G * 8 + (size_t)(G / kTile + 2) * 12;
    if (j.data.y && j.mcmc.weights) b += (size_t)G * 4 + (size_t)n * 4;
    if (j.kind == GC_JOB_MCMC) {
        const int C = j.mcmc.sampler == GC_SAMPLER_ENSEMBLE ? j.mcmc.n_walkers : j.n_chains;
        const size_t rs = j.mcmc.precision == GC_PREC_FP64 ? 8 : 4;
        b += (size_t)n * C * (m->P * rs + rs + 4 + 2 * m->P * 8);
        b += (size_t)n * m->P * 16 + (size_t)G * m->P * 16 + (size_t)G * C * 4;
    } else {
        b += (size_t)n * m->P * 4 * 5 + (size_t)n * 24 + (size_t)G * m->P * 4;
        const bool each = j.adam.tol > 0 || j.adam.conv_value > 0;
        if (j.adam.prior_lambda > 0 && j.adam.prior_mask)
            b += (size_t)(G + n) * m->P * 8;   // staged and gathered prior maps
        if (j.adam.lambda > 0 && j.adam.tv_mask && j.adam.tv_kind == GC_TV_GRAPH)
            b += (size_t)(n + 1) * 8 + (size_t)std::max<int64_t>(j.adam.graph_nnz, 0) * 4;
        b += (size_t)((n + kBlock - 1) / kBlock) * (each ? j.adam.n_iter : 1) * 4 +
             (size_t)j.adam.n_iter * 8;
    }
    return b + (1 << 20);
}

int64_t count_mask_host(const uint8_t* mask, int64_t G) {
    if (!mask) return G;
    int64_t c = 0;
    for (int64_t i = 0; i < G; ++i) c += mask[i] ? 1 : 0;
    return c;
}

}  // namespace

// Stage, compact and initialise one admitted job on the prep stream.
static int prepare_job(gc_server* S, Job* J) {
    const gc_model* m = J->spec.model;
    J->mem.reset(new Scratch(S->prep, &S->arena));
    Scratch& sc = *J->mem;
    int rc;
    if ((rc = model_acq(m, S->cfg.device, &J->acq))) return rc;
    J->kind = m->kind;
    const bool mcmc = J->spec.kind == GC_JOB_MCMC;
    const float* w = mcmc ? J->spec.mcmc.weights : J->spec.adam.weights;
    const float* x0map = J->spec.bounds.x0_map;
    if (mcmc && J->spec.mcmc.x0_mode != GC_X0_GIVEN) x0map = nullptr;
    if ((rc = pack_problem(sc, m, &J->spec.data, J->spec.mask, w, x0map, GC_MEM_HOST, &J->pk)))
        return rc;
    J->n = J->pk.n;
    const int64_t n = J->n;
    const int P = m->P;
    gc_bounds b{J->lb.data(), J->ub.data(), J->x0.empty() ? nullptr : J->x0.data(), nullptr};
    if (mcmc) {
        const gc_mcmc_hyper& h = J->spec.mcmc;
        J->ens = h.sampler == GC_SAMPLER_ENSEMBLE;
        J->fp64 = h.precision == GC_PREC_FP64;
        J->C = J->ens ? h.n_walkers : J->spec.n_chains;
        gc_mcmc_hyper hh = h;
        hh.step = J->step.empty() ? nullptr : J->step.data();
        if ((rc = fill_mh_job(m, &b, &hh, J->C, J->spec.n_iter, J->spec.burnin, J->spec.thin,
                              J->acq, &J->mh)))
            return rc;
        MhJob& q = J->mh;
        q.y = J->pk.y;
        q.w = J->pk.w;
        q.x0map = J->pk.x0;
        q.n = n;
        const size_t rs = J->fp64 ? 8 : 4;
        const size_t NL = (size_t)std::max<int64_t>(n * J->C, 1);
        GC_TRY_HIP(sc.alloc(&q.th, NL * P * rs));
        GC_TRY_HIP(sc.alloc(&q.ll, NL * rs));
        GC_TRY_HIP(sc.alloc_n(&q.acc, NL));
        GC_TRY_HIP(sc.alloc_n(&q.mean, NL * P));
        GC_TRY_HIP(sc.alloc_n(&q.m2, NL * P));
        GC_TRY_HIP(sc.alloc_n(&J->mean_c, (size_t)std::max<int64_t>(n, 1) * P));
        GC_TRY_HIP(sc.alloc_n(&J->std_c, (size_t)std::max<int64_t>(n, 1) * P));
        J->t_total = J->spec.n_iter;
        J->maxm = mh_pick_variant(m->kind, m->M, m->uniform ? 1 : 0);
        if (n > 0) {
            const int64_t nb = (n * J->C + kBlock - 1) / kBlock;
            std::vector<BlkMap> mp((size_t)nb);
            for (int64_t i = 0; i < nb; ++i) mp[i] = BlkMap{0, 0, i * kBlock};
            BlkMap* dmap = nullptr;
            MhJob* dj = nullptr;
            GC_TRY_HIP(sc.alloc_n(&dmap, mp.size()));
            GC_TRY_HIP(sc.alloc_n(&dj, 1));
            GC_TRY_HIP(hipMemcpyAsync(dmap, mp.data(), mp.size() * sizeof(BlkMap), hipMemcpyHostToDevice, S->prep));
            GC_TRY_HIP(hipMemcpyAsync(dj, &q, sizeof(MhJob), hipMemcpyHostToDevice, S->prep));
            if (J->ens) GC_TRY_HIP(ens_init(m->kind, J->fp64, dj, dmap, (int)nb, S->prep));
            else GC_TRY_HIP(mh_init(m->kind, J->fp64, dj, dmap, (int)nb, S->prep));
            GC_TRY_HIP(hipStreamSynchronize(S->prep));   // host vectors above go out of scope
        }
        J->voxel_iters = (double)n * J->C * J->spec.n_iter;
    } else {
        const gc_adam_hyper& h = J->spec.adam;
        if ((rc = fill_fit_job(m, &b, &h, n, J->acq, &J->fit))) return rc;
        FitJob& q = J->fit;
        q.y = J->pk.y;
        q.w = J->pk.w;
        q.x0map = J->pk.x0;
        float *pmu = nullptr, *psg = nullptr;
        if ((rc = pack_prior(sc, m, &h, J->pk, GC_MEM_HOST, &pmu, &psg))) return rc;
        q.mu = pmu;
        q.sigma = psg;
        if ((rc = pack_graph(sc, &h, n, GC_MEM_HOST, &q))) return rc;
        const size_t np = (size_t)std::max<int64_t>(n, 1) * P;
        GC_TRY_HIP(sc.alloc_n(&J->u0, np));
        GC_TRY_HIP(sc.alloc_n(&J->u1, np));
        GC_TRY_HIP(sc.alloc_n(&q.m, np));
        GC_TRY_HIP(sc.alloc_n(&q.v, np));
        GC_TRY_HIP(sc.alloc_n(&J->theta_c, np));
        q.u = J->u0;
        J->nblk = (n + kBlock - 1) / kBlock;
        J->step_path = q.tv_mask != 0 || h.tol > 0 || h.conv_value > 0;
        J->t_total = h.n_iter;
        J->t_next = 0;
        J->maxm = fit_pick_maxm(m->kind, m->M);
        if (J->step_path) {
            int32_t* nbr = nullptr;
            if (q.tv_mask && q.tv_kind != GC_TV_GRAPH) {
                GC_TRY_HIP(sc.alloc_n(&nbr, (size_t)std::max<int64_t>(n, 1) * 6));
                GC_TRY_HIP(build_neighbours(J->pk.c2g, J->pk.g2c, n, J->spec.data.nx, J->spec.data.ny,
                                            J->spec.data.nz, h.tv_dim, nbr, S->prep));
            }
            q.nbr = nbr;
            J->loss_each = h.tol > 0 || h.conv_value > 0;
            GC_TRY_HIP(sc.alloc_n(&J->partial, (size_t)std::max<int64_t>(J->nblk, 1) *
                                                   (J->loss_each ? h.n_iter : 1)));
            GC_TRY_HIP(sc.alloc_n(&J->hist, (size_t)h.n_iter));
            GC_TRY_HIP(sc.alloc_n(&J->stop, 2));
            GC_TRY_HIP(fill_i32(J->stop, 2, 0, S->prep));
            q.stop = J->stop;
        } else {
            GC_TRY_HIP(sc.alloc_n(&J->lossv, (size_t)std::max<int64_t>(n, 1)));
            q.loss_v = J->lossv;
            q.t_rec = h.n_iter;
        }
        if (n > 0) {
            std::vector<BlkMap> mp((size_t)J->nblk);
            for (int64_t i = 0; i < J->nblk; ++i) mp[i] = BlkMap{0, 0, i * kBlock};
            BlkMap* dmap = nullptr;
            FitJob* dj = nullptr;
            GC_TRY_HIP(sc.alloc_n(&dmap, mp.size()));
            GC_TRY_HIP(sc.alloc_n(&dj, 1));
            GC_TRY_HIP(hipMemcpyAsync(dmap, mp.data(), mp.size() * sizeof(BlkMap), hipMemcpyHostToDevice, S->prep));
            GC_TRY_HIP(hipMemcpyAsync(dj, &q, sizeof(FitJob), hipMemcpyHostToDevice, S->prep));
            GC_TRY_HIP(fit_init(dj, dmap, (int)J->nblk, S->prep));
            GC_TRY_HIP(hipStreamSynchronize(S->prep));
        }
        J->voxel_iters = (double)n * h.n_iter;
    }
    GC_TRY_HIP(hipEventCreateWithFlags(&J->ready, hipEventDisableTiming));
    GC_TRY_HIP(hipEventCreateWithFlags(&J->done, hipEventDisableTiming));
    GC_TRY_HIP(hipEventRecord(J->ready, S->prep));
    return GC_OK;
}

// One group of same-kernel work in a round: descriptors + block work-list.
struct Group {
    int kernel;   // 0 mh_chunk, 1 fit_fused, 2 ens_chunk, 3 fit_step
    int kind, maxm, walkers;   // walkers: ensemble walkers, or the shared chain count (mh_chunk)
    bool fp64;
    std::vector<MhJob> mh;
    std::vector<FitJob> fit;
    std::vector<BlkMap> map;
    std::vector<Job*> owners;   // owner job per descriptor
    std::vector<int> iter;      // fit_step: iteration of each descriptor (1-based)
    int meff = 0;               // mh_chunk / ens_chunk: largest effective measurement count
};

// Host-side check of a round before anything of it is enqueued: every row of
// a group's work-list names one of the group's descriptors and a lane range
// inside that job, and every array a descriptor points to lies inside a live
// block of the server's arena, large enough for what the kernels index.  A
// failure ends the round with an error instead of a launch that could touch
// memory outside its job.
static int check_arr(gc_server* S, const Job* J, const void* p, size_t bytes, const char* what) {
    if (bytes == 0) return GC_OK;
    if (p && S->arena.owns(p, bytes)) return GC_OK;
    set_error("job %llu: %s (%zu bytes at %p) is not inside a live block of the server's memory",
              (unsigned long long)J->id, what, bytes, p);
    return GC_E_DEVICE;
}

static int check_group(gc_server* S, const Group& g) {
    int rc;
#define GC_CHECK_ARR(p, b, w) \
    if ((rc = check_arr(S, J, (p), (b), (w)))) return rc
    const size_t nd = g.kernel == 0 || g.kernel == 2 ? g.mh.size() : g.fit.size();
    GC_REQUIRE(g.owners.size() == nd, GC_E_DEVICE, "round: %zu descriptors, %zu owners", nd,
               g.owners.size());
    for (size_t k = 0; k < nd; ++k) {
        const Job* J = g.owners[k];
        const int Meff = J->spec.model->Meff;
        if (g.kernel == 0 || g.kernel == 2) {
            const MhJob& q = g.mh[k];
            const int64_t n = q.n, NL = n * (int64_t)q.C;
            const size_t rs = g.fp64 ? 8 : 4, P = (size_t)q.P;
            GC_REQUIRE(n == J->n && q.C == J->C && q.P == J->spec.model->P, GC_E_DEVICE,
                       "job %llu: descriptor sizes differ from the job's", (unsigned long long)J->id);
            GC_REQUIRE(g.walkers == 0 || q.C == g.walkers, GC_E_DEVICE,
                       "job %llu: %d chains in a launch for %d", (unsigned long long)J->id, q.C,
                       g.walkers);
            GC_REQUIRE(q.samples == nullptr && q.init_state == nullptr, GC_E_DEVICE,
                       "job %llu: server jobs keep no samples and start fresh",
                       (unsigned long long)J->id);
            GC_CHECK_ARR(q.th, P * NL * rs, "chain states");
            GC_CHECK_ARR(q.ll, NL * rs, "log-likelihoods");
            GC_CHECK_ARR(q.acc, NL * 4, "accept counts");
            GC_CHECK_ARR(q.mean, P * NL * 8, "Welford means");
            GC_CHECK_ARR(q.m2, P * NL * 8, "Welford M2");
            GC_CHECK_ARR(q.y, (size_t)Meff * n * 4, "data");
            if (q.w) GC_CHECK_ARR(q.w, n * 4, "weights");
            if (q.x0map) GC_CHECK_ARR(q.x0map, P * n * 4, "start map");
        } else {
            const FitJob& q = g.fit[k];
            const int64_t n = q.n;
            const size_t P = (size_t)q.P, np = P * n * 4;
            GC_REQUIRE(n == J->n && q.P == J->spec.model->P, GC_E_DEVICE,
                       "job %llu: descriptor sizes differ from the job's", (unsigned long long)J->id);
            GC_CHECK_ARR(q.y, (size_t)Meff * n * 4, "data");
            if (q.w) GC_CHECK_ARR(q.w, n * 4, "weights");
            if (q.x0map) GC_CHECK_ARR(q.x0map, np, "start map");
            GC_CHECK_ARR(q.m, np, "first moments");
            GC_CHECK_ARR(q.v, np, "second moments");
            if (q.prior_mask) {
                GC_CHECK_ARR(q.mu, np, "prior means");
                GC_CHECK_ARR(q.sigma, np, "prior SDs");
            }
            if (g.kernel == 1) {
                GC_CHECK_ARR(q.u, np, "iterate");
                if (q.loss_v) GC_CHECK_ARR(q.loss_v, n * 4, "per-voxel losses");
            } else {
                GC_CHECK_ARR(q.u_in, np, "iterate (read)");
                GC_CHECK_ARR(q.u_out, np, "iterate (written)");
                GC_CHECK_ARR(q.stop, 8, "stop flags");
                if (q.tv_mask && q.tv_kind != GC_TV_GRAPH) GC_CHECK_ARR(q.nbr, 6 * n * 4, "neighbours");
                if (q.tv_mask && q.tv_kind == GC_TV_GRAPH) {
                    GC_CHECK_ARR(q.g_rowptr, (n + 1) * 8, "graph offsets");
                    if (J->spec.adam.graph_nnz > 0)
                        GC_CHECK_ARR(q.g_col, (size_t)J->spec.adam.graph_nnz * 4, "graph columns");
                }
                if (q.record) GC_CHECK_ARR(q.partial, (size_t)J->nblk * 4, "loss partials");
            }
        }
    }
#undef GC_CHECK_ARR
    // work-list rows
    for (size_t r = 0; r < g.map.size(); ++r) {
        const BlkMap& b = g.map[r];
        GC_REQUIRE(b.job >= 0 && (size_t)b.job < nd, GC_E_DEVICE,
                   "round: work-list row %zu names descriptor %d of %zu", r, b.job, nd);
        const Job* J = g.owners[b.job];
        int64_t lanes;
        if (g.kernel == 0) lanes = g.mh[b.job].n * g.mh[b.job].C;
        else if (g.kernel == 2) lanes = g.mh[b.job].n;          // rows cover voxel groups
        else lanes = g.fit[b.job].n;
        GC_REQUIRE(b.lane0 >= 0 && b.lane0 < lanes, GC_E_DEVICE,
                   "job %llu: work-list row %zu starts at lane %lld of %lld",
                   (unsigned long long)J->id, r, (long long)b.lane0, (long long)lanes);
        if (g.kernel == 3) {
            const FitJob& q = g.fit[b.job];
            GC_REQUIRE((int64_t)r >= q.blk0 && (int64_t)r - q.blk0 < J->nblk &&
                           b.lane0 == ((int64_t)r - q.blk0) * kBlock,
                       GC_E_DEVICE, "job %llu: work-list row %zu outside the job's rows",
                       (unsigned long long)J->id, r);
        }
    }
    return GC_OK;
}

// Enqueue one round of shared launches on the compute stream.
static int launch_round(gc_server* S, int round, std::vector<Job*>& active, void*& rec_host,
                        void*& rec_dev, std::vector<std::unique_ptr<LaunchTimer>>& timers) {
    rec_host = nullptr;
    rec_dev = nullptr;
    const int chunk = S->cfg.chunk_iters > 0 ? S->cfg.chunk_iters : 500;
    std::vector<Group> groups;
    auto find = [&](int kernel, int kind, int maxm, bool fp64, int walkers) -> Group& {
        for (auto& g : groups)
            if (g.kernel == kernel && g.kind == kind && g.maxm == maxm && g.fp64 == fp64 &&
                g.walkers == walkers)
                return g;
        groups.push_back(Group{kernel, kind, maxm, walkers, fp64, {}, {}, {}, {}, {}});
        return groups.back();
    };
    // fit_step jobs advance in sub-steps: one launch per iteration, all such jobs together
    std::vector<Job*> stepjobs;
    for (Job* J : active) {
        if (J->n == 0) continue;
        GC_TRY_HIP(hipStreamWaitEvent(S->compute, J->ready, 0));
        if (J->spec.kind == GC_JOB_MCMC) {
            MhJob q = J->mh;
            q.t0 = J->t_next;
            q.t1 = std::min(J->t_total, J->t_next + chunk);
            J->t_next = q.t1;
            if (J->ens) {
                Group& g = find(2, J->kind, 0, J->fp64, J->C);
                g.meff = std::max(g.meff, J->spec.model->Meff);
                const int vpb = kBlock / (J->C / 2);
                const int jb = (int)g.mh.size();
                g.mh.push_back(q);
                g.owners.push_back(J);
                for (int64_t v0 = 0; v0 < J->n; v0 += vpb) g.map.push_back(BlkMap{jb, 0, v0});
            } else {
                // instantiations that read their data from memory share it among
                // the chains of a voxel when all jobs of the launch have the same
                // chain count dividing the block: such jobs are grouped by it
                const bool mem = J->fp64 || (J->maxm & 0xFFFF) == 0;
                const int share = mem && kBlock % J->C == 0 ? J->C : 0;
                Group& g = find(0, J->kind, J->fp64 ? 0 : J->maxm, J->fp64, share);
                g.meff = std::max(g.meff, J->spec.model->Meff);
                const int jb = (int)g.mh.size();
                g.mh.push_back(q);
                g.owners.push_back(J);
                const int64_t NL = J->n * J->C;
                for (int64_t l0 = 0; l0 < NL; l0 += kBlock) g.map.push_back(BlkMap{jb, 0, l0});
            }
        } else if (!J->step_path) {
            FitJob q = J->fit;
            q.t0 = J->t_next + 1;
            q.t1 = std::min(J->t_total, J->t_next + 10 * chunk);
            q.b1pow = J->b1;
            q.b2pow = J->b2;
            for (int t = q.t0; t <= q.t1; ++t) {
                J->b1 *= J->spec.adam.beta1;
                J->b2 *= J->spec.adam.beta2;
            }
            J->t_next = q.t1;
            Group& g = find(1, J->kind, J->maxm, false, 0);
            const int jb = (int)g.fit.size();
            g.fit.push_back(q);
            g.owners.push_back(J);
            for (int64_t v0 = 0; v0 < J->n; v0 += kBlock) g.map.push_back(BlkMap{jb, 0, v0});
        } else {
            stepjobs.push_back(J);
        }
        J->last_round = round;
    }
    // per-iteration groups for step-path fits
    std::vector<std::vector<Group>> steps;
    const int step_round = S->cfg.baseline ? kFitStepRound : std::max(kFitStepRound, chunk / 5);
    for (int s = 0; s < step_round; ++s) {
        std::vector<Group> gs;
        for (Job* J : stepjobs) {
            const int t = J->t_next + 1;
            if (t > J->t_total) continue;
            FitJob q = J->fit;
            J->b1 *= J->spec.adam.beta1;
            J->b2 *= J->spec.adam.beta2;
            q.c1 = (float)(1.0 / (1.0 - J->b1));
            q.c2 = (float)(1.0 / (1.0 - J->b2));
            q.u = J->u0;
            q.u_in = (t % 2 == 1) ? J->u0 : J->u1;
            q.u_out = (t % 2 == 1) ? J->u1 : J->u0;
            // the loss is reduced on every iteration only under stopping rules,
            // else once, on the last iteration (the reported final loss)
            q.record = (J->loss_each || t == J->t_total) ? 1 : 0;
            q.partial = J->partial + (J->loss_each ? (size_t)(t - 1) * J->nblk : 0);
            J->t_next = t;
            Group* g = nullptr;
            for (auto& x : gs)
                if (x.kind == J->kind) g = &x;
            if (!g) {
                gs.push_back(Group{3, J->kind, 0, 0, false, {}, {}, {}, {}, {}});
                g = &gs.back();
            }
            const int jb = (int)g->fit.size();
            q.blk0 = (int64_t)g->map.size();
            g->fit.push_back(q);
            g->owners.push_back(J);
            g->iter.push_back(t);
            for (int64_t v0 = 0; v0 < J->n; v0 += kBlock) g->map.push_back(BlkMap{jb, 0, v0});
        }
        if (gs.empty()) break;
        steps.push_back(std::move(gs));
    }
    for (auto& g : groups) {
        int rc = check_group(S, g);
        if (rc) return rc;
    }
    for (auto& gs : steps)
        for (auto& g : gs) {
            int rc = check_group(S, g);
            if (rc) return rc;
        }
    // upload all descriptors of the round through one pinned buffer
    size_t bytes = 0;
    auto add = [&](size_t b) { size_t o = bytes; bytes += (b + 255) / 256 * 256; return o; };
    struct Up { Group* g; size_t od, om; };
    std::vector<Up> ups;
    for (auto& g : groups) ups.push_back(Up{&g, add(g.mh.size() * sizeof(MhJob) + g.fit.size() * sizeof(FitJob)), add(g.map.size() * sizeof(BlkMap))});
    for (auto& gs : steps)
        for (auto& g : gs) ups.push_back(Up{&g, add(g.fit.size() * sizeof(FitJob)), add(g.map.size() * sizeof(BlkMap))});
    if (ups.empty()) return GC_OK;
    char* host = (char*)S->pinned.get(bytes);
    GC_REQUIRE(host != nullptr, GC_E_NOMEM, "pinned staging of %zu bytes failed", bytes);
    char* dev = nullptr;
    hipError_t e = S->arena.alloc((void**)&dev, bytes);
    if (e != hipSuccess) {
        S->pinned.put(host);
        set_error("descriptor allocation failed");
        return GC_E_NOMEM;
    }
    // both staging buffers belong to the round record from here on: they are
    // released when the host has seen the round's event complete
    rec_host = host;
    rec_dev = dev;
    for (auto& u : ups) {
        if (!u.g->mh.empty()) std::memcpy(host + u.od, u.g->mh.data(), u.g->mh.size() * sizeof(MhJob));
        else std::memcpy(host + u.od, u.g->fit.data(), u.g->fit.size() * sizeof(FitJob));
        std::memcpy(host + u.om, u.g->map.data(), u.g->map.size() * sizeof(BlkMap));
    }
    GC_TRY_HIP(hipMemcpyAsync(dev, host, bytes, hipMemcpyHostToDevice, S->compute));
    // Streams of the round's launches.  One-job-per-launch mode keeps every
    // launch on `compute`.  Batched mode spreads the groups (each holds
    // different jobs) over lanes 1.. by largest work first onto the least
    // loaded lane, and runs the per-iteration fit steps, which must stay in
    // order, on lane 0; every lane starts after the upload and is joined
    // back into `compute` on every exit from here, so the round's event
    // (recorded on `compute` by the caller) still covers all its launches.
    struct LaneJoin {
        gc_server* S = nullptr;
        ~LaneJoin() {
            if (!S) return;
            for (int k = 0; k < gc_server::kLanes; ++k) {
                (void)hipEventRecord(S->lane_end[k], S->lane[k]);
                (void)hipStreamWaitEvent(S->compute, S->lane_end[k], 0);
            }
        }
    } join;
    const bool lanes = !S->cfg.baseline;
    std::vector<hipStream_t> gstream(groups.size(), S->compute);
    hipStream_t step_stream = S->compute;
    if (lanes) {
        GC_TRY_HIP(hipEventRecord(S->lane_start, S->compute));
        join.S = S;
        for (int k = 0; k < gc_server::kLanes; ++k)
            GC_TRY_HIP(hipStreamWaitEvent(S->lane[k], S->lane_start, 0));
        std::vector<double> work(groups.size(), 0.0);
        for (size_t i = 0; i < groups.size(); ++i) {
            const Group& g = groups[i];
            for (const MhJob& q : g.mh) work[i] += (double)q.n * q.C * (q.t1 - q.t0);
            for (const FitJob& q : g.fit) work[i] += (double)q.n * (q.t1 - q.t0 + 1);
        }
        std::vector<size_t> order(groups.size());
        for (size_t i = 0; i < order.size(); ++i) order[i] = i;
        std::sort(order.begin(), order.end(), [&](size_t a, size_t b) { return work[a] > work[b]; });
        double load[gc_server::kLanes] = {};
        for (size_t i : order) {
            int best = 1;
            for (int k = 2; k < gc_server::kLanes; ++k)
                if (load[k] < load[best]) best = k;
            load[best] += work[i];
            gstream[i] = S->lane[best];
        }
        step_stream = S->lane[0];
    }
    size_t ui = 0;
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        Group& g = groups[gi];
        Up& u = ups[ui++];
        const int nb = (int)g.map.size();
        const BlkMap* mp = (const BlkMap*)(dev + u.om);
        const hipStream_t st = gstream[gi];
        // timed launches are read out when the round has completed
        timers.push_back(std::make_unique<LaunchTimer>(
            g.kernel == 0 ? "mh_chunk" : (g.kernel == 1 ? "fit_fused" : "ens_chunk"), st));
        LaunchTimer& tm = *timers.back();
        tm.begin();
        if (g.kernel == 0) GC_TRY_HIP(mh_chunk(g.kind, g.fp64, g.maxm, (const MhJob*)(dev + u.od), mp, nb, g.walkers, g.meff, st));
        else if (g.kernel == 1) GC_TRY_HIP(fit_fused(g.kind, g.maxm, (const FitJob*)(dev + u.od), mp, nb, st));
        else GC_TRY_HIP(ens_chunk_walkers(g.kind, g.fp64, (const MhJob*)(dev + u.od), mp, nb, g.walkers, g.meff, st));
        tm.end();
    }
    for (auto& gs : steps) {
        for (auto& g : gs) {
            Up& u = ups[ui++];
            const int nb = (int)g.map.size();
            const FitJob* dj = (const FitJob*)(dev + u.od);
            timers.push_back(std::make_unique<LaunchTimer>("fit_step", step_stream));
            timers.back()->begin();
            GC_TRY_HIP(fit_step(g.kind, dj, (const BlkMap*)(dev + u.om), nb, 1, step_stream));
            timers.back()->end();
            for (size_t k = 0; k < g.fit.size(); ++k) {
                if (!g.fit[k].record) continue;
                Job* J = g.owners[k];
                const gc_adam_hyper& h = J->spec.adam;
                const int t = g.iter[k];
                GC_TRY_HIP(fit_loss_stop(g.fit[k].partial, J->nblk, J->hist, t,
                                         h.tol > 0 ? h.tol : -INFINITY, h.conv_value,
                                         h.conv_window, J->stop, step_stream));
            }
        }
    }
    return GC_OK;
}

// Results of a finished job: moment merge / final iterate, scatter to grid
// maps and one device-to-host copy into pinned staging (copy stream, after
// the job's last round); completion is detected by polling J->done.
static int finalize_job(gc_server* S, Job* J, hipEvent_t after) {
    const gc_model* m = J->spec.model;
    const int P = m->P;
    const int64_t n = J->n, G = J->pk.G;
    const hipStream_t c = S->copy;
    if (after) GC_TRY_HIP(hipStreamWaitEvent(c, after, 0));
    GC_TRY_HIP(hipStreamWaitEvent(c, J->ready, 0));
    if (J->spec.kind == GC_JOB_MCMC) {
        const int C = J->C;
        const bool acc = J->spec.out_accept != nullptr;
        J->out_bytes = (size_t)G * P * 16 + (acc ? (size_t)G * C * 4 : 0);
        char* dout = nullptr;
        GC_TRY_HIP(S->arena.alloc((void**)&dout, J->out_bytes));
        J->dout = dout;
        if (n > 0) {
            MhJob q = J->mh;
            const int64_t vb = (n + kBlock - 1) / kBlock;
            MhJob* dj = nullptr;
            BlkMap* vm = nullptr;
            GC_TRY_HIP(S->arena.alloc((void**)&dj, sizeof(MhJob) + (size_t)vb * sizeof(BlkMap)));
            J->dj = dj;
            vm = (BlkMap*)((char*)dj + sizeof(MhJob));
            char* pin = (char*)S->pinned.get(sizeof(MhJob) + (size_t)vb * sizeof(BlkMap));
            GC_REQUIRE(pin, GC_E_NOMEM, "pinned staging failed");
            std::memcpy(pin, &q, sizeof(MhJob));
            BlkMap* hm = (BlkMap*)(pin + sizeof(MhJob));
            for (int64_t b = 0; b < vb; ++b) hm[b] = BlkMap{0, 0, b * kBlock};
            GC_TRY_HIP(hipMemcpyAsync(dj, pin, sizeof(MhJob) + (size_t)vb * sizeof(BlkMap), hipMemcpyHostToDevice, c));
            GC_TRY_HIP(mh_finalize(J->fp64, dj, vm, (int)vb, J->mean_c, J->std_c, c));
            J->pin_aux = pin;
        }
        GC_TRY_HIP(scatter_rows_f64(J->mean_c, P, n, J->pk.g2c, G, (double*)dout, c));
        GC_TRY_HIP(scatter_rows_f64(J->std_c, P, n, J->pk.g2c, G, (double*)dout + (size_t)G * P, c));
        if (acc)
            GC_TRY_HIP(scatter_rows_i32(J->mh.acc, C, n, J->pk.g2c, G,
                                        (int32_t*)(dout + (size_t)G * P * 16), c));
        J->pin_out = S->pinned.get(J->out_bytes);
        GC_REQUIRE(J->pin_out, GC_E_NOMEM, "pinned staging failed");
        GC_TRY_HIP(hipMemcpyAsync(J->pin_out, dout, J->out_bytes, hipMemcpyDeviceToHost, c));
    } else {
        J->out_bytes = (size_t)G * P * 4 + 3 * sizeof(double) + 2 * sizeof(int);
        char* dout = nullptr;
        GC_TRY_HIP(S->arena.alloc((void**)&dout, J->out_bytes));
        double* dl = (double*)(dout + (size_t)G * P * 4);
        if (n > 0) {
            const float* ufin = J->u0;
            if (J->step_path) {
                // the final iterate buffer depends on the stopping iteration:
                // a tiny device-side selection keeps this asynchronous
                GC_TRY_HIP(hipMemcpyAsync((char*)dl + 3 * sizeof(double), J->stop, 2 * sizeof(int), hipMemcpyDeviceToDevice, c));
                ufin = nullptr;
            } else {
                GC_TRY_HIP(sum_partials(J->lossv, n, dl, c));
            }
            if (ufin) GC_TRY_HIP(fit_theta(P, J->fit.lb, J->fit.rng, ufin, n, J->theta_c, c));
        }
        if (!J->step_path || n == 0)
            GC_TRY_HIP(scatter_rows_f32(J->theta_c, P, n, J->pk.g2c, G, (float*)dout, c));
        J->dout = dout;
        J->pin_out = S->pinned.get(J->out_bytes);
        GC_REQUIRE(J->pin_out, GC_E_NOMEM, "pinned staging failed");
        if (!J->step_path || n == 0) {
            GC_TRY_HIP(hipMemcpyAsync(J->pin_out, dout, J->out_bytes, hipMemcpyDeviceToHost, c));
        } else {
            // stop flag first (small copy), the maps follow once it is known
            GC_TRY_HIP(hipMemcpyAsync((char*)J->pin_out + (size_t)G * P * 4 + 3 * sizeof(double),
                                      (char*)dl + 3 * sizeof(double), 2 * sizeof(int),
                                      hipMemcpyDeviceToHost, c));
            J->stage = 1;
        }
    }
    GC_TRY_HIP(hipEventRecord(J->done, c));
    J->finishing = true;
    return GC_OK;
}

// Second stage of a per-iteration fit: with the stopping iteration known,
// pick the final iterate, scatter, and copy the maps and loss history.
static int finalize_fit_maps(gc_server* S, Job* J) {
    const gc_model* m = J->spec.model;
    const int P = m->P;
    const int64_t n = J->n, G = J->pk.G;
    const hipStream_t c = S->copy;
    const int* st = (const int*)((char*)J->pin_out + (size_t)G * P * 4 + 3 * sizeof(double));
    J->iters_run = st[0] != 0 ? st[0] : J->t_total;
    J->stop_reason = st[0] != 0 ? st[1] : 0;
    const float* ufin = (J->iters_run % 2 == 1) ? J->u1 : J->u0;
    GC_TRY_HIP(fit_theta(P, J->fit.lb, J->fit.rng, ufin, n, J->theta_c, c));
    GC_TRY_HIP(scatter_rows_f32(J->theta_c, P, n, J->pk.g2c, G, (float*)J->dout, c));
    GC_TRY_HIP(hipMemcpyAsync(J->pin_out, J->dout, (size_t)G * P * 4, hipMemcpyDeviceToHost, c));
    GC_TRY_HIP(hipMemcpyAsync((char*)J->pin_out + (size_t)G * P * 4, J->hist + (J->iters_run - 1),
                              sizeof(double), hipMemcpyDeviceToHost, c));
    GC_TRY_HIP(hipEventRecord(J->done, c));
    J->stage = 2;
    return GC_OK;
}

// Host side of completion: results into the caller's buffers, release.
static void complete_job(gc_server* S, Job* J, int status) {
    const gc_model* m = J->spec.model;
    const int P = m->P;
    const int64_t G = J->pk.G;
    if (status == GC_OK && J->pin_out) {
        if (J->spec.kind == GC_JOB_MCMC) {
            std::memcpy(J->spec.out_mean, J->pin_out, (size_t)G * P * 8);
            std::memcpy(J->spec.out_std, (char*)J->pin_out + (size_t)G * P * 8, (size_t)G * P * 8);
            if (J->spec.out_accept)
                std::memcpy(J->spec.out_accept, (char*)J->pin_out + (size_t)G * P * 16,
                            (size_t)G * J->C * 4);
        } else {
            if (J->spec.out_maps) std::memcpy(J->spec.out_maps, J->pin_out, (size_t)G * P * 4);
            if (J->spec.report) {
                J->spec.report->iters_run = J->n > 0 ? (J->step_path ? J->iters_run : J->t_total) : 0;
                J->spec.report->stop_reason = J->step_path ? J->stop_reason : 0;
                std::memcpy(&J->spec.report->final_loss, (char*)J->pin_out + (size_t)G * P * 4,
                            sizeof(double));
            }
        }
    }
    // every piece of GPU work on this job has completed (its rounds drained,
    // its result copies observed), so its memory returns to the arena now
    S->arena.free(J->dout);
    S->arena.free(J->dj);
    J->dout = nullptr;
    J->dj = nullptr;
    S->pinned.put(J->pin_out);
    S->pinned.put(J->pin_aux);
    J->pin_out = J->pin_aux = nullptr;
    J->mem.reset();
    if (J->ready) (void)hipEventDestroy(J->ready);
    if (J->done) (void)hipEventDestroy(J->done);
    J->ready = J->done = nullptr;
    std::lock_guard<std::mutex> lk(S->mu);
    J->t_done = now_seconds();
    J->status = status;
    J->state = status == GC_OK ? GC_JOB_DONE
                               : (status == GC_E_CANCELLED ? GC_JOB_CANCELLED : GC_JOB_FAILED);
    if (status == GC_OK) {
        S->n_done++;
        S->voxel_iters += J->voxel_iters;
        S->latencies.push_back(J->t_done - J->t_submit);
    } else if (status == GC_E_CANCELLED) {
        S->n_cancel++;
    } else {
        S->n_fail++;
    }
    S->used -= J->footprint;
    S->resident_lanes -= J->lanes;
    S->resident.erase(std::remove(S->resident.begin(), S->resident.end(), J), S->resident.end());
    model_release(J->spec.model);   // the job's reference (taken at submission)
    J->spec.model = nullptr;
    S->cv.notify_all();
}

struct RoundRec {
    hipEvent_t ev = nullptr;
    void* host = nullptr;      // pinned descriptor staging
    void* dev = nullptr;       // device descriptors (arena)
    std::vector<Job*> ended;   // jobs whose last work is in this round
    std::vector<std::unique_ptr<LaunchTimer>> timers;   // the round's timed launches
};

static void scheduler(gc_server* S) {
    (void)hipSetDevice(S->cfg.device);
    std::deque<RoundRec> inflight;
    int round = 0;
    const int max_inflight = S->cfg.baseline ? 1 : 2;
    for (;;) {
        // ---------------------------------------------------------- admission
        std::vector<Job*> admit;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->wake.wait_for(lk, std::chrono::milliseconds(inflight.empty() && S->resident.empty() ? 50 : 0),
                             [&] { return S->stopping || !S->queue.empty() || !S->resident.empty(); });
            const int slots = S->cfg.baseline ? 1 : (S->cfg.max_slots > 0 ? S->cfg.max_slots : 64);
            // default slots: beyond 64 (up to kMaxSlotsSmall) while the
            // resident jobs' lanes are too few to fill the GPU, so that many
            // small jobs share launches; large jobs fill it with few slots
            const bool grow = !S->cfg.baseline && S->cfg.max_slots <= 0;
            for (auto it = S->queue.begin(); it != S->queue.end();) {
                Job* J = S->jobs[*it].get();
                if (J->cancel) {
                    J->state = GC_JOB_CANCELLED;
                    J->status = GC_E_CANCELLED;
                    S->n_cancel++;
                    model_release(J->spec.model);
                    J->spec.model = nullptr;
                    it = S->queue.erase(it);
                    S->cv.notify_all();
                    continue;
                }
                if ((int)S->resident.size() >= slots &&
                    !(grow && (int)S->resident.size() < kMaxSlotsSmall &&
                      S->resident_lanes + J->lanes <= kFillLanes))
                    break;
                if (S->used + J->footprint > S->cfg.hbm_budget) {
                    if (S->cfg.baseline) break;
                    ++it;   // a later, smaller job may fit
                    continue;
                }
                S->used += J->footprint;
                S->resident_lanes += J->lanes;
                S->peak_resident = std::max(S->peak_resident, (int)S->resident.size() + 1);
                S->resident.push_back(J);
                J->state = GC_JOB_RUNNING;
                admit.push_back(J);
                it = S->queue.erase(it);
            }
            if (S->busy_since < 0 && !S->resident.empty()) S->busy_since = now_seconds();
            if (S->stopping && S->queue.empty() && S->resident.empty() && inflight.empty()) break;
        }
        for (Job* J : admit) {
            int rc = prepare_job(S, J);
            if (rc != GC_OK) {
                J->err = gc_last_error();
                (void)hipStreamSynchronize(S->prep);   // nothing of it may still run
                complete_job(S, J, rc);
            } else if (J->n == 0 || J->t_total == 0) {
                J->last_round = round - 1;
                if (finalize_job(S, J, nullptr) != GC_OK) complete_job(S, J, GC_E_DEVICE);
            }
        }
        // --------------------------------------------------------------- work
        std::vector<Job*> active;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            for (Job* J : S->resident)
                if (!J->finishing && J->n > 0 && J->t_next < J->t_total && !J->cancel) active.push_back(J);
        }
        if (!active.empty()) {
            RoundRec rec;
            int rc = launch_round(S, round, active, rec.host, rec.dev, rec.timers);
            if (rc != GC_OK) {
                // work of earlier rounds may still be running on these jobs:
                // they leave (failed) only once those rounds have drained
                const std::string msg = gc_last_error();
                for (Job* J : active) {
                    J->cancel = true;
                    J->fail_status = rc;
                    J->err = msg;
                }
            } else {
                for (Job* J : active)
                    if (J->t_next >= J->t_total) rec.ended.push_back(J);
            }
            // the record owns the staging buffers and marks the end of every
            // launch enqueued so far (also after a partial failure)
            (void)hipEventCreateWithFlags(&rec.ev, hipEventDisableTiming);
            (void)hipEventRecord(rec.ev, S->compute);
            inflight.push_back(std::move(rec));
            ++round;
        }
        // cancelled (or failed) resident jobs leave once their rounds have drained
        {
            std::vector<Job*> gone;
            {
                std::lock_guard<std::mutex> lk(S->mu);
                for (Job* J : S->resident)
                    if (J->cancel && !J->finishing && J->last_round < round - (int)inflight.size())
                        gone.push_back(J);
            }
            for (Job* J : gone) complete_job(S, J, J->fail_status != GC_OK ? J->fail_status : GC_E_CANCELLED);
        }
        // ----------------------------------------------- retire finished rounds
        while (!inflight.empty()) {
            RoundRec& r = inflight.front();
            const bool must_wait = (int)inflight.size() > max_inflight - (active.empty() ? 0 : 1) ||
                                   active.empty();
            hipError_t q = must_wait ? hipEventSynchronize(r.ev) : hipEventQuery(r.ev);
            if (q == hipErrorNotReady) break;
            for (auto& tm : r.timers) tm->flush();
            S->pinned.put(r.host);
            S->arena.free(r.dev);
            for (Job* J : r.ended)
                if (!J->cancel && finalize_job(S, J, r.ev) != GC_OK) complete_job(S, J, GC_E_DEVICE);
            (void)hipEventDestroy(r.ev);
            inflight.pop_front();
            if (!must_wait) break;
        }
        // ------------------------------------------------ completed result copies
        std::vector<Job*> fin;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            for (Job* J : S->resident)
                if (J->finishing) fin.push_back(J);
        }
        for (Job* J : fin) {
            hipError_t q = (S->cfg.baseline || active.empty()) ? hipEventSynchronize(J->done)
                                                               : hipEventQuery(J->done);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) {
                complete_job(S, J, GC_E_DEVICE);
                continue;
            }
            if (J->spec.kind == GC_JOB_FIT && J->step_path && J->n > 0 && J->stage == 1) {
                if (finalize_fit_maps(S, J) != GC_OK) complete_job(S, J, GC_E_DEVICE);
                continue;
            }
            complete_job(S, J, GC_OK);
        }
        {
            std::lock_guard<std::mutex> lk(S->mu);
            if (S->resident.empty() && S->busy_since >= 0) {
                S->busy += now_seconds() - S->busy_since;
                S->busy_since = -1.0;
            }
        }
    }
}

static double percentile(std::vector<double> v, double q) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double pos = q * (double)(v.size() - 1);
    const size_t i = (size_t)pos;
    const double f = pos - (double)i;
    return i + 1 < v.size() ? v[i] * (1.0 - f) + v[i + 1] * f : v[i];
}

}  // namespace gc

using namespace gc;

extern "C" {

int gc_server_create(const gc_server_cfg* cfg, gc_server** out) {
    try {
        clear_error();
        GC_REQUIRE(cfg && out, GC_E_INVAL, "null argument");
        int count = 0;
        GC_TRY_HIP(hipGetDeviceCount(&count));
        GC_REQUIRE(cfg->device >= 0 && cfg->device < count, GC_E_INVAL, "bad device");
        GC_TRY_HIP(hipSetDevice(cfg->device));
        mempool_setup(cfg->device);
        std::unique_ptr<gc_server> S(new gc_server());
        S->cfg = *cfg;
        if (S->cfg.hbm_budget == 0) {
            size_t fr = 0, tot = 0;
            GC_TRY_HIP(hipMemGetInfo(&fr, &tot));
            S->cfg.hbm_budget = fr / 2;
        }
        if (S->cfg.chunk_iters <= 0) S->cfg.chunk_iters = 500;
        GC_TRY_HIP(hipStreamCreateWithFlags(&S->prep, hipStreamNonBlocking));
        GC_TRY_HIP(hipStreamCreateWithFlags(&S->compute, hipStreamNonBlocking));
        GC_TRY_HIP(hipStreamCreateWithFlags(&S->copy, hipStreamNonBlocking));
        GC_TRY_HIP(hipEventCreateWithFlags(&S->lane_start, hipEventDisableTiming));
        for (int k = 0; k < gc_server::kLanes; ++k) {
            GC_TRY_HIP(hipStreamCreateWithFlags(&S->lane[k], hipStreamNonBlocking));
            GC_TRY_HIP(hipEventCreateWithFlags(&S->lane_end[k], hipEventDisableTiming));
        }
        gc_server* raw = S.release();
        raw->thr = std::thread(scheduler, raw);
        *out = raw;
        return GC_OK;
    } catch (...) {
        set_error("server creation failed");
        return GC_E_DEVICE;
    }
}

int gc_submit(gc_server* S, const gc_job* job, uint64_t* job_id) {
    try {
        clear_error();
        GC_REQUIRE(S && job && job_id && job->model, GC_E_INVAL, "null argument");
        const gc_model* m = job->model;
        int rc;
        if ((rc = validate_volume(m, &job->data))) return rc;
        if ((rc = validate_bounds(m, &job->bounds))) return rc;
        std::unique_ptr<Job> J(new Job());
        J->spec = *job;
        const int P = m->P;
        J->lb.assign(job->bounds.lb, job->bounds.lb + P);
        J->ub.assign(job->bounds.ub, job->bounds.ub + P);
        if (job->bounds.x0) J->x0.assign(job->bounds.x0, job->bounds.x0 + P);
        J->G = (int64_t)job->data.nx * job->data.ny * job->data.nz;
        if (job->kind == GC_JOB_MCMC) {
            const gc_mcmc_hyper& h = job->mcmc;
            GC_REQUIRE(job->out_mean && job->out_std, GC_E_INVAL, "MCMC job needs out_mean/out_std");
            const bool ens = h.sampler == GC_SAMPLER_ENSEMBLE;
            const int C = ens ? h.n_walkers : job->n_chains;
            GC_REQUIRE(!ens || (h.n_walkers >= 4 && h.n_walkers % 2 == 0 && h.n_walkers <= 512),
                       GC_E_INVAL, "n_walkers must be even, in 4..512");
            GC_REQUIRE(C >= 1 && C <= 65535, GC_E_INVAL, "bad chain count");
            GC_REQUIRE(job->n_iter >= 1 && job->burnin >= 0 && job->burnin < job->n_iter &&
                           job->thin >= 1 && (job->n_iter - job->burnin) / job->thin >= 2,
                       GC_E_INVAL, "bad iteration / burn-in / thinning");
            GC_REQUIRE(h.sigma > 0, GC_E_INVAL, "sigma must be > 0");
            GC_REQUIRE(h.t_start == 0 && !h.init_state, GC_E_INVAL,
                       "resume (t_start, init_state) is a gc_mcmc option, not a server job's");
            GC_REQUIRE(!h.sample_sink, GC_E_INVAL,
                       "server jobs return moments only; stream samples with gc_mcmc");
            if (h.step) J->step.assign(h.step, h.step + P);
        } else if (job->kind == GC_JOB_FIT) {
            const gc_adam_hyper& h = job->adam;
            GC_REQUIRE(job->out_maps, GC_E_INVAL, "fit job needs out_maps");
            if ((rc = validate_adam(m, &h))) return rc;
            GC_REQUIRE(h.t_start == 0 && !h.init_state && !h.final_state, GC_E_INVAL,
                       "checkpoint / resume (t_start, init_state, final_state) is a "
                       "gc_fit_askadam option, not a server job's");
            GC_REQUIRE(h.precision == GC_PREC_FP32, GC_E_INVAL,
                       "server fit jobs run in FP32 (the FP64 fit is gc_fit_askadam's)");
        } else {
            set_error("unknown job kind");
            return GC_E_INVAL;
        }
        const int64_t n = count_mask_host(job->mask, J->G);
        J->footprint = footprint_of(m, *job, J->G, n);
        J->lanes = n * (job->kind != GC_JOB_MCMC ? 1
                        : job->mcmc.sampler == GC_SAMPLER_ENSEMBLE ? job->mcmc.n_walkers
                                                                   : job->n_chains);
        GC_REQUIRE(J->footprint <= S->cfg.hbm_budget, GC_E_NOMEM,
                   "job needs %zu bytes, budget %zu", J->footprint, S->cfg.hbm_budget);
        std::lock_guard<std::mutex> lk(S->mu);
        GC_REQUIRE(!S->stopping, GC_E_INVAL, "server is shutting down");
        J->id = S->next_id++;
        J->t_submit = now_seconds();
        model_retain(m);   // released when the job finishes
        *job_id = J->id;
        S->queue.push_back(J->id);
        S->jobs[J->id] = std::move(J);
        S->n_sub++;
        S->wake.notify_all();
        return GC_OK;
    } catch (...) {
        set_error("submit failed");
        return GC_E_DEVICE;
    }
}

int gc_poll(gc_server* S, uint64_t id, int* state) {
    GC_REQUIRE(S && state, GC_E_INVAL, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->jobs.find(id);
    GC_REQUIRE(it != S->jobs.end(), GC_E_NOTFOUND, "unknown job %llu", (unsigned long long)id);
    *state = it->second->state;
    return GC_OK;
}

int gc_wait(gc_server* S, uint64_t id, int timeout_ms, int* job_status) {
    GC_REQUIRE(S, GC_E_INVAL, "null server");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->jobs.find(id);
    GC_REQUIRE(it != S->jobs.end(), GC_E_NOTFOUND, "unknown job %llu", (unsigned long long)id);
    Job* J = it->second.get();
    auto finished = [&] { return J->state >= GC_JOB_DONE; };
    if (timeout_ms < 0) S->cv.wait(lk, finished);
    else if (!S->cv.wait_for(lk, std::chrono::milliseconds(timeout_ms), finished)) {
        set_error("job %llu still running", (unsigned long long)id);
        return GC_E_TIMEOUT;
    }
    if (job_status) *job_status = J->status;
    if (J->status != GC_OK && !J->err.empty()) set_error("%s", J->err.c_str());
    return GC_OK;
}

int gc_release(gc_server* S, uint64_t id) {
    GC_REQUIRE(S, GC_E_INVAL, "null server");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->jobs.find(id);
    GC_REQUIRE(it != S->jobs.end(), GC_E_NOTFOUND, "unknown job %llu", (unsigned long long)id);
    GC_REQUIRE(it->second->state >= GC_JOB_DONE, GC_E_INVAL,
               "job %llu is still queued or running", (unsigned long long)id);
    S->jobs.erase(it);
    return GC_OK;
}

int gc_cancel(gc_server* S, uint64_t id) {
    GC_REQUIRE(S, GC_E_INVAL, "null server");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->jobs.find(id);
    GC_REQUIRE(it != S->jobs.end(), GC_E_NOTFOUND, "unknown job %llu", (unsigned long long)id);
    if (it->second->state < GC_JOB_DONE) it->second->cancel = true;
    S->wake.notify_all();
    return GC_OK;
}

int gc_job_latency(gc_server* S, uint64_t id, double* seconds) {
    GC_REQUIRE(S && seconds, GC_E_INVAL, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->jobs.find(id);
    GC_REQUIRE(it != S->jobs.end(), GC_E_NOTFOUND, "unknown job");
    GC_REQUIRE(it->second->state == GC_JOB_DONE, GC_E_INVAL, "job not finished");
    *seconds = it->second->t_done - it->second->t_submit;
    return GC_OK;
}

int gc_server_stats(gc_server* S, gc_stats* st) {
    GC_REQUIRE(S && st, GC_E_INVAL, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    st->submitted = S->n_sub;
    st->completed = S->n_done;
    st->failed = S->n_fail;
    st->cancelled = S->n_cancel;
    st->resident = (int)S->resident.size();
    st->queued = (int)S->queue.size();
    st->hbm_in_use = S->used;
    st->voxel_iters = S->voxel_iters;
    st->busy_seconds = S->busy + (S->busy_since >= 0 ? now_seconds() - S->busy_since : 0.0);
    st->p50_latency_s = percentile(S->latencies, 0.50);
    st->p99_latency_s = percentile(S->latencies, 0.99);
    st->peak_resident = S->peak_resident;
    return GC_OK;
}

int gc_server_destroy(gc_server* S) {
    if (!S) return GC_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stopping = true;
        S->wake.notify_all();
    }
    if (S->thr.joinable()) S->thr.join();
    (void)hipStreamSynchronize(S->compute);
    (void)hipStreamSynchronize(S->copy);
    (void)hipStreamSynchronize(S->prep);
    for (int k = 0; k < gc_server::kLanes; ++k) {
        (void)hipStreamSynchronize(S->lane[k]);
        (void)hipStreamDestroy(S->lane[k]);
        (void)hipEventDestroy(S->lane_end[k]);
    }
    (void)hipEventDestroy(S->lane_start);
    (void)hipStreamDestroy(S->prep);
    (void)hipStreamDestroy(S->compute);
    (void)hipStreamDestroy(S->copy);
    delete S;
    return GC_OK;
}

}  // extern "C"
