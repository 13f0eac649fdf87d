// Replays a serving trace through the continuous-batching server on the
// host-only stand-in runtime (see harness.hpp) and reports every access the
// stand-in kernels found outside live memory, plus the jobs' outcomes.
//
// usage: replay TRACE [--saturated] [--baseline] [--budget BYTES] [--slots N]
//                     [--chunk N] [--cancel K] [--cancel-delay MS STEP_MS] [--scale S]
// TRACE: one job per line:
//   arrival_s model kind n_vox seed n_chains n_iter burnin thin tv
// (kind: mcmc | fit; model: monoexp_t2s | gre3 | dwi2; tv: 0 | 1).
// --saturated submits every job at once; otherwise arrivals are paced at
// arrival_s * S seconds.  --cancel K cancels every K-th job (0 = none),
// alternately right after submitting it and, once all jobs are submitted,
// MS + STEP_MS * (i mod 11) milliseconds later (default 5 and 7).
// --expect-failures: a launch failure is injected (HH_FAIL_LAUNCH, see the
// stand-in launchers); the jobs of that round must then fail.
// Exit status: 0 when no violation was found, every job ended and none
// failed (with --expect-failures: some failed).
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "../../include/gacelle.h"
#include "harness.hpp"

namespace {

struct TraceJob {
    double arrival;
    std::string model, kind;
    long n_vox;
    unsigned long seed;
    int chains, iters, burnin, thin, tv;
};

struct ModelDef {
    gc_model* m = nullptr;
    int P = 0, Meff = 0;
    std::vector<double> lb, ub, step;
};

ModelDef make_model(const std::string& name) {
    ModelDef d;
    std::vector<double> te, bval, bvec;
    gc_acq acq{};
    if (name == "dwi2") {
        // 3 shells x 32 directions on a spiral over the sphere
        for (int sh = 1; sh <= 3; ++sh)
            for (int i = 0; i < 32; ++i) {
                const double z = 1.0 - (2.0 * i + 1.0) / 32.0, r = std::sqrt(1.0 - z * z);
                const double ph = 2.399963229728653 * i;
                bval.push_back(1000.0 * sh);
                bvec.insert(bvec.end(), {r * std::cos(ph), r * std::sin(ph), z});
            }
        acq.n_meas = 96;
        acq.bval = bval.data();
        acq.bvec = bvec.data();
        d.lb = {0.0, 0.1, 0.1, 0.0, -3.141592653589793};
        d.ub = {1.0, 3.5, 3.5, 1.5707963267948966, 3.141592653589793};
    } else if (name == "gre3") {
        for (int i = 0; i < 24; ++i) te.push_back(2.0 + 2.0 * i);
        acq.n_meas = 24;
        acq.te = te.data();
        d.lb = {0, 0, 0, 2, 40, 20, -25, -25, -25};
        d.ub = {1, 1, 1, 20, 120, 40, 25, 25, 25};
    } else {
        for (int i = 0; i < 12; ++i) te.push_back(2.0 + 4.0 * i);
        acq.n_meas = 12;
        acq.te = te.data();
        d.lb = {0.0, 1.0};
        d.ub = {3.0, 250.0};
    }
    if (gc_model_create(name.c_str(), &acq, &d.m) != GC_OK) {
        std::fprintf(stderr, "model %s: %s\n", name.c_str(), gc_last_error());
        std::exit(2);
    }
    int cplx = 0;
    gc_model_info(d.m, &d.P, &d.Meff, &cplx);
    for (int p = 0; p < d.P; ++p) d.step.push_back(0.02 * (d.ub[p] - d.lb[p]));
    return d;
}

}  // namespace

int main(int argc, char** argv) {
    if (argc < 2) {
        std::fprintf(stderr, "usage: replay TRACE [options]\n");
        return 2;
    }
    bool saturated = false, baseline = false, expect_failures = false;
    size_t budget = 0;
    int slots = 0, chunk = 256, cancel_every = 0, cancel_ms = 5, cancel_step_ms = 7;
    double scale = 1.0;
    for (int i = 2; i < argc; ++i) {
        const std::string a = argv[i];
        auto next = [&]() -> const char* { return i + 1 < argc ? argv[++i] : "0"; };
        if (a == "--saturated") saturated = true;
        else if (a == "--baseline") baseline = true;
        else if (a == "--budget") budget = std::strtoull(next(), nullptr, 10);
        else if (a == "--slots") slots = std::atoi(next());
        else if (a == "--chunk") chunk = std::atoi(next());
        else if (a == "--cancel") cancel_every = std::atoi(next());
        else if (a == "--cancel-delay") {
            cancel_ms = std::atoi(next());
            cancel_step_ms = std::atoi(next());
        }
        else if (a == "--scale") scale = std::atof(next());
        else if (a == "--expect-failures") expect_failures = true;
        else {
            std::fprintf(stderr, "unknown option %s\n", a.c_str());
            return 2;
        }
    }
    std::vector<TraceJob> trace;
    {
        std::ifstream f(argv[1]);
        std::string line;
        while (std::getline(f, line)) {
            if (line.empty() || line[0] == '#') continue;
            std::istringstream is(line);
            TraceJob j;
            is >> j.arrival >> j.model >> j.kind >> j.n_vox >> j.seed >> j.chains >> j.iters >>
                j.burnin >> j.thin >> j.tv;
            if (!is) {
                std::fprintf(stderr, "bad trace line: %s\n", line.c_str());
                return 2;
            }
            trace.push_back(j);
        }
    }
    std::map<std::string, ModelDef> models;
    for (const char* nm : {"monoexp_t2s", "gre3", "dwi2"}) models[nm] = make_model(nm);

    // one shared data buffer (contents do not matter to the stand-in kernels)
    // and one shared set of result buffers, sized for the largest job
    size_t ymax = 1, omax = 1, amax = 1;
    for (const auto& j : trace) {
        const long ny = (j.n_vox + 63) / 64;
        const ModelDef& d = models[j.model];
        ymax = std::max(ymax, (size_t)64 * ny * d.Meff);
        omax = std::max(omax, (size_t)64 * ny * d.P);
        amax = std::max(amax, (size_t)64 * ny * std::max(j.chains, 1));
    }
    std::vector<float> y(ymax, 0.5f), maps(omax);
    std::vector<double> mean(omax), sd(omax);
    std::vector<int32_t> acc(amax);
    std::vector<std::vector<uint8_t>> masks(trace.size());
    std::vector<gc_fit_report> reps(trace.size());
    std::vector<std::vector<int64_t>> g_rowptr(trace.size());
    std::vector<std::vector<int32_t>> g_col(trace.size());

    gc_server_cfg cfg{};
    cfg.device = 0;
    cfg.hbm_budget = budget;
    cfg.max_slots = slots;
    cfg.chunk_iters = chunk;
    cfg.baseline = baseline ? 1 : 0;
    gc_server* srv = nullptr;
    if (gc_server_create(&cfg, &srv) != GC_OK) {
        std::fprintf(stderr, "server: %s\n", gc_last_error());
        return 2;
    }
    std::vector<uint64_t> ids(trace.size(), 0);
    std::vector<bool> cancelled(trace.size(), false);
    const auto t0 = std::chrono::steady_clock::now();
    int refused = 0;
    std::vector<std::pair<uint64_t, std::chrono::steady_clock::time_point>> late;
    for (size_t i = 0; i < trace.size(); ++i) {
        const TraceJob& j = trace[i];
        if (!saturated) {
            const auto due = t0 + std::chrono::duration<double>(j.arrival * scale);
            std::this_thread::sleep_until(due);
        }
        const ModelDef& d = models[j.model];
        const int nx = 64, ny = (int)((j.n_vox + 63) / 64);
        masks[i].assign((size_t)nx * ny, 0);
        std::fill(masks[i].begin(), masks[i].begin() + j.n_vox, 1);
        gc_job job{};
        job.model = d.m;
        job.data = gc_volume{nx, ny, 1, y.data()};
        job.mask = masks[i].data();
        job.bounds = gc_bounds{d.lb.data(), d.ub.data(), nullptr, nullptr};
        if (j.kind == "mcmc") {
            job.kind = GC_JOB_MCMC;
            job.n_chains = j.chains;
            job.n_iter = j.iters;
            job.burnin = j.burnin;
            job.thin = j.thin;
            gc_mcmc_defaults(&job.mcmc);
            job.mcmc.sigma = 0.01;
            job.mcmc.step = d.step.data();
            job.mcmc.seed = j.seed;
            job.out_mean = mean.data();
            job.out_std = sd.data();
            job.out_accept = (i % 3 == 0) ? acc.data() : nullptr;
        } else {
            job.kind = GC_JOB_FIT;
            gc_adam_defaults(&job.adam);
            job.adam.n_iter = j.iters;
            if (j.tv) {
                job.adam.lambda = 1e-3;
                job.adam.tv_mask = 0x7;
                job.adam.tv_dim = 3;
                if (i % 4 == 2) {
                    // graph TV over the compacted voxels (the first n_vox of
                    // a 64-wide grid): neighbours one and one row apart
                    const int64_t n = j.n_vox;
                    std::vector<int64_t>& rp = g_rowptr[i];
                    std::vector<int32_t>& cl = g_col[i];
                    rp.assign(1, 0);
                    for (int64_t v = 0; v < n; ++v) {
                        for (int64_t w : {v - 64, v - 1, v + 1, v + 64})
                            if (w >= 0 && w < n) cl.push_back((int32_t)w);
                        rp.push_back((int64_t)cl.size());
                    }
                    job.adam.tv_kind = GC_TV_GRAPH;
                    job.adam.graph_n = n;
                    job.adam.graph_rowptr = rp.data();
                    job.adam.graph_col = cl.data();
                    job.adam.graph_nnz = (int64_t)cl.size();
                }
            }
            if (i % 5 == 1) {   // stopping rules: per-iteration launches with loss reductions
                job.adam.tol = 1e-12;
                job.adam.conv_value = 1e-12;
                job.adam.conv_window = 20;
            }
            job.out_maps = maps.data();
            job.report = &reps[i];
        }
        if (gc_submit(srv, &job, &ids[i]) != GC_OK) {
            std::fprintf(stderr, "job %zu refused: %s\n", i, gc_last_error());
            ++refused;
            ids[i] = 0;
            continue;
        }
        if (cancel_every > 0 && i % cancel_every == (size_t)cancel_every - 1) {
            // alternately at once (still queued) and a little later (likely running)
            cancelled[i] = true;
            if ((i / cancel_every) % 2 == 0) gc_cancel(srv, ids[i]);
            else late.push_back({ids[i], std::chrono::steady_clock::now() +
                                             std::chrono::milliseconds(cancel_ms + cancel_step_ms * (i % 11))});
        }
    }
    for (auto& lc : late) {
        std::this_thread::sleep_until(lc.second);
        gc_cancel(srv, lc.first);
    }
    int done = 0, failed = 0, canc = 0, late_done = 0;
    for (size_t i = 0; i < trace.size(); ++i) {
        if (!ids[i]) continue;
        int st = 0;
        if (gc_wait(srv, ids[i], -1, &st) != GC_OK) {
            std::fprintf(stderr, "wait %zu: %s\n", i, gc_last_error());
            ++failed;
            continue;
        }
        if (st == GC_OK) ++done;
        else if (st == GC_E_CANCELLED) ++canc;
        else {
            if (!expect_failures)
                std::fprintf(stderr, "job %zu (%s %s, %ld voxels) failed: %d %s\n", i,
                             trace[i].model.c_str(), trace[i].kind.c_str(), trace[i].n_vox, st,
                             gc_last_error());
            ++failed;
        }
        if (st == GC_OK && cancelled[i]) ++late_done;   // finished before the cancel arrived
        if (st == GC_E_CANCELLED && !cancelled[i]) {
            std::fprintf(stderr, "job %zu cancelled without being asked\n", i);
            ++failed;
        }
        gc_release(srv, ids[i]);
    }
    gc_stats stt{};
    gc_server_stats(srv, &stt);
    const double span =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    gc_server_destroy(srv);
    for (auto& kv : models) gc_model_destroy(kv.second.m);
    const size_t nv = hh::violations();
    std::printf("replay: %zu jobs, %d done (%d before their cancel), %d cancelled, %d failed, "
                "%d refused; resident %d (peak %d), in use %zu B after; %.2f s; violations %zu\n",
                trace.size(), done, late_done, canc, failed, refused, stt.resident,
                stt.peak_resident, stt.hbm_in_use, span, nv);
    // with an injected launch failure the jobs of that round fail (once their
    // earlier rounds have drained); every job still ends
    const bool ok = nv == 0 && (expect_failures ? failed > 0 : failed == 0) && refused == 0 &&
                    stt.resident == 0 && stt.hbm_in_use == 0;
    return ok ? 0 : 1;
}
