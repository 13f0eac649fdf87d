// Stand-ins for every kernel launcher of the library (see harness.hpp): a
// launch is queued on its stream like a real one and, when it runs, checks
// each address range the real kernel indexes -- per block of its work-list,
// following the kernel's own index arithmetic -- against the allocations
// live at that moment.  Nothing of the method is computed; only the index
// bookkeeping the host reads back is done (mask compaction, fills).
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <set>
#include <vector>

#include "../../paper_2511_22094_amd/csrc/gc_internal.hpp"
#include "../../paper_2511_22094_amd/csrc/gc_sense.hpp"
#include "harness.hpp"

namespace gc {

namespace {

using hh::dev_ok;
using hh::violation;

const int kParams[5] = {2, 2, 9, 5, 3};   // monoexp_t2s, monoexp_r2s, gre3, dwi2, linear3

int meff_of(int kind, const AcqDev& a) { return kind == GRE3 ? 2 * a.M : a.M; }

template <typename T> bool rd(const T* base, const T* p, uint64_t seq, const char* k,
                              const char* what, T* out) {
    if (!dev_ok(base, p, sizeof(T), seq, k, what)) return false;
    std::memcpy((void*)out, (const void*)p, sizeof(T));
    return true;
}

bool acq_ok(const AcqDev& a, uint64_t seq, const char* k) {
    bool ok = a.M >= 1;
    if (!ok) violation("%s: acquisition with %d measurements", k, a.M);
    ok &= dev_ok(nullptr, a.te, (size_t)a.M * 4, seq, k, "acq te");
    ok &= dev_ok(nullptr, a.bval, (size_t)a.M * 4, seq, k, "acq b");
    ok &= dev_ok(nullptr, a.bvec, (size_t)a.M * 12, seq, k, "acq g");
    ok &= dev_ok(nullptr, a.te_d, (size_t)a.M * 8, seq, k, "acq te (f64)");
    ok &= dev_ok(nullptr, a.bval_d, (size_t)a.M * 8, seq, k, "acq b (f64)");
    ok &= dev_ok(nullptr, a.bvec_d, (size_t)a.M * 24, seq, k, "acq g (f64)");
    ok &= dev_ok(nullptr, a.run_end, (size_t)a.nrun * 4, seq, k, "acq shell runs");
    return ok;
}

// retained samples of steps [0, T): (T - burnin) / thin for T > burnin
int kept_before(int T, int burnin, int thin) { return T > burnin ? (T - burnin) / thin : 0; }

// The arrays an MCMC descriptor points to, at the extents the kernels index.
void mh_arrays(int kind, bool fp64, const MhJob& J, uint64_t seq, const char* k, bool chunk,
               bool init) {
    const int P = kParams[kind];
    if (J.P != P) violation("%s: descriptor has P = %d for a model with %d", k, J.P, P);
    const int64_t n = J.n, NL = n * J.C;
    const size_t rs = fp64 ? 8 : 4;
    acq_ok(J.acq, seq, k);
    dev_ok(J.th, J.th, (size_t)P * NL * rs, seq, k, "chain states");
    dev_ok(J.ll, J.ll, (size_t)NL * rs, seq, k, "log-likelihoods");
    dev_ok(J.acc, J.acc, (size_t)NL * 4, seq, k, "accept counts");
    if (J.mean) {
        dev_ok(J.mean, J.mean, (size_t)P * NL * 8, seq, k, "Welford means");
        dev_ok(J.m2, J.m2, (size_t)P * NL * 8, seq, k, "Welford M2");
    }
    dev_ok(J.y, J.y, (size_t)meff_of(kind, J.acq) * n * 4, seq, k, "data");
    if (J.w) dev_ok(J.w, J.w, (size_t)n * 4, seq, k, "weights");
    if (init) {
        if (J.init_state) {
            dev_ok(J.init_state, J.init_state, (size_t)P * NL * 8, seq, k, "resume states");
            if (J.init_logl) dev_ok(J.init_logl, J.init_logl, (size_t)NL * 8, seq, k, "resume logL");
        } else if (J.x0_mode != 1 && J.x0map) {
            dev_ok(J.x0map, J.x0map, (size_t)P * n * 4, seq, k, "start map");
        }
    }
    if (chunk && J.samples) {
        dev_ok(J.samples, J.samples, (size_t)J.C * J.s_K * P * n * 4, seq, k, "samples");
        // draws retained in [t0, t1) must fall in the buffer's window
        const int lo = kept_before(J.t0, J.burnin, J.thin), hi = kept_before(J.t1, J.burnin, J.thin);
        if (hi > lo && (lo < J.s_base || hi > J.s_base + J.s_K))
            violation("%s: steps [%d, %d) retain draws %d..%d outside the buffer's %d..%d", k,
                      J.t0, J.t1, lo + 1, hi, J.s_base + 1, J.s_base + J.s_K);
    }
}

// Walks a launch's work-list: reads row b and its descriptor (checked), and
// hands both to f once per row; the descriptor arrays are checked once per
// distinct descriptor.
template <typename Desc, typename F>
void rows(const Desc* jobs, const BlkMap* map, int nblk, uint64_t seq, const char* k, F f,
          std::function<void(const Desc&)> once) {
    std::set<int> seen;
    for (int b = 0; b < nblk; ++b) {
        BlkMap bm;
        if (!rd(map, map + b, seq, k, "work-list row", &bm)) return;
        if (bm.job < 0) {
            violation("%s: row %d names descriptor %d", k, b, bm.job);
            return;
        }
        Desc J;
        if (!rd(jobs, jobs + bm.job, seq, k, "descriptor", &J)) return;
        if (seen.insert(bm.job).second) once(J);
        if (bm.lane0 < 0) violation("%s: row %d starts at negative lane %lld", k, b, (long long)bm.lane0);
        f(b, bm, J);
    }
}

bool in_list(int m, std::initializer_list<int> l) {
    for (int x : l)
        if (x == m) return true;
    return false;
}

// HH_FAIL_LAUNCH=family:k makes the k-th launch (1-based) of that launcher
// family report a launch failure, as a real launch can (the failure path of
// the host code is then exercised; nothing is queued for that launch).
bool injected_failure(const char* family) {
    static const char* spec = std::getenv("HH_FAIL_LAUNCH");
    if (!spec) return false;
    const char* colon = std::strchr(spec, ':');
    if (!colon || std::strncmp(spec, family, (size_t)(colon - spec)) != 0 ||
        std::strlen(family) != (size_t)(colon - spec))
        return false;
    static std::atomic<long> count{0};
    return count.fetch_add(1) + 1 == std::atol(colon + 1);
}

}  // namespace

// ------------------------------------------------------------------ MCMC
hipError_t mh_init(int kind, bool fp64, const MhJob* jobs, const BlkMap* map, int nblk,
                   hipStream_t s) {
    hh::count_launch("mh_init");
    hh::enqueue(s, "mh_init", [=](uint64_t seq) {
        rows<MhJob>(jobs, map, nblk, seq, "mh_init", [](int, const BlkMap&, const MhJob&) {},
                    [&](const MhJob& J) { mh_arrays(kind, fp64, J, seq, "mh_init", false, true); });
    });
    return hipSuccess;
}

hipError_t mh_chunk(int kind, bool fp64, int maxm, const MhJob* jobs, const BlkMap* map, int nblk,
                    int chains, int meff, hipStream_t s) {
    hh::count_launch("mh_chunk");
    if (injected_failure("mh_chunk")) return hipErrorLaunchFailure;
    // the launcher's dispatch: which instantiation runs, with how much LDS
    const bool share = chains > 0 && kBlock % chains == 0 && meff > 0 &&
                       (size_t)(kBlock / chains) * meff * sizeof(float) <= kMhSharedData;
    const size_t lds = share ? (size_t)(kBlock / chains) * meff * sizeof(float) : 0;
    int MAXM = 0;
    bool exact = false;
    if (!fp64 && kind != DWI2) {
        const int m = maxm & 0xFFFF;
        const bool known = kind == GRE3 ? in_list(m, {12, 24, 32}) : in_list(m, {12, 16, 32});
        if (known && !(kind == LINEAR3 && m == 32)) {
            MAXM = m;
            exact = (maxm >> 16) & 1;
        }
    }
    const bool shared_path = MAXM == 0 && lds > 0;
    hh::enqueue(s, "mh_chunk", [=](uint64_t seq) {
        const char* k = "mh_chunk";
        rows<MhJob>(
            jobs, map, nblk, seq, k,
            [&](int b, const BlkMap& bm, const MhJob& J) {
                if (shared_path) {
                    if (J.C != chains)
                        violation("%s: row %d: job with %d chains in a launch shared by %d", k, b,
                                  J.C, chains);
                    const size_t need = (size_t)(kBlock / J.C) * meff_of(kind, J.acq) * 4;
                    if (need > lds)
                        violation("%s: row %d: data staging needs %zu B of LDS, launch has %zu", k, b,
                                  need, lds);
                }
                if (MAXM > 0) {
                    if (exact && J.acq.M != MAXM)
                        violation("%s: straight-line %d-measurement instantiation for %d", k, MAXM,
                                  J.acq.M);
                    if (!exact && J.acq.M > MAXM)
                        violation("%s: %d-measurement registers for %d measurements", k, MAXM, J.acq.M);
                }
            },
            [&](const MhJob& J) {
                mh_arrays(kind, fp64, J, seq, k, true, false);
                if (J.t0 < 0 || J.t1 < J.t0) violation("%s: steps [%d, %d)", k, J.t0, J.t1);
            });
    });
    return hipSuccess;
}

hipError_t mh_finalize(bool fp64, const MhJob* jobs, const BlkMap* vmap, int nblk,
                       double* out_mean, double* out_std, hipStream_t s) {
    hh::count_launch("mh_finalize");
    hh::enqueue(s, "mh_finalize", [=](uint64_t seq) {
        const char* k = "mh_finalize";
        rows<MhJob>(jobs, vmap, nblk, seq, k, [](int, const BlkMap&, const MhJob&) {},
                    [&](const MhJob& J) {
                        const int64_t NL = J.n * J.C;
                        if (!J.mean || !J.m2) violation("%s: no Welford arrays", k);
                        dev_ok(J.mean, J.mean, (size_t)J.P * NL * 8, seq, k, "Welford means");
                        dev_ok(J.m2, J.m2, (size_t)J.P * NL * 8, seq, k, "Welford M2");
                        dev_ok(out_mean, out_mean, (size_t)J.P * J.n * 8, seq, k, "pooled means");
                        dev_ok(out_std, out_std, (size_t)J.P * J.n * 8, seq, k, "pooled SDs");
                    });
        (void)fp64;
    });
    return hipSuccess;
}

hipError_t ens_init(int kind, bool fp64, const MhJob* jobs, const BlkMap* map, int nblk,
                    hipStream_t s) {
    hh::count_launch("ens_init");
    hh::enqueue(s, "ens_init", [=](uint64_t seq) {
        rows<MhJob>(jobs, map, nblk, seq, "ens_init", [](int, const BlkMap&, const MhJob&) {},
                    [&](const MhJob& J) { mh_arrays(kind, fp64, J, seq, "ens_init", false, true); });
    });
    return hipSuccess;
}

hipError_t ens_chunk_walkers(int kind, bool fp64, const MhJob* jobs, const BlkMap* map, int nblk,
                             int walkers, int meff, hipStream_t s) {
    hh::count_launch("ens_chunk");
    hh::enqueue(s, "ens_chunk", [=](uint64_t seq) {
        const char* k = "ens_chunk";
        const int P = kParams[kind];
        const int hp = walkers / 2, vpb = kBlock / hp;
        const size_t lds = (size_t)vpb * walkers * (P + 1) * (fp64 ? 8 : 4);
        const size_t lds_y = (lds + 15) / 16 * 16 + (size_t)vpb * meff * 4;
        const bool staged = meff > 0 && lds_y <= 64 * 1024;
        if (lds > 64 * 1024) violation("%s: %zu B of walker LDS", k, lds);
        rows<MhJob>(
            jobs, map, nblk, seq, k,
            [&](int b, const BlkMap&, const MhJob& J) {
                if (J.C != walkers)
                    violation("%s: row %d: job with %d walkers in a launch for %d", k, b, J.C, walkers);
                if (staged && meff_of(kind, J.acq) > meff)
                    violation("%s: row %d: %d measurements staged in room for %d", k, b,
                              meff_of(kind, J.acq), meff);
            },
            [&](const MhJob& J) {
                mh_arrays(kind, fp64, J, seq, k, false, false);
                if (J.samples) {
                    dev_ok(J.samples, J.samples, (size_t)J.C * J.s_K * P * J.n * 4, seq, k,
                           "samples");
                    const int lo = kept_before(J.t0, J.burnin, J.thin);
                    const int hi = kept_before(J.t1, J.burnin, J.thin);
                    if (hi > lo && (lo < J.s_base || hi > J.s_base + J.s_K))
                        violation("%s: draws %d..%d outside the buffer's %d..%d", k, lo + 1, hi,
                                  J.s_base + 1, J.s_base + J.s_K);
                }
            });
    });
    return hipSuccess;
}

// ------------------------------------------------------------------ fits
namespace {
void fit_common(int kind, const FitJob& J, uint64_t seq, const char* k) {
    const int P = kParams[kind];
    if (J.P != P) violation("%s: descriptor has P = %d for a model with %d", k, J.P, P);
    const size_t np = (size_t)P * J.n * 4;
    acq_ok(J.acq, seq, k);
    dev_ok(J.y, J.y, (size_t)meff_of(kind, J.acq) * J.n * 4, seq, k, "data");
    if (J.w) dev_ok(J.w, J.w, (size_t)J.n * 4, seq, k, "weights");
    dev_ok(J.m, J.m, np, seq, k, "first moments");
    dev_ok(J.v, J.v, np, seq, k, "second moments");
    if (J.prior_mask) {
        dev_ok(J.mu, J.mu, np, seq, k, "prior means");
        dev_ok(J.sigma, J.sigma, np, seq, k, "prior SDs");
    }
}
}  // namespace

hipError_t fit_init(const FitJob* jobs, const BlkMap* map, int nblk, hipStream_t s) {
    hh::count_launch("fit_init");
    hh::enqueue(s, "fit_init", [=](uint64_t seq) {
        const char* k = "fit_init";
        rows<FitJob>(jobs, map, nblk, seq, k, [](int, const BlkMap&, const FitJob&) {},
                     [&](const FitJob& J) {
                         const size_t np = (size_t)J.P * J.n * 4;
                         dev_ok(J.u, J.u, np, seq, k, "iterate");
                         dev_ok(J.m, J.m, np, seq, k, "first moments");
                         dev_ok(J.v, J.v, np, seq, k, "second moments");
                         if (J.x0map) dev_ok(J.x0map, J.x0map, np, seq, k, "start map");
                     });
    });
    return hipSuccess;
}

hipError_t fit_fused(int kind, int maxm, const FitJob* jobs, const BlkMap* map, int nblk,
                     hipStream_t s) {
    hh::count_launch("fit_fused");
    int MAXM = 0;
    if (kind != DWI2 && (kind == GRE3 ? in_list(maxm, {12, 24, 32}) : in_list(maxm, {12, 16, 32})))
        MAXM = maxm;
    hh::enqueue(s, "fit_fused", [=](uint64_t seq) {
        const char* k = "fit_fused";
        rows<FitJob>(
            jobs, map, nblk, seq, k,
            [&](int, const BlkMap&, const FitJob& J) {
                if (MAXM > 0 && J.acq.M > MAXM)
                    violation("%s: %d-measurement registers for %d measurements", k, MAXM, J.acq.M);
            },
            [&](const FitJob& J) {
                fit_common(kind, J, seq, k);
                dev_ok(J.u, J.u, (size_t)J.P * J.n * 4, seq, k, "iterate");
                if (J.loss_v && J.t_rec >= J.t0 && J.t_rec <= J.t1)
                    dev_ok(J.loss_v, J.loss_v, (size_t)J.n * 4, seq, k, "per-voxel losses");
            });
    });
    return hipSuccess;
}

hipError_t fit_step(int kind, const FitJob* jobs, const BlkMap* map, int nblk, int xcd_remap,
                    hipStream_t s) {
    hh::count_launch("fit_step");
    if (injected_failure("fit_step")) return hipErrorLaunchFailure;
    hh::enqueue(s, "fit_step", [=](uint64_t seq) {
        const char* k = "fit_step";
        std::set<int> seen;
        std::vector<char> hit((size_t)nblk, 0);
        for (int hw = 0; hw < nblk; ++hw) {
            int b = hw;
            if (xcd_remap) {
                const int q = nblk / 8, r = nblk % 8, x = hw % 8;
                b = x * q + (x < r ? x : r) + hw / 8;
            }
            if (b < 0 || b >= nblk || hit[b]) {
                violation("%s: block %d maps to row %d (not a permutation of %d rows)", k, hw, b, nblk);
                return;
            }
            hit[b] = 1;
            BlkMap bm;
            if (!rd(map, map + b, seq, k, "work-list row", &bm)) return;
            FitJob J;
            if (bm.job < 0 || !rd(jobs, jobs + bm.job, seq, k, "descriptor", &J)) return;
            int stop0 = 0;
            if (J.stop && !rd(J.stop, J.stop, seq, k, "stop flag", &stop0)) return;
            if (!J.active || stop0 != 0) continue;
            if (seen.insert(bm.job).second) {
                fit_common(kind, J, seq, k);
                const size_t np = (size_t)J.P * J.n * 4;
                dev_ok(J.u_in, J.u_in, np, seq, k, "iterate (read)");
                dev_ok(J.u_out, J.u_out, np, seq, k, "iterate (written)");
                if (J.tv_mask && J.tv_kind != 2)
                    dev_ok(J.nbr, J.nbr, (size_t)6 * J.n * 4, seq, k, "neighbours");
                if (J.tv_mask && J.tv_kind == 2) {
                    int64_t nnz = 0;
                    if (dev_ok(J.g_rowptr, J.g_rowptr, (size_t)(J.n + 1) * 8, seq, k, "graph offsets"))
                        std::memcpy(&nnz, J.g_rowptr + J.n, 8);
                    // the kernel clamps its column reads with the descriptor's count
                    if (J.g_nnz != nnz)
                        violation("%s: descriptor graph count %lld, offsets end at %lld", k,
                                  (long long)J.g_nnz, (long long)nnz);
                    if (nnz > 0) dev_ok(J.g_col, J.g_col, (size_t)nnz * 4, seq, k, "graph columns");
                }
            }
            if (J.record) {
                if (b < J.blk0) violation("%s: row %d before its job's first row %lld", k, b, (long long)J.blk0);
                dev_ok(J.partial, J.partial + (b - J.blk0), 4, seq, k, "loss partial");
            }
        }
    });
    return hipSuccess;
}

hipError_t fit_loss_stop(const float* partial, int64_t count, double* hist, int t, double, double,
                         int W, int* stop, hipStream_t s) {
    hh::count_launch("fit_loss_stop");
    hh::enqueue(s, "fit_loss_stop", [=](uint64_t seq) {
        const char* k = "fit_loss_stop";
        dev_ok(partial, partial, (size_t)count * 4, seq, k, "loss partials");
        dev_ok(hist, hist + (t - 1), 8, seq, k, "loss history entry");
        if (W > 1 && t >= W) dev_ok(hist, hist + (t - W), (size_t)W * 8, seq, k, "loss window");
        dev_ok(stop, stop, 8, seq, k, "stop flags");
    });
    return hipSuccess;
}

hipError_t fit_theta(int P, const float*, const float*, const float* u, int64_t n, float* out,
                     hipStream_t s) {
    hh::count_launch("fit_theta");
    if (n == 0) return hipSuccess;
    hh::enqueue(s, "fit_theta", [=](uint64_t seq) {
        dev_ok(u, u, (size_t)P * n * 4, seq, "fit_theta", "iterate");
        dev_ok(out, out, (size_t)P * n * 4, seq, "fit_theta", "maps");
    });
    return hipSuccess;
}

hipError_t f32_to_f64(const float* a, double* b, int64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hh::enqueue(s, "f32_to_f64", [=](uint64_t seq) {
        dev_ok(a, a, (size_t)n * 4, seq, "f32_to_f64", "source");
        dev_ok(b, b, (size_t)n * 8, seq, "f32_to_f64", "destination");
    });
    return hipSuccess;
}

// ------------------------------------------------------------------ layout
hipError_t pack_index(const uint8_t* mask, PackPlan& plan, hipStream_t s) {
    hh::count_launch("pack_index");
    const PackPlan pl = plan;
    hh::enqueue(s, "pack_index", [=](uint64_t seq) {
        const char* k = "pack_index";
        const int64_t G = pl.n_grid, nt = pl.n_tiles;
        if (nt != (G + kTile - 1) / kTile) violation("%s: %lld tiles for %lld voxels", k, (long long)nt, (long long)G);
        bool ok = true;
        if (mask) ok &= dev_ok(mask, mask, (size_t)G, seq, k, "mask");
        ok &= dev_ok(pl.tile_count, pl.tile_count, (size_t)nt * 4, seq, k, "tile counts");
        ok &= dev_ok(pl.tile_offset, pl.tile_offset, (size_t)(nt + 1) * 8, seq, k, "tile offsets");
        ok &= dev_ok(pl.g2c, pl.g2c, (size_t)G * 4, seq, k, "grid -> compact");
        ok &= dev_ok(pl.c2g, pl.c2g, (size_t)G * 4, seq, k, "compact -> grid");
        if (!ok) return;
        int64_t c = 0;
        for (int64_t t = 0; t < nt; ++t) {
            pl.tile_offset[t] = c;
            int32_t cnt = 0;
            for (int64_t i = t * kTile; i < std::min<int64_t>(G, (t + 1) * kTile); ++i) {
                const bool in = mask ? mask[i] != 0 : true;
                pl.g2c[i] = in ? (int32_t)c : -1;
                if (in) pl.c2g[c++] = (int32_t)i;
                cnt += in ? 1 : 0;
            }
            pl.tile_count[t] = cnt;
        }
        pl.tile_offset[nt] = c;
    });
    return hipSuccess;
}

hipError_t gather_rows(const float* src, int64_t rws, int64_t G, const int32_t* c2g, int64_t n,
                       float* dst, int* flag, hipStream_t s) {
    hh::count_launch("gather_rows");
    if (n == 0 || rws == 0) return hipSuccess;
    hh::enqueue(s, "gather_rows", [=](uint64_t seq) {
        const char* k = "gather_rows";
        dev_ok(c2g, c2g, (size_t)n * 4, seq, k, "compact -> grid");
        dev_ok(src, src, (size_t)rws * G * 4, seq, k, "grid rows");
        dev_ok(dst, dst, (size_t)rws * n * 4, seq, k, "compacted rows");
        dev_ok(flag, flag, 4, seq, k, "non-finite flag");
    });
    return hipSuccess;
}

namespace {
template <typename T>
hipError_t scatter_stub(const T* src, int64_t rws, int64_t n, const int32_t* g2c, int64_t G, T* dst,
                        hipStream_t s) {
    hh::count_launch("scatter_rows");
    hh::enqueue(s, "scatter_rows", [=](uint64_t seq) {
        const char* k = "scatter_rows";
        dev_ok(g2c, g2c, (size_t)G * 4, seq, k, "grid -> compact");
        if (n > 0) dev_ok(src, src, (size_t)rws * n * sizeof(T), seq, k, "compacted rows");
        dev_ok(dst, dst, (size_t)rws * G * sizeof(T), seq, k, "grid rows");
    });
    return hipSuccess;
}
}  // namespace

hipError_t scatter_rows_f32(const float* src, int64_t rows, int64_t n, const int32_t* g2c,
                            int64_t n_grid, float* dst, hipStream_t s) {
    return scatter_stub(src, rows, n, g2c, n_grid, dst, s);
}
hipError_t scatter_rows_f64(const double* src, int64_t rows, int64_t n, const int32_t* g2c,
                            int64_t n_grid, double* dst, hipStream_t s) {
    return scatter_stub(src, rows, n, g2c, n_grid, dst, s);
}
hipError_t scatter_rows_i32(const int32_t* src, int64_t rows, int64_t n, const int32_t* g2c,
                            int64_t n_grid, int32_t* dst, hipStream_t s) {
    return scatter_stub(src, rows, n, g2c, n_grid, dst, s);
}

hipError_t build_neighbours(const int32_t* c2g, const int32_t* g2c, int64_t n, int nx, int ny,
                            int nz, int, int32_t* nbr, hipStream_t s) {
    hh::count_launch("build_neighbours");
    if (n == 0) return hipSuccess;
    hh::enqueue(s, "build_neighbours", [=](uint64_t seq) {
        const char* k = "build_neighbours";
        const int64_t G = (int64_t)nx * ny * nz;
        dev_ok(c2g, c2g, (size_t)n * 4, seq, k, "compact -> grid");
        dev_ok(g2c, g2c, (size_t)G * 4, seq, k, "grid -> compact");
        if (dev_ok(nbr, nbr, (size_t)6 * n * 4, seq, k, "neighbours"))
            for (int64_t i = 0; i < 6 * n; ++i) nbr[i] = -1;
    });
    return hipSuccess;
}

hipError_t sum_partials(const float* p, int64_t count, double* out, hipStream_t s) {
    hh::enqueue(s, "sum_partials", [=](uint64_t seq) {
        dev_ok(p, p, (size_t)count * 4, seq, "sum_partials", "partials");
        dev_ok(out, out, 8, seq, "sum_partials", "sum");
    });
    return hipSuccess;
}
hipError_t sum_partials_f64(const double* p, int64_t count, double* out, hipStream_t s) {
    hh::enqueue(s, "sum_partials_f64", [=](uint64_t seq) {
        dev_ok(p, p, (size_t)count * 8, seq, "sum_partials_f64", "partials");
        dev_ok(out, out, 8, seq, "sum_partials_f64", "sum");
    });
    return hipSuccess;
}

hipError_t fill_f32(float* p, int64_t n, float v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hh::enqueue(s, "fill_f32", [=](uint64_t seq) {
        if (dev_ok(p, p, (size_t)n * 4, seq, "fill_f32", "array"))
            for (int64_t i = 0; i < n; ++i) p[i] = v;
    });
    return hipSuccess;
}
hipError_t fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hh::enqueue(s, "fill_i32", [=](uint64_t seq) {
        if (dev_ok(p, p, (size_t)n * 4, seq, "fill_i32", "array"))
            for (int64_t i = 0; i < n; ++i) p[i] = v;
    });
    return hipSuccess;
}
hipError_t check_positive(const float* p, int64_t n, int* flag, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hh::enqueue(s, "check_positive", [=](uint64_t seq) {
        dev_ok(p, p, (size_t)n * 4, seq, "check_positive", "array");
        dev_ok(flag, flag, 4, seq, "check_positive", "flag");
    });
    return hipSuccess;
}
hipError_t check_graph(int64_t n, int64_t nnz, const int64_t* rowptr, const int32_t* col, int* flag,
                       hipStream_t s) {
    hh::enqueue(s, "check_graph", [=](uint64_t seq) {
        dev_ok(rowptr, rowptr, (size_t)(n + 1) * 8, seq, "check_graph", "offsets");
        if (nnz > 0) dev_ok(col, col, (size_t)nnz * 4, seq, "check_graph", "columns");
        dev_ok(flag, flag, 4, seq, "check_graph", "flag");
    });
    return hipSuccess;
}

// ------------------------------------------------------------------ not used by the server
#define GC_UNUSED_LAUNCHER(name)                                                     \
    do {                                                                             \
        violation("launcher %s is not modelled by the host harness", name);          \
        return hipErrorInvalidValue;                                                 \
    } while (0)

hipError_t model_forward(int, const AcqDev&, const float*, int64_t, float*, hipStream_t) {
    GC_UNUSED_LAUNCHER("model_forward");
}
hipError_t model_vjp(int, const AcqDev&, const float*, int64_t, const float*, float*, hipStream_t) {
    GC_UNUSED_LAUNCHER("model_vjp");
}
hipError_t loss_vjp(int, const AcqDev&, const float*, const float*, const float*, int64_t, int,
                    float, float*, float*, hipStream_t) {
    GC_UNUSED_LAUNCHER("loss_vjp");
}
hipError_t tv_grid(int, int, int, const uint8_t*, const float*, int, float, double*, int64_t,
                   float*, hipStream_t) {
    GC_UNUSED_LAUNCHER("tv_grid");
}
hipError_t tv_grid_iso(int, int, int, const uint8_t*, const float*, int, float, double*, int64_t,
                       float*, hipStream_t) {
    GC_UNUSED_LAUNCHER("tv_grid_iso");
}
hipError_t tv_graph(int64_t, const int64_t*, const int32_t*, const float*, float, double*, int64_t,
                    float*, hipStream_t) {
    GC_UNUSED_LAUNCHER("tv_graph");
}
hipError_t philox_batch(uint64_t, const uint32_t*, int64_t, uint32_t*, hipStream_t) {
    GC_UNUSED_LAUNCHER("philox_batch");
}
hipError_t philox_uniform_normal(uint64_t, const uint32_t*, int64_t, bool, void*, void*,
                                 hipStream_t) {
    GC_UNUSED_LAUNCHER("philox_uniform_normal");
}
hipError_t sense_pack_kspace(const SenseDev&, const float2*, float2*, hipStream_t) {
    GC_UNUSED_LAUNCHER("sense_pack_kspace");
}
hipError_t sense_forward_rows(const SenseDev&, const float2*, float2*, hipStream_t) {
    GC_UNUSED_LAUNCHER("sense_forward_rows");
}
hipError_t sense_stage(int, const SenseDev&, const SenseOpt&, const float2*, float2*, float2*,
                       float2*, float2*, float*, const int*, int, hipStream_t) {
    GC_UNUSED_LAUNCHER("sense_stage");
}
int64_t sense_partials(const SenseDev&) { return 0; }
hipError_t sense_forward_op(const SenseDev&, const float2*, float2*, float2*, hipStream_t) {
    GC_UNUSED_LAUNCHER("sense_forward_op");
}
hipError_t sense_adjoint_op(const SenseDev&, const float2*, float2*, float2*, hipStream_t) {
    GC_UNUSED_LAUNCHER("sense_adjoint_op");
}
// the FP64 fit path is gc_fit_askadam's; server jobs are FP32
hipError_t fit_init_f64(const FitJob*, const BlkMap*, int, hipStream_t) {
    GC_UNUSED_LAUNCHER("fit_init_f64");
}
hipError_t fit_step_f64(int, const FitJob*, const BlkMap*, int, int, hipStream_t) {
    GC_UNUSED_LAUNCHER("fit_step_f64");
}
hipError_t fit_loss_stop_f64(const double*, int64_t, double*, int, double, double, int, int*,
                             hipStream_t) {
    GC_UNUSED_LAUNCHER("fit_loss_stop_f64");
}
hipError_t fit_theta_f64(int, const double*, const double*, const double*, int64_t, float*,
                         hipStream_t) {
    GC_UNUSED_LAUNCHER("fit_theta_f64");
}

}  // namespace gc
