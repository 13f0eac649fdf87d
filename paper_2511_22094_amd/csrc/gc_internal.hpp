// Internal structures shared by the host runtime and the kernels: per-job
// descriptors that live in device memory (so one launch can serve many
// jobs), the block -> job work-list entry, and the launcher entry points.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gc_device.hpp"

namespace gc {

// One row of the block work-list: block b serves lanes [lane0, lane0+kBlock)
// of job `job` (lanes are (voxel, chain) pairs for MCMC, voxels for fits).
struct BlkMap {
    int32_t job;
    int32_t pad;
    int64_t lane0;
};

// Metropolis-Hastings / ensemble job descriptor (device memory).
struct MhJob {
    const float* y;          // [M_eff][n] compacted data
    const float* w;          // [n] weights or nullptr
    const float* x0map;      // [P][n] start map or nullptr
    int64_t n;               // voxels
    int C;                   // chains (or walkers)
    int P;
    uint32_t k0, k1;         // Philox key = seed
    int t0, t1;              // iterations of this launch
    int burnin, thin, K;     // retention; K = samples per chain in this call
    int k_base;              // samples retained before this call's first step
    int s_base, s_K;         // sample buffer: retained draws s_base + 1 .. s_base + s_K
                             // (counted from step 0) of every chain, [C][s_K][P][n]
    int x0_mode;
    const double* init_state;   // [P][C n] start states (resume) or nullptr
    const double* init_logl;    // [C][n] their log-likelihoods or nullptr
    float lb[kMaxP], ub[kMaxP], step[kMaxP], x0c[kMaxP];
    double lbd[kMaxP], ubd[kMaxP], stepd[kMaxP], x0cd[kMaxP];
    float inv2s2;
    double inv2s2d;
    float stretch;           // ensemble scale a
    double stretchd;
    float ball[kMaxP];       // ensemble start: half-width of the box around x0
    double balld[kMaxP];
    // chain state, [.][C*n] with lane = c*n + v
    void* th;                // [P][C n] Real
    void* ll;                // [C n] Real
    int32_t* acc;            // [C n]
    double* mean;            // [P][C n] Welford mean
    double* m2;              // [P][C n] Welford M2
    float* samples;          // [C][K][P][n] or nullptr
    AcqDev acq;
};

// Whole-volume fit job descriptor (device memory).
struct FitJob {
    const float* y;          // [M_eff][n]
    const float* w;          // [n] or nullptr
    const int32_t* nbr;      // [6][n] neighbours (x-,x+,y-,y+,z-,z+), -1 = none
    const float* x0map;      // [P][n] start map (parameter units) or nullptr
    int64_t n;
    int P;
    int loss_p;              // 1 or 2
    int optimizer;           // 0 Adam, 1 SGDM, 2 RMSProp
    uint32_t tv_mask;
    int tv_kind;             // 0 anisotropic grid, 1 isotropic grid, 2 graph
    const int64_t* g_rowptr; // graph TV: CSR offsets [n + 1] over compact voxels
    const int32_t* g_col;    // graph TV: neighbour compact indices
    int64_t g_nnz;           // graph TV: number of entries of g_col
    uint32_t prior_mask;     // prior (Eq. 6) on these parameters
    float scale_prior;       // prior_lambda / N
    const float* mu;         // [P][n] prior means (compacted) or nullptr
    const float* sigma;      // [P][n] prior SDs (compacted) or nullptr
    float lb[kMaxP], rng[kMaxP];   // theta = lb + rng * u
    float u0[kMaxP];         // start in u units when there is no map
    float lr, beta1, beta2, eps, momentum, rho;
    float omb1, omb2, omrho; // 1 - beta1, 1 - beta2, 1 - rho (rounded from FP64)
    float scale_data;        // 1 / (N M_eff)
    float scale_tv;          // lambda / N
    int t0, t1;              // fused: iterations t0..t1 (1-based, inclusive)
    int t_rec;               // fused: iteration whose per-voxel loss is stored (0 = none)
    double b1pow, b2pow;     // fused: beta1^(t0-1), beta2^(t0-1) (FP64)
    double beta1d, beta2d;   // the decays in FP64 for the bias corrections
    float c1, c2;            // step path: bias corrections of this iteration
    int active;              // step path: 0 = job finished, skip
    const int* stop;         // step path: stop[0] != 0 -> the fit has stopped, skip
    int record;              // step path: write the block loss partials
    float* u;                // [P][n] iterate (fused, in place)
    const float* u_in;       // step path: read
    float* u_out;            // step path: write
    float* m;                // [P][n]
    float* v;                // [P][n]
    float* loss_v;           // [n] per-voxel loss of iteration t_rec (fused) or nullptr
    float* partial;          // [nblk of this job] block loss partials (step path)
    int64_t blk0;            // first block of this job in the launch
    AcqDev acq;
    // FP64 instantiation of the step path (the deterministic test path): the
    // same constants unrounded and the iterate, moments and loss partials in
    // FP64 (data, weights, prior maps and the start map stay FP32 inputs)
    double lbd[kMaxP], rngd[kMaxP], u0d[kMaxP];
    double lrd, epsd, momentumd, rhod, omb1d, omb2d, omrhod;
    double scale_datad, scale_tvd, scale_priord;
    double c1d, c2d;
    double* ud;
    const double* u_ind;
    double* u_outd;
    double* md;
    double* vd;
    double* partiald;
};

// ---------------------------------------------------------------- launchers
// MCMC (gc_mh.hip)
hipError_t mh_init(int kind, bool fp64, const MhJob* jobs, const BlkMap* map, int nblk,
                   hipStream_t s);
// chains > 0: every job of the launch has that many chains, and instantiations
// that read their data from memory then share it through LDS among the chains
// of a voxel (when kBlock / chains rows of (meff | 1) floats fit in
// kMhSharedData bytes);
// meff = the jobs' effective measurement count (M, or 2 M if complex)
constexpr size_t kMhSharedData = 48 * 1024;
hipError_t mh_chunk(int kind, bool fp64, int maxm, const MhJob* jobs, const BlkMap* map,
                    int nblk, int chains, int meff, hipStream_t s);
hipError_t mh_finalize(bool fp64, const MhJob* jobs, const BlkMap* vmap, int nblk,
                       double* out_mean, double* out_std, hipStream_t s);
// ensemble: map rows cover groups of kBlock / (walkers / 2) voxels (lane0 = first voxel);
// meff = the largest effective measurement count (M, or 2 M if complex) of the jobs
hipError_t ens_chunk_walkers(int kind, bool fp64, const MhJob* jobs, const BlkMap* map, int nblk,
                             int walkers, int meff, hipStream_t s);
hipError_t ens_init(int kind, bool fp64, const MhJob* jobs, const BlkMap* map, int nblk,
                    hipStream_t s);
int mh_pick_maxm(int kind, int M);
int mh_pick_variant(int kind, int M, int uniform);   // code passed to mh_chunk

// fits (gc_fit.hip)
hipError_t fit_init(const FitJob* jobs, const BlkMap* map, int nblk, hipStream_t s);
// FP64 instantiations of the step path: init, one iteration, and the map
// theta = lb + rng u from an FP64 iterate, rounded once to FP32
hipError_t fit_init_f64(const FitJob* jobs, const BlkMap* map, int nblk, hipStream_t s);
hipError_t fit_step_f64(int kind, const FitJob* jobs, const BlkMap* map, int nblk, int xcd_remap,
                        hipStream_t s);
hipError_t fit_loss_stop_f64(const double* partial, int64_t count, double* hist, int t, double tol,
                             double conv, int W, int* stop, hipStream_t s);
hipError_t fit_theta_f64(int P, const double* lb, const double* rng, const double* u, int64_t n,
                         float* out, hipStream_t s);
hipError_t fit_fused(int kind, int maxm, const FitJob* jobs, const BlkMap* map, int nblk,
                     hipStream_t s);
hipError_t fit_step(int kind, const FitJob* jobs, const BlkMap* map, int nblk, int xcd_remap,
                    hipStream_t s);
int fit_pick_maxm(int kind, int M);
hipError_t fit_loss_stop(const float* partial, int64_t count, double* hist, int t, double tol,
                         double conv, int W, int* stop, hipStream_t s);
hipError_t fit_theta(int P, const float* lb, const float* rng, const float* u, int64_t n,
                     float* out, hipStream_t s);
hipError_t f32_to_f64(const float* a, double* b, int64_t n, hipStream_t s);
hipError_t model_forward(int kind, const AcqDev& a, const float* theta, int64_t n, float* s,
                         hipStream_t st);
hipError_t model_vjp(int kind, const AcqDev& a, const float* theta, int64_t n,
                     const float* ds, float* dtheta, hipStream_t st);
hipError_t loss_vjp(int kind, const AcqDev& a, const float* theta, const float* y,
                    const float* w, int64_t n, int p, float scale, float* loss, float* dtheta,
                    hipStream_t st);
hipError_t tv_grid(int nx, int ny, int nz, const uint8_t* mask, const float* u, int dim,
                   float scale, double* partial, int64_t nblk, float* dR, hipStream_t st);
hipError_t tv_grid_iso(int nx, int ny, int nz, const uint8_t* mask, const float* u, int dim,
                       float scale, double* partial, int64_t nblk, float* dR, hipStream_t st);
hipError_t tv_graph(int64_t n, const int64_t* rowptr, const int32_t* col, const float* u,
                    float scale, double* partial, int64_t nblk, float* dR, hipStream_t st);
// flag |= 1 unless rowptr[0] = 0, rowptr non-decreasing, rowptr[n] = nnz and
// every col[k] (k < nnz) in [0, n)
hipError_t check_graph(int64_t n, int64_t nnz, const int64_t* rowptr, const int32_t* col,
                       int* flag, hipStream_t st);

// layout and reductions (gc_pack.hip)
struct PackPlan {
    int64_t n_grid;
    int64_t n_tiles;         // tiles of kTile grid voxels
    int32_t* tile_count;     // [n_tiles]
    int64_t* tile_offset;    // [n_tiles + 1]
    int32_t* g2c;            // [n_grid] compact index or -1
    int32_t* c2g;            // [n_grid] (first n entries valid)
};
constexpr int kTile = 1024;
hipError_t pack_index(const uint8_t* mask, PackPlan& plan, hipStream_t s);
hipError_t gather_rows(const float* src, int64_t rows, int64_t n_grid, const int32_t* c2g,
                       int64_t n, float* dst, int* nonfinite_flag, hipStream_t s);
hipError_t scatter_rows_f32(const float* src, int64_t rows, int64_t n, const int32_t* g2c,
                            int64_t n_grid, float* dst, hipStream_t s);
hipError_t scatter_rows_f64(const double* src, int64_t rows, int64_t n, const int32_t* g2c,
                            int64_t n_grid, double* dst, hipStream_t s);
hipError_t scatter_rows_i32(const int32_t* src, int64_t rows, int64_t n, const int32_t* g2c,
                            int64_t n_grid, int32_t* dst, hipStream_t s);
hipError_t build_neighbours(const int32_t* c2g, const int32_t* g2c, int64_t n, int nx, int ny,
                            int nz, int tv_dim, int32_t* nbr, hipStream_t s);
hipError_t sum_partials(const float* partial, int64_t count, double* out, hipStream_t s);
hipError_t sum_partials_f64(const double* partial, int64_t count, double* out, hipStream_t s);
hipError_t philox_batch(uint64_t seed, const uint32_t* ctr, int64_t n, uint32_t* out,
                        hipStream_t s);
hipError_t philox_uniform_normal(uint64_t seed, const uint32_t* ctr, int64_t n, bool fp64,
                                 void* out_u, void* out_z, hipStream_t s);
hipError_t fill_f32(float* p, int64_t n, float v, hipStream_t s);
hipError_t fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
hipError_t check_positive(const float* p, int64_t n, int* flag, hipStream_t s);

}  // namespace gc
