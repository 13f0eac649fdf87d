/*
 * gacelle.h -- C ABI of the MI355X voxel-parallel model-fitting library.
 *
 * The library implements the data-parallel hot path of the two solvers of
 * Chan et al., "GACELLE: GPU-accelerated tools for model parameter
 * estimation and image reconstruction" (2025):
 *   - gc_fit_askadam: whole-volume gradient fit (paper §2.2.1, Eq. 2; with
 *     the regulariser of §2.4, Eq. 4 and Eq. 5), optimisers Adam / SGDM /
 *     RMSProp, stopping rules tol / iteration / convergence window;
 *   - gc_mcmc: per-voxel Metropolis-Hastings chains with Gaussian likelihood
 *     and normal proposals, burn-in, thinning and posterior mean / std
 *     (paper §2.2.2);
 *   - a registry of forward models (paper §2.3.1: a model is a forward
 *     function of named parameters and acquisition arrays);
 *   - forward / adjoint entry points for automatic differentiation;
 *   - a continuous-batching server that runs many fit and MCMC jobs in
 *     shared launches.
 *
 * Conventions (every call):
 *   - Return value: GC_OK (0) or a negative gc_status.  gc_last_error()
 *     gives a message for the calling thread's last failure.  No C++
 *     exception crosses the ABI.
 *   - Outputs are written only when the call returns GC_OK.
 *   - All arrays are owned by the caller; synchronous calls keep no pointer
 *     after they return.  The library allocates its own scratch device
 *     memory (stream-ordered) and frees it before returning.
 *   - gc_exec selects the device, the HIP stream (hipStream_t, NULL = the
 *     legacy default stream) and whether the *bulk* array arguments (data,
 *     mask, weights, maps, samples) are host or device memory.  Small
 *     descriptor arrays (acquisition, bounds, steps, lb/ub/x0) are always
 *     host memory.  Synchronous calls return after the stream has finished
 *     the work they enqueued.
 *   - Grid layout: data y[M_eff][nz][ny][nx] (x fastest); complex models
 *     store the M real planes then the M imaginary planes (M_eff = 2M).
 *     Parameter maps are [P][nz][ny][nx] and hold 0 outside the mask.
 *   - "Compacted" order = the masked voxels in grid order (x fastest); the
 *     forward / adjoint entry points and MCMC samples use it.
 *   - Units: echo times in ms, T2* in ms, R2* in 1/s, frequency shifts in
 *     Hz, b-values in s/mm^2, diffusivities in um^2/ms, angles in radians.
 */
#ifndef GACELLE_H
#define GACELLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GC_OK = 0,
    GC_E_INVAL = -1,      /* invalid argument (sizes, bounds, options) */
    GC_E_NOMODEL = -2,    /* unknown model name */
    GC_E_NOMEM = -3,      /* device memory or server budget exhausted */
    GC_E_NONFINITE = -4,  /* non-finite data / weights inside the mask */
    GC_E_DEVICE = -5,     /* HIP runtime or launch failure */
    GC_E_CANCELLED = -6,  /* job cancelled */
    GC_E_TIMEOUT = -7,    /* gc_wait timed out */
    GC_E_NOTFOUND = -8    /* unknown job id */
} gc_status;

enum { GC_MEM_HOST = 0, GC_MEM_DEVICE = 1 };

typedef struct {
    int device;       /* HIP device ordinal; -1 = current device */
    void *stream;     /* hipStream_t; NULL = default stream */
    int mem_kind;     /* GC_MEM_HOST or GC_MEM_DEVICE for bulk arrays */
} gc_exec;

/* Message describing the calling thread's most recent failure ("" if none). */
const char *gc_last_error(void);

/* Library version string. */
const char *gc_version(void);

/* ------------------------------------------------------------------------
 * Model registry (paper §2.3.1: forward function + acquisition arrays).
 *
 *   name          P  parameters (index order)            measurements
 *   monoexp_t2s   2  S0, T2*                             M echoes (te)
 *   monoexp_r2s   2  S0, R2*            (Eq. 3)          M echoes (te)
 *   gre3          9  A1..A3, T2*1..3, df1..3             M complex echoes (te)
 *   dwi2          5  f, Da, De, theta, phi               M (bval, bvec)
 *   linear3       3  A1..A3 (basis exp(-te/tau), tau = 10, 30, 80 ms)
 *
 *   monoexp_t2s: s = S0 exp(-TE/T2*);  monoexp_r2s: s = S0 exp(-TE 1e-3 R2*)
 *   gre3:        s = sum_k A_k exp(-TE/T2*_k) exp(+i 2 pi df_k TE 1e-3)
 *   dwi2:        s = f exp(-b 1e-3 Da (g.n)^2) + (1-f) exp(-b 1e-3 De),
 *                n = (sin theta cos phi, sin theta sin phi, cos theta)
 *   linear3:     s = sum_k A_k exp(-TE/tau_k)
 * ------------------------------------------------------------------------ */
typedef struct gc_model gc_model;

typedef struct {
    int n_meas;            /* M: echoes or diffusion measurements (1..4096) */
    const double *te;      /* [M] echo times, ms (TE models; NULL for dwi2) */
    const double *bval;    /* [M] b-values, s/mm^2 (dwi2) */
    const double *bvec;    /* [M][3] unit gradient directions (dwi2) */
} gc_acq;

/* Creates a model; the acquisition arrays are copied.  GC_E_NOMODEL for an
 * unknown name, GC_E_INVAL for a missing / non-finite acquisition array. */
int gc_model_create(const char *name, const gc_acq *acq, gc_model **out);
/* P, M_eff (= 2M for complex models) and whether the signal is complex. */
int gc_model_info(const gc_model *m, int *n_params, int *n_meas_eff, int *is_complex);
/* Name of parameter p (library-owned string), NULL if p is out of range. */
const char *gc_model_param_name(const gc_model *m, int p);
int gc_model_destroy(gc_model *m);

/* ------------------------------------------------------------------------
 * Shared problem description.
 * ------------------------------------------------------------------------ */
typedef struct {
    int nx, ny, nz;        /* grid size (each >= 1) */
    const float *y;        /* [M_eff][nz][ny][nx] measured data (exec memory) */
} gc_volume;

typedef struct {
    const double *lb;      /* [P] lower bounds (host), lb < ub */
    const double *ub;      /* [P] upper bounds (host) */
    const double *x0;      /* [P] start value (host) or NULL = midpoint */
    const float *x0_map;   /* [P][nz][ny][nx] per-voxel start (exec memory) or
                              NULL; overrides x0.  Must lie inside the bounds. */
} gc_bounds;

/* Counts the voxels of a mask (the compacted length); mask == NULL counts
 * all voxels. */
int gc_count_mask(const uint8_t *mask, int64_t n_grid, int64_t *n_masked,
                  const gc_exec *exec);

/* ------------------------------------------------------------------------
 * askadam: whole-volume fit (paper §2.2.1 Eq. 2, §2.4 Eq. 4-5).
 *
 * Objective in normalised coordinates u = (theta - lb)/(ub - lb) in [0,1]:
 *   L(u) = 1/(N M_eff) sum_{v in mask} sum_j |w_v (y_vj - s_vj)|^p
 *        + lambda/N sum_{q in TV set} R_TV(u_q)
 *        + prior_lambda/N sum_{q in prior set} sum_v |(theta_qv - mu_qv) / sigma_qv|
 * N = masked voxels; p = 2 (squared) or 1 (real and imaginary parts count
 * separately).  R_TV (Eq. 5) takes one of three forms (tv_kind):
 *   GC_TV_ANISO  sum over forward neighbour pairs (a,b) in the mask of
 *                |u(b) - u(a)|, along x, y (and z if tv_dim = 3);
 *   GC_TV_ISO    sum over masked voxels a of sqrt(sum_d (u(a+e_d) - u(a))^2),
 *                the same forward differences (subgradient 0 where the norm
 *                is 0);
 *   GC_TV_GRAPH  sum over vertices i of sum_{j in N(i)} |u_i - u_j| (the
 *                surface-mesh form of §2.6.1), N(i) from a CSR adjacency over
 *                the masked voxels in grid order (vertex k = k-th masked
 *                voxel); the adjacency must be symmetric, so each edge counts
 *                from both ends.
 * The prior term is Eq. 6.  After every update u is clamped to [0,1].  Iteration t
 * evaluates L and its (sub)gradient at u_{t-1}, updates to u_t, then stops
 * if L_t < tol (reason 1), if |least-squares slope of the last conv_window
 * losses| < conv_value once t >= conv_window (reason 2), or at t = n_iter
 * (reason 0).  out_maps receives the last iterate theta(u_t).
 * ------------------------------------------------------------------------ */
enum { GC_OPT_ADAM = 0, GC_OPT_SGDM = 1, GC_OPT_RMSPROP = 2 };
enum { GC_TV_ANISO = 0, GC_TV_ISO = 1, GC_TV_GRAPH = 2 };

typedef struct {
    int optimizer;         /* GC_OPT_* */
    double lr;             /* initialLearnRate, in u units (default 0.01) */
    double beta1, beta2;   /* Adam moment decays (0.9, 0.999) */
    double eps;            /* Adam / RMSProp epsilon (1e-8) */
    double momentum;       /* SGDM (0.9) */
    double rho;            /* RMSProp squared-gradient decay (0.9) */
    int n_iter;            /* maximum iterations (>= 1) */
    int loss;              /* 1 = L1, 2 = L2 */
    const float *weights;  /* [nz][ny][nx] w_v >= 0 (exec memory) or NULL = 1 */
    double lambda;         /* TV weight (0 = off) */
    uint32_t tv_mask;      /* bit p set: TV on parameter p */
    int tv_dim;            /* 2 or 3 */
    double tol;            /* stop when L < tol (0 = off) */
    double conv_value;     /* stop when |slope| < conv_value (0 = off) */
    int conv_window;       /* window length (> 1; default 20) */
    double *loss_history;  /* host [n_iter] per-iteration loss, or NULL */
    int tv_kind;           /* GC_TV_* (default GC_TV_ANISO) */
    int64_t graph_n;       /* GC_TV_GRAPH: vertices, = number of masked voxels */
    int64_t graph_nnz;     /* GC_TV_GRAPH: adjacency entries */
    const int64_t *graph_rowptr; /* [graph_n + 1] CSR offsets: rowptr[0] = 0,
                                    non-decreasing, rowptr[graph_n] = graph_nnz
                                    (exec memory; checked on the device) */
    const int32_t *graph_col;    /* [graph_nnz] neighbour vertices in [0, graph_n)
                                    (exec memory; checked on the device) */
    double prior_lambda;   /* Eq. 6 weight (0 = off) */
    uint32_t prior_mask;   /* bit p set: prior on parameter p */
    const float *prior_mu;    /* [P][nz][ny][nx] prior means (exec memory) */
    const float *prior_sigma; /* [P][nz][ny][nx] prior SDs > 0 (exec memory) */
    /* Checkpoint / resume.  The optimiser state after iteration t is the
     * normalised iterate u_t with the first and second moments m_t, v_t
     * (SGDM keeps its velocity in m, RMSProp its squared-gradient average in
     * v; the unused plane is 0), laid out [3][P][n_masked] FP32 (u, m, v;
     * voxels in mask order, n_masked = gc_count_mask), exec memory.
     * final_state (or NULL) receives the state after the last iteration run.
     * With t_start > 0 the call runs iterations t_start + 1 .. n_iter from
     * init_state, the final_state of a call that ran t_start iterations
     * (the bounds' start values are then ignored): with the same data and
     * settings the iterates, losses and stopping decisions are those of one
     * uninterrupted call.  A convergence window (conv_value > 0) looks back
     * over earlier iterations: on resume loss_history is then required and
     * must hold the first t_start losses, which the call keeps and extends.
     * iters_run in the report counts from iteration 1.  Not for server
     * jobs. */
    int t_start;              /* iterations already run (0 = fresh start) */
    const float *init_state;  /* [3][P][n_masked] state after t_start (t_start > 0) */
    float *final_state;       /* [3][P][n_masked] state after the last iteration, or NULL */
    /* Arithmetic: GC_PREC_FP32 (0, production) or GC_PREC_FP64 (1), the
     * deterministic test path: the per-iteration kernels with the iterate,
     * moments, bias corrections and losses in FP64 (data stay FP32 inputs;
     * out_maps receives theta rounded once to FP32).  FP64 runs one launch
     * per iteration whatever the regulariser and takes no checkpoint /
     * resume fields. */
    int precision;
} gc_adam_hyper;

typedef struct {
    int iters_run;
    double final_loss;     /* L at the last iteration run */
    int stop_reason;       /* 0 iterations, 1 tol, 2 convergence window */
} gc_fit_report;

/* Fills gc_adam_hyper with the defaults listed above (n_iter = 200, L2). */
void gc_adam_defaults(gc_adam_hyper *h);

int gc_fit_askadam(const gc_model *model, const gc_volume *data, const uint8_t *mask,
                   const gc_bounds *bounds, const gc_adam_hyper *hyper, float *out_maps,
                   gc_fit_report *report, const gc_exec *exec);

/* ------------------------------------------------------------------------
 * MCMC (paper §2.2.2).  Target: uniform prior on [lb, ub] times
 *   log L(theta) = -1/(2 sigma^2) sum_j w_v^2 (y_vj - s_j(theta))^2.
 * Metropolis-Hastings step t = 0..n_iter-1 of chain c of voxel v: draw
 * z ~ N(0, I) and u ~ U(0,1) from Philox4x32-10 with key = seed and counter
 * (v, c, t, block) (v = compacted voxel index); theta' = theta + step .* z;
 * outside the box -> reject; else accept iff log u < logL(theta') -
 * logL(theta).  The state after step t is retained when t >= burnin and
 * (t - burnin + 1) is a multiple of thin; samples of all chains are pooled:
 * out_mean / out_std (n-1 normalisation) are FP64 grid maps [P][nz][ny][nx].
 * Retained samples per chain K = (n_iter - burnin) / thin (>= 2 required).
 * gc_burnin_from_ratio mirrors the paper's burn-in ratio: floor(r n_iter).
 *
 * Resume (MH only): with t_start > 0 the call runs steps t_start..n_iter-1
 * of the same random streams, starting from init_state (and init_logl),
 * e.g. the final_state / final_logl of a run that stopped at t_start: the
 * chains then continue bit for bit as if never interrupted.  Retention keeps
 * the absolute rule above; the moments, samples (K = retained steps in
 * [t_start, n_iter), >= 2) and accept counts cover this call's steps only,
 * so the moments of consecutive calls combine by the pooled-variance rule.
 *
 * Sampler GC_SAMPLER_ENSEMBLE runs the affine-invariant ensemble sampler
 * (Goodman & Weare 2010, stretch move with scale `stretch`, n_walkers
 * walkers per voxel, two half-ensembles updated in turn); n_chains is then
 * ignored and the walkers play the role of chains in every output.
 * ------------------------------------------------------------------------ */
enum { GC_X0_MIDPOINT = 0, GC_X0_UNIFORM = 1, GC_X0_GIVEN = 2 };

/* Receiver of retained samples while the chains run (paper §2.2.2: the
 * sampler keeps every thin-th state after burn-in).  Called on the calling
 * thread, in order, once per delivery: `samples` is FP32 host memory owned by
 * the library, [n_chains][k_count][n_params][n_masked], holding the retained
 * draws k_first .. k_first + k_count - 1 (0-based, counted within this call)
 * of every chain, in compacted voxel order; it is valid only during the call.
 * A nonzero return stops the run: gc_mcmc then returns GC_E_CANCELLED and
 * writes no output. */
typedef int (*gc_sample_sink)(void *user, int k_first, int k_count, const float *samples,
                              int64_t n_masked, int n_chains, int n_params);
enum { GC_PREC_FP32 = 0, GC_PREC_FP64 = 1 };
enum { GC_SAMPLER_MH = 0, GC_SAMPLER_ENSEMBLE = 1 };

typedef struct {
    double sigma;          /* noise SD of the Gaussian likelihood (> 0) */
    const double *step;    /* [P] proposal SDs, xStepSize (host); NULL = 2 % of ub-lb */
    uint64_t seed;
    int x0_mode;           /* GC_X0_*; GIVEN uses bounds->x0 / x0_map */
    const float *weights;  /* [nz][ny][nx] w_v (exec memory) or NULL = 1 */
    int precision;         /* GC_PREC_FP32 (production) or GC_PREC_FP64 */
    int sampler;           /* GC_SAMPLER_MH or GC_SAMPLER_ENSEMBLE */
    int n_walkers;         /* ensemble size (even, >= 4) */
    double stretch;        /* ensemble stepSize a > 1 (default 2) */
    int chunk_iters;       /* iterations per launch (0 = library default) */
    double *final_state;   /* [P][C][n_masked] last states (exec memory) or NULL */
    double *final_logl;    /* [C][n_masked] last log-likelihoods or NULL */
    int t_start;           /* first step of this call (resume; 0 = fresh run) */
    const double *init_state; /* [P][C][n_masked] chain states at t_start (exec
                                 memory, inside the bounds); required when
                                 t_start > 0, else overrides x0_mode */
    const double *init_logl;  /* [C][n_masked] their log-likelihoods (exec
                                 memory) or NULL = recomputed */
    gc_sample_sink sample_sink;  /* streams the retained samples (out_samples must
                                    then be NULL), or NULL */
    void *sink_user;             /* passed to sample_sink */
    size_t sink_bytes;           /* bytes per delivery (>= one draw of every chain
                                    and voxel is always delivered); 0 = 256 MiB.
                                    The library holds two device buffers and two
                                    pinned host buffers of this size while the
                                    call runs, and overlaps the copy of one
                                    delivery with the chains' next steps. */
} gc_mcmc_hyper;

void gc_mcmc_defaults(gc_mcmc_hyper *h);
int gc_burnin_from_ratio(double ratio, int n_iter);

/* out_samples: [C][K][P][n_masked] retained samples in FP32 (exec memory) or
 * NULL (then hyper->sample_sink, if set, receives them as they are drawn);
 * out_accept: [C][nz][ny][nx] accepted-move counts or NULL. */
int gc_mcmc(const gc_model *model, const gc_volume *data, const uint8_t *mask,
            const gc_bounds *bounds, int n_chains, int n_iter, int burnin, int thin,
            const gc_mcmc_hyper *hyper, double *out_mean, double *out_std,
            float *out_samples, int32_t *out_accept, const gc_exec *exec);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): gc_mcmc with the
 * same arguments and results, but every piece of device scratch (compacted
 * data, index maps, chain state, moments, descriptors, the model's
 * acquisition tables) comes from one fixed device array per GPU of
 * gc_noalloc_scratch_bytes() bytes (128 MiB), held until the process ends;
 * nothing is allocated or freed.  All bulk arguments must be device memory
 * (exec->mem_kind = GC_MEM_DEVICE) and no sample sink may be given
 * (GC_E_INVAL otherwise).  A problem whose scratch does not fit is refused
 * with GC_E_NOMEM (gc_last_error says by how much); work queued before the
 * refusal has finished when the call returns.  Calls on one GPU share its
 * array: the library runs them one at a time, and each returns only after
 * its work on the array has finished, so results never depend on an earlier
 * call's leftovers.  Calls from other processes use their own arrays. */
int gc_mcmc_noalloc(const gc_model *model, const gc_volume *data, const uint8_t *mask,
                    const gc_bounds *bounds, int n_chains, int n_iter, int burnin, int thin,
                    const gc_mcmc_hyper *hyper, double *out_mean, double *out_std,
                    float *out_samples, int32_t *out_accept, const gc_exec *exec);
/* Size in bytes of gc_mcmc_noalloc's per-GPU scratch array. */
size_t gc_noalloc_scratch_bytes(void);

/* ------------------------------------------------------------------------
 * Forward / adjoint entry points (compacted voxels, exec memory), the
 * building blocks of automatic differentiation (paper §2.2.1 relies on
 * autodiff; here the adjoints are written by hand).
 * ------------------------------------------------------------------------ */
/* s[M_eff][n] = f(theta[P][n]) */
int gc_model_forward(const gc_model *m, const float *theta, int64_t n, float *s,
                     const gc_exec *exec);
/* dtheta[P][n] = J(theta)^T ds, ds [M_eff][n] */
int gc_model_vjp(const gc_model *m, const float *theta, int64_t n, const float *ds,
                 float *dtheta, const gc_exec *exec);
/* Per-voxel data term and its gradient:
 *   loss[v] = scale * sum_j |w_v (y_vj - s_vj)|^p,
 *   dtheta[p][v] = d loss[v] / d theta_p (sign(0) = 0 for p = 1).
 * w may be NULL (= 1); loss may be NULL. */
int gc_loss_vjp(const gc_model *m, const float *theta, const float *y, const float *w,
                int64_t n, int p, double scale, float *loss, float *dtheta,
                const gc_exec *exec);
/* Total variation of one grid map u[nz][ny][nx] over the masked forward
 * neighbour pairs (Eq. 5, anisotropic L1): *R = sum |u_b - u_a| (FP64 sum,
 * host pointer); dR (grid, exec memory, may be NULL) = scale * subgradient
 * (0 outside the mask). */
int gc_tv(int nx, int ny, int nz, const uint8_t *mask, const float *u, int tv_dim,
          double scale, double *R, float *dR, const gc_exec *exec);
/* Isotropic form of the same (GC_TV_ISO above): *R = sum over masked voxels
 * of the Euclidean norm of their in-mask forward differences; dR as gc_tv. */
int gc_tv_iso(int nx, int ny, int nz, const uint8_t *mask, const float *u, int tv_dim,
              double scale, double *R, float *dR, const gc_exec *exec);
/* Graph TV (GC_TV_GRAPH above, §2.6.1) of one vertex map u[n]:
 * *R = sum_i sum_{j in N(i)} |u_i - u_j| (FP64 sum, host pointer);
 * dR[n] (exec memory, may be NULL) = scale * subgradient, which for the
 * required symmetric adjacency is 2 sum_{j in N(i)} sign(u_i - u_j).
 * rowptr [n+1] (int64) and col [nnz] (int32) in exec memory; both are
 * checked on the device first (GC_E_INVAL unless rowptr[0] = 0, rowptr is
 * non-decreasing, rowptr[n] = nnz and every col entry is in [0, n)). */
int gc_tv_graph(int64_t n, const int64_t *rowptr, const int32_t *col, int64_t nnz,
                const float *u, double scale, double *R, float *dR, const gc_exec *exec);

/* ------------------------------------------------------------------------
 * Image reconstruction with the askadam solver (paper §2.6.4, Eq. 7):
 * multi-coil, multi-echo SENSE-type reconstruction of one slice after the
 * read-out transform.  With k_ec the measured samples of echo e and coil c,
 * C_c the coil sensitivities, M_e the sampling mask and F2 the unitary 2D
 * DFT over (y, z) (exponent -2 pi i), the solver minimises over the complex
 * image I [E][Ny][Nz]
 *   L(I) = 1/Nk sum_{e,c,(y,z) in M_e} l(F2(C_c I_e) - k_ec)
 *        + lambda/Npix sum_e TV2(Re I_e) + TV2(Im I_e)
 * with l = |Re r|^2 + |Im r|^2 (loss 2) or |Re r| + |Im r| (loss 1),
 * Nk = 2 Nc (number of sampled entries over all echoes), Npix = E Ny Nz and
 * TV2 the anisotropic sum of |forward differences| along y and z.  The
 * optimiser (gc_adam_hyper: optimizer, lr in image units, betas, eps,
 * momentum, rho, n_iter, loss, lambda, tol, conv_value, conv_window,
 * loss_history) updates Re I and Im I without bounds, from `init` or 0.
 * Complex arrays are interleaved (re, im) floats.  Ny and Nz are powers of
 * two, 2 <= Ny <= 1024, 16 <= Nz <= 1024, and 1 <= n_echo, n_coil <= 1024
 * (GC_E_INVAL otherwise; also for a reconstruction whose mask samples
 * nothing).  Working memory per call, released before return: the coil-image
 * buffer 8 E Nc Ny Nz bytes, image, Adam state and loss terms about
 * 32 E Ny Nz bytes, the measured samples 8 Nc S bytes (S sampled entries)
 * and, for host (GC_MEM_HOST) arguments, device copies of the inputs.
 * ------------------------------------------------------------------------ */
typedef struct {
    int ny, nz, n_echo, n_coil;
    const float *kspace;   /* [E][Nc][Ny][Nz] complex, exec memory; entries
                              outside the mask are ignored (NULL for the
                              operator entry points) */
    const float *coils;    /* [Nc][Ny][Nz] complex, exec memory */
    const uint8_t *mask;   /* [E][Ny][Nz] 1 = sampled, exec memory */
    const float *init;     /* [E][Ny][Nz] complex start image or NULL = 0 */
} gc_sense_problem;

/* Reconstruction; out_image [E][Ny][Nz] complex (exec memory). */
int gc_sense_recon(const gc_sense_problem *prob, const gc_adam_hyper *hyper, float *out_image,
                   gc_fit_report *report, const gc_exec *exec);
/* The operator and its adjoint (autograd building blocks):
 * out [E][Nc][Ny][Nz] = M_e F2(C_c I_e) (zero outside the mask);
 * out [E][Ny][Nz] = sum_c conj(C_c) F2^H(M_e r_ec). */
int gc_sense_forward(const gc_sense_problem *prob, const float *image, float *out,
                     const gc_exec *exec);
int gc_sense_adjoint(const gc_sense_problem *prob, const float *kspace, float *out,
                     const gc_exec *exec);

/* ------------------------------------------------------------------------
 * Counter-based random stream.  The paper states that its MCMC solver gives
 * the same numbers on CPU and GPU (§2.2.2, last paragraph; Abstract); here
 * every random draw of the samplers is a pure function of (seed; voxel,
 * chain | purpose, iteration, block) through Philox4x32-10 (Salmon et al.,
 * SC'11), so a CPU implementation reproduces the GPU's draws exactly.  These
 * entry points expose the stream for that check.
 * ------------------------------------------------------------------------ */
/* out[n][4] = Philox4x32-10(ctr[n][4], key = (seed lo, seed hi)) */
int gc_philox(uint64_t seed, const uint32_t *ctr, int64_t n, uint32_t *out,
              const gc_exec *exec);
/* For each counter: the 4 words as uniforms (2k+1)/2^24 and two Box-Muller
 * pairs (words 0,1 and 2,3) as normals, in FP32 (precision 0) or FP64 (1);
 * out_u / out_z are [n][4] of float or double. */
int gc_philox_uniform_normal(uint64_t seed, const uint32_t *ctr, int64_t n, int precision,
                             void *out_u, void *out_z, const gc_exec *exec);

/* ------------------------------------------------------------------------
 * Kernel timing (profiling aid).  While enabled, a timed launch of a hot
 * kernel family carries a pair of HIP events on its dispatch
 * (hipExtLaunchKernelGGL), so the time is the kernel's own execution;
 * totals accumulate per family: "mh_chunk", "ens_chunk", "fit_fused",
 * "fit_step", the two reconstruction passes "sense_ycols" and
 * "sense_zrows", and "gather_rows" (the pack step's gather of the measured
 * data into compacted rows).  on = 0 disables (the default); on = k > 0 times every k-th
 * launch of a family within one call (k = 1: every launch), which bounds
 * the host cost of the event pair per timed launch for families launched
 * once per iteration.  The count returned by gc_timing_get is that of the
 * timed launches.  Server rounds are read out when the round completes.
 *
 * Trace: with the environment variable GACELLE_TRACE set to a file name when
 * the library is loaded, timing is on (every launch) and each timed launch
 * is also recorded -- family, device, stream, start and duration -- and
 * written at process exit to that file as Chrome trace-event JSON
 * ({"traceEvents": [{"name", "ph": "X", "pid": device, "tid": stream,
 * "ts", "dur"} ...]}, microseconds).  Start times count from a reference
 * event recorded once per device, after a device synchronisation, when its
 * first traced launch begins.  Creating and reading the event pair of every
 * launch costs host time: tracing is a profiling mode, not for timing runs.
 * ------------------------------------------------------------------------ */
int gc_timing_enable(int on);
/* Total event time (ms) and launch count of a family since the last reset. */
int gc_timing_get(const char *family, double *total_ms, int64_t *launches);
int gc_timing_reset(void);

/* ------------------------------------------------------------------------
 * Continuous-batching server.  The paper's back end batches work to fit GPU
 * memory (Abstract) and names memory-efficient batching of large or many
 * datasets as future work (§4, Discussion); this server admits fit and MCMC
 * jobs by device-memory footprint and runs them in shared launches.
 * Jobs arrive with host buffers; a scheduler
 * thread admits them while their device footprint fits the HBM budget and
 * a slot is free, packs them, and advances all resident jobs together in
 * chunks of iterations (shared launches per model); finished jobs are
 * copied back and their memory and slot are released at once, so later
 * arrivals join while others run.  Results are identical to the
 * synchronous calls with the same arguments (alone or in any mix).
 * ------------------------------------------------------------------------ */
typedef struct gc_server gc_server;

typedef struct {
    int device;            /* HIP device ordinal */
    size_t hbm_budget;     /* bytes of device memory for resident jobs (0 = half free) */
    int max_slots;         /* resident jobs at most; 0 = 64, and beyond that up
                              to 256 while the resident jobs hold fewer than
                              2^21 voxel x chain lanes (many small jobs then
                              share launches) */
    int chunk_iters;       /* MCMC iterations per shared launch (0 = 500) */
    int baseline;          /* 1 = one job at a time, synchronous copies, one job per
                              launch (the comparison path); 0 = batching */
} gc_server_cfg;

enum { GC_JOB_FIT = 0, GC_JOB_MCMC = 1 };
enum { GC_JOB_QUEUED = 0, GC_JOB_RUNNING = 1, GC_JOB_DONE = 2, GC_JOB_FAILED = 3,
       GC_JOB_CANCELLED = 4 };

typedef struct {
    int kind;                  /* GC_JOB_FIT or GC_JOB_MCMC */
    const gc_model *model;     /* the server keeps a reference until the job
                                  finishes: gc_model_destroy may come earlier */
    gc_volume data;            /* host memory */
    const uint8_t *mask;       /* host, or NULL = all voxels */
    gc_bounds bounds;          /* x0_map, if any, host memory */
    gc_adam_hyper adam;        /* FIT: weights host memory; loss_history ignored */
    int n_chains, n_iter, burnin, thin;   /* MCMC */
    gc_mcmc_hyper mcmc;        /* MCMC: weights host; final_* ignored; no sample sink */
    float *out_maps;           /* FIT: host [P][grid] */
    double *out_mean, *out_std;/* MCMC: host [P][grid] */
    int32_t *out_accept;       /* MCMC: host [C][grid] or NULL */
    gc_fit_report *report;     /* FIT: host or NULL */
} gc_job;

typedef struct {
    uint64_t submitted, completed, failed, cancelled;
    int resident, queued;
    size_t hbm_in_use;
    double voxel_iters;        /* completed voxel(-chain)-iterations */
    double busy_seconds;       /* wall time with at least one job resident */
    double p50_latency_s, p99_latency_s;   /* submit -> result on host */
    int peak_resident;         /* most jobs resident at once so far */
} gc_stats;

int gc_server_create(const gc_server_cfg *cfg, gc_server **out);
/* The caller keeps every buffer of the job alive until gc_wait returns. */
int gc_submit(gc_server *srv, const gc_job *job, uint64_t *job_id);
int gc_poll(gc_server *srv, uint64_t job_id, int *state);
/* Waits for a job (timeout_ms < 0: forever); *job_status = the job's
 * result code.  GC_E_TIMEOUT if it is still running. */
int gc_wait(gc_server *srv, uint64_t job_id, int timeout_ms, int *job_status);
int gc_cancel(gc_server *srv, uint64_t job_id);
/* Forgets a finished (done, failed or cancelled) job: its record is freed
 * and its id becomes unknown (GC_E_NOTFOUND afterwards).  GC_E_INVAL while
 * the job is queued or running.  A long-running server keeps every job's
 * record until it is released or the server is destroyed. */
int gc_release(gc_server *srv, uint64_t job_id);
/* Per-job latency (submit -> result) in seconds, for finished jobs. */
int gc_job_latency(gc_server *srv, uint64_t job_id, double *seconds);
int gc_server_stats(gc_server *srv, gc_stats *stats);
/* Drains queued and running jobs (they finish) and frees the server. */
int gc_server_destroy(gc_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* GACELLE_H */
