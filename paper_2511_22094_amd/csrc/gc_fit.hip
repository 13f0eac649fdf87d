// Whole-volume gradient fitting kernels (paper §2.2.1 Eq. 2, §2.4 Eq. 4-5):
// forward model + residual + loss + hand-written adjoint + TV subgradient +
// Adam / SGDM / RMSProp update + projection, one lane per voxel.
//
// Two shapes of the same arithmetic:
//   * fused  -- no spatial coupling: the whole iteration loop runs inside the
//               kernel with the voxel's data and iterate in registers;
//   * step   -- one launch per iteration (TV couples neighbours; stopping
//               rules need the global loss): u is double-buffered so every
//               lane reads iterate t-1 and writes iterate t without a grid
//               barrier, and each block writes its loss partial.
// The per-voxel operations are the same functions in the same order, so the
// two shapes give bit-identical iterates.
#include "gc_internal.hpp"
#include "gc_timing.hpp"

namespace gc {

namespace {

template <int MAXM, bool CPLX> struct YReg {
    float r[MAXM];
    float i[CPLX ? MAXM : 1];
    __device__ __forceinline__ float re(int m) const { return r[m]; }
    __device__ __forceinline__ float im(int m) const { return i[CPLX ? m : 0]; }
};

struct YGlob {
    const float* y;
    int64_t n;
    int64_t v;
    int M;
    __device__ __forceinline__ float re(int m) const { return gload(y)[(int64_t)m * n + v]; }
    __device__ __forceinline__ float im(int m) const { return gload(y)[(int64_t)(M + m) * n + v]; }
};

// Per-component loss |w (y - s)|^LP of one voxel without its weight w >= 0,
// which is constant over the voxel and applied once by the caller:
//   LP = 2: loss += r^2, returns r          (dLoss/ds = -2 w^2 r, loss w^2)
//   LP = 1: loss += |r|, returns -sign(r)   (dLoss/ds = w (-sign r), loss w)
// with r = y - s.  LP is a template parameter so that the measurement loops
// carry no branch.
template <class Y, int LP, typename R = float> struct DLoss {
    const Y& y;
    R loss;
    __device__ __forceinline__ R one(R ym, R s) {
        const R r = ym - s;
        if constexpr (LP == 2) {
            loss += r * r;
            return r;
        } else {
            if constexpr (sizeof(R) == 4) loss += fabsf(r);
            else loss += fabs(r);
            return r > (R)0 ? (R)-1 : (r < (R)0 ? (R)1 : (R)0);
        }
    }
    __device__ __forceinline__ R re(int m, R s) { return one((R)y.re(m), s); }
    __device__ __forceinline__ R im(int m, R s) { return one((R)y.im(m), s); }
};

// upstream gradient ds read from HBM (vector-Jacobian product)
struct DGiven {
    const float* ds;
    int64_t n, v;
    int M;
    __device__ __forceinline__ float re(int m, float) const {
        return gload(ds)[(int64_t)m * n + v];
    }
    __device__ __forceinline__ float im(int m, float) const {
        return gload(ds)[(int64_t)(M + m) * n + v];
    }
};

struct SOut {
    float* s;
    int64_t n, v;
    int M;
    __device__ __forceinline__ void re(int m, float x) { s[(int64_t)m * n + v] = x; }
    __device__ __forceinline__ void im(int m, float x) { s[(int64_t)(M + m) * n + v] = x; }
};

// The descriptor's constants and arrays in the arithmetic of an
// instantiation: FP32 (production) or FP64 (the deterministic test path of
// the per-iteration shape).
template <typename R> struct FitR;
template <> struct FitR<float> {
    static __device__ __forceinline__ float lb(const FitJob& J, int p) { return J.lb[p]; }
    static __device__ __forceinline__ float rng(const FitJob& J, int p) { return J.rng[p]; }
    static __device__ __forceinline__ float u0(const FitJob& J, int p) { return J.u0[p]; }
    static __device__ __forceinline__ float lr(const FitJob& J) { return J.lr; }
    static __device__ __forceinline__ float beta1(const FitJob& J) { return J.beta1; }
    static __device__ __forceinline__ float beta2(const FitJob& J) { return J.beta2; }
    static __device__ __forceinline__ float eps(const FitJob& J) { return J.eps; }
    static __device__ __forceinline__ float momentum(const FitJob& J) { return J.momentum; }
    static __device__ __forceinline__ float rho(const FitJob& J) { return J.rho; }
    static __device__ __forceinline__ float omb1(const FitJob& J) { return J.omb1; }
    static __device__ __forceinline__ float omb2(const FitJob& J) { return J.omb2; }
    static __device__ __forceinline__ float omrho(const FitJob& J) { return J.omrho; }
    static __device__ __forceinline__ float scale_data(const FitJob& J) { return J.scale_data; }
    static __device__ __forceinline__ float scale_tv(const FitJob& J) { return J.scale_tv; }
    static __device__ __forceinline__ float scale_prior(const FitJob& J) { return J.scale_prior; }
    static __device__ __forceinline__ float c1(const FitJob& J) { return J.c1; }
    static __device__ __forceinline__ float c2(const FitJob& J) { return J.c2; }
    static __device__ __forceinline__ float* u(const FitJob& J) { return J.u; }
    static __device__ __forceinline__ const float* u_in(const FitJob& J) { return J.u_in; }
    static __device__ __forceinline__ float* u_out(const FitJob& J) { return J.u_out; }
    static __device__ __forceinline__ float* m(const FitJob& J) { return J.m; }
    static __device__ __forceinline__ float* v(const FitJob& J) { return J.v; }
    static __device__ __forceinline__ float* partial(const FitJob& J) { return J.partial; }
    static __device__ __forceinline__ float sqrt(float x) { return sqrtf(x); }
    static __device__ __forceinline__ float clamp01(float x) { return fminf(fmaxf(x, 0.f), 1.f); }
};
template <> struct FitR<double> {
    static __device__ __forceinline__ double lb(const FitJob& J, int p) { return J.lbd[p]; }
    static __device__ __forceinline__ double rng(const FitJob& J, int p) { return J.rngd[p]; }
    static __device__ __forceinline__ double u0(const FitJob& J, int p) { return J.u0d[p]; }
    static __device__ __forceinline__ double lr(const FitJob& J) { return J.lrd; }
    static __device__ __forceinline__ double beta1(const FitJob& J) { return J.beta1d; }
    static __device__ __forceinline__ double beta2(const FitJob& J) { return J.beta2d; }
    static __device__ __forceinline__ double eps(const FitJob& J) { return J.epsd; }
    static __device__ __forceinline__ double momentum(const FitJob& J) { return J.momentumd; }
    static __device__ __forceinline__ double rho(const FitJob& J) { return J.rhod; }
    static __device__ __forceinline__ double omb1(const FitJob& J) { return J.omb1d; }
    static __device__ __forceinline__ double omb2(const FitJob& J) { return J.omb2d; }
    static __device__ __forceinline__ double omrho(const FitJob& J) { return J.omrhod; }
    static __device__ __forceinline__ double scale_data(const FitJob& J) { return J.scale_datad; }
    static __device__ __forceinline__ double scale_tv(const FitJob& J) { return J.scale_tvd; }
    static __device__ __forceinline__ double scale_prior(const FitJob& J) { return J.scale_priord; }
    static __device__ __forceinline__ double c1(const FitJob& J) { return J.c1d; }
    static __device__ __forceinline__ double c2(const FitJob& J) { return J.c2d; }
    static __device__ __forceinline__ double* u(const FitJob& J) { return J.ud; }
    static __device__ __forceinline__ const double* u_in(const FitJob& J) { return J.u_ind; }
    static __device__ __forceinline__ double* u_out(const FitJob& J) { return J.u_outd; }
    static __device__ __forceinline__ double* m(const FitJob& J) { return J.md; }
    static __device__ __forceinline__ double* v(const FitJob& J) { return J.vd; }
    static __device__ __forceinline__ double* partial(const FitJob& J) { return J.partiald; }
    static __device__ __forceinline__ double sqrt(double x) { return ::sqrt(x); }
    static __device__ __forceinline__ double clamp01(double x) { return fmin(fmax(x, 0.0), 1.0); }
};

// One optimiser update of one coordinate in u units, then the projection.
template <typename R = float>
__device__ __forceinline__ R opt_update(const FitJob& J, R u, R g, R& m, R& v, R c1, R c2) {
    using F = FitR<R>;
    R un;
    if (J.optimizer == 0) {
        m = F::beta1(J) * m + F::omb1(J) * g;
        v = F::beta2(J) * v + F::omb2(J) * g * g;
        un = u - F::lr(J) * (m * c1) / (F::sqrt(v * c2) + F::eps(J));
    } else if (J.optimizer == 1) {
        m = F::momentum(J) * m - F::lr(J) * g;
        un = u + m;
    } else {
        v = F::rho(J) * v + F::omrho(J) * g * g;
        un = u - F::lr(J) * g / (F::sqrt(v) + F::eps(J));
    }
    return F::clamp01(un);
}

// data term of one voxel: loss (scaled) and dL/du (scaled) at iterate u
template <class Mdl, int MAXM, class Y, typename R = float>
__device__ __forceinline__ R data_grad(const FitJob& J, const R* u, const Y& y, R w, R* gu) {
    using F = FitR<R>;
    constexpr int P = Mdl::P;
    R th[P], g[P];
#pragma unroll
    for (int p = 0; p < P; ++p) th[p] = F::lb(J, p) + F::rng(J, p) * u[p];
    R loss, gs;   // loss and gradient factors of the voxel weight
    if (J.loss_p == 2) {
        DLoss<Y, 2, R> d{y, (R)0};
        Mdl::template grad<MAXM>(th, d, J.acq, g);
        loss = d.loss * (w * w);
        gs = (R)-2 * (w * w);
    } else {
        DLoss<Y, 1, R> d{y, (R)0};
        Mdl::template grad<MAXM>(th, d, J.acq, g);
        loss = d.loss * w;
        gs = w;
    }
#pragma unroll
    for (int p = 0; p < P; ++p) gu[p] = F::rng(J, p) * (g[p] * (gs * F::scale_data(J)));
    return loss * F::scale_data(J);
}

template <typename R> __device__ __forceinline__ R sgn(R x) {
    return x > (R)0 ? (R)1 : (x < (R)0 ? (R)-1 : (R)0);
}
__device__ __forceinline__ float sgnf(float x) { return sgn(x); }

template <typename T> __device__ __forceinline__ T absr(T x) {
    if constexpr (sizeof(T) == 4) return fabsf(x);
    else return fabs(x);
}

// Anisotropic grid TV at voxel v for one map (iterate t-1): the pairs
// (v, forward neighbour) add |difference| to R; the subgradient collects the
// pairs in which v takes part.  nb = (x-, x+, y-, y+, z-, z+), -1 = none.
// Split in two so that the neighbour values of every regularised map are in
// flight together before any subgradient waits on them.  They are read
// unconditionally (a missing neighbour, index -1, reads element 0 and is then
// ignored) so that no read waits behind a branch on the one before.
template <typename T = float>
__device__ __forceinline__ void tv_aniso_load(const T* __restrict__ up, const int32_t (&nb)[6],
                                              T (&un)[6]) {
#pragma unroll
    for (int d = 0; d < 6; ++d) un[d] = gload(up)[nb[d] >= 0 ? nb[d] : 0];
}
template <typename T = float>
__device__ __forceinline__ T tv_aniso_sub(const T (&un)[6], T uv, const int32_t (&nb)[6], T& R) {
    T g = 0;
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        const bool in = nb[d] >= 0;
        if (d & 1) {          // forward neighbour: pair (v, nb)
            const T diff = in ? un[d] - uv : (T)0;
            R += absr(diff);
            g -= sgn(diff);
        } else {              // backward neighbour: pair (nb, v)
            g += in ? sgn(uv - un[d]) : (T)0;
        }
    }
    return g;
}

// Isotropic grid TV at voxel v: R gains v's own norm G_v of its forward
// differences; the subgradient is -sum_d D_d / G_v from that norm plus, for
// each backward neighbour b, (u_v - u_b) / G_b from b's norm.  G_b needs b's
// other forward neighbours: dg[d][e] is the forward neighbour along axis e of
// the backward neighbour along axis d (dg[d][d] is v itself, unused).
template <typename T = float>
__device__ __forceinline__ T tv_iso_at(const T* __restrict__ up, T uv, const int32_t (&nb)[6],
                                       const int32_t (&dg)[3][3], T& R) {
    // all neighbour values first (unconditional reads, as for the anisotropic form)
    T uf[3], ubk[3], ud[3][3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        uf[d] = gload(up)[nb[2 * d + 1] >= 0 ? nb[2 * d + 1] : 0];
        ubk[d] = gload(up)[nb[2 * d] >= 0 ? nb[2 * d] : 0];
#pragma unroll
        for (int e = 0; e < 3; ++e) ud[d][e] = gload(up)[dg[d][e] >= 0 ? dg[d][e] : 0];
    }
    T D[3], ss = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        D[d] = nb[2 * d + 1] >= 0 ? uf[d] - uv : (T)0;
        ss += D[d] * D[d];
    }
    const T Gv = FitR<T>::sqrt(ss);
    R += Gv;
    T g = 0;
    if (Gv > (T)0) {
#pragma unroll
        for (int d = 0; d < 3; ++d) g -= D[d] / Gv;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (nb[2 * d] < 0) continue;
        const T ub = ubk[d];
        const T Dv = uv - ub;
        T sb = 0;
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            if (e == d) {
                sb += Dv * Dv;
            } else if (dg[d][e] >= 0) {
                const T t = ud[d][e] - ub;
                sb += t * t;
            }
        }
        const T Gb = FitR<T>::sqrt(sb);
        if (Gb > (T)0) g += Dv / Gb;
    }
    return g;
}

// Graph TV at vertex v: R gains sum_{j in N(v)} |u_v - u_j|; with a symmetric
// adjacency every edge also appears from j's side, so the subgradient is
// 2 sum_j sign(u_v - u_j).
template <typename T = float>
__device__ __forceinline__ T tv_graph_at(const T* __restrict__ up, T uv,
                                         const int64_t* __restrict__ rowptr,
                                         const int32_t* __restrict__ col, int64_t v, T& R) {
    T g = 0;
    const int64_t k1 = rowptr[v + 1];
    for (int64_t k = rowptr[v]; k < k1; ++k) {
        const T diff = uv - up[col[k]];
        R += absr(diff);
        g += (T)2 * sgn(diff);
    }
    return g;
}

// Graph TV split like the anisotropic form: the column indices of v's first
// kGraphNb neighbours are read once for all regularised maps (unconditionally,
// clamped into the adjacency; entries past v's degree are ignored), then each
// map's values at them, all in flight together; a vertex with more
// neighbours takes the rest one by one.  Same pairs in the same order as
// tv_graph_at.
constexpr int kGraphNb = 6;
struct GraphNb {
    int64_t k0, k1;
    int32_t c[kGraphNb];
};
__device__ __forceinline__ void graph_nb_load(const int64_t* __restrict__ rowptr,
                                              const int32_t* __restrict__ col, int64_t nnz,
                                              int64_t v, GraphNb& gn) {
    gn.k0 = gload(rowptr)[v];
    gn.k1 = gload(rowptr)[v + 1];
#pragma unroll
    for (int j = 0; j < kGraphNb; ++j) {
        const int64_t k = gn.k0 + j;
        gn.c[j] = nnz > 0 ? gload(col)[k < nnz ? k : nnz - 1] : 0;
    }
}
template <typename T = float>
__device__ __forceinline__ void tv_graph_load(const T* __restrict__ up, const GraphNb& gn,
                                              T (&un)[kGraphNb]) {
#pragma unroll
    for (int j = 0; j < kGraphNb; ++j) un[j] = gload(up)[gn.c[j]];
}
template <typename T = float>
__device__ __forceinline__ T tv_graph_sub(const T (&un)[kGraphNb], T uv, const GraphNb& gn,
                                          const T* __restrict__ up,
                                          const int32_t* __restrict__ col, T& R) {
    T g = 0;
    const int64_t deg = gn.k1 - gn.k0;
#pragma unroll
    for (int j = 0; j < kGraphNb; ++j) {
        if (j < deg) {
            const T diff = uv - un[j];
            R += absr(diff);
            g += (T)2 * sgn(diff);
        }
    }
    for (int64_t k = gn.k0 + kGraphNb; k < gn.k1; ++k) {
        const T diff = uv - up[col[k]];
        R += absr(diff);
        g += (T)2 * sgn(diff);
    }
    return g;
}

// Prior term (Eq. 6) of one voxel: scale_prior |(theta - mu) / sigma| summed
// over the parameters of prior_mask, added to the loss (returned) and its
// subgradient in u units to gu.
template <int P, typename T = float>
__device__ __forceinline__ T prior_at(const FitJob& J, const T* u, const T* mu, const T* sg,
                                      T* gu) {
    using F = FitR<T>;
    T R = 0;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        if (!((J.prior_mask >> p) & 1u)) continue;
        const T th = F::lb(J, p) + F::rng(J, p) * u[p];
        const T r = (th - mu[p]) / sg[p];
        R += absr(r);
        gu[p] += F::scale_prior(J) * sgn(r) * (F::rng(J, p) / sg[p]);
    }
    return F::scale_prior(J) * R;
}

}  // namespace

// ----------------------------------------------------------------- init
__global__ __launch_bounds__(kBlock) void fit_init_kernel(const FitJob* __restrict__ jobs,
                                                         const BlkMap* __restrict__ map) {
    const BlkMap bm = map[blockIdx.x];
    const FitJob& J = jobs[bm.job];
    const int64_t v = bm.lane0 + threadIdx.x;
    if (v >= J.n) return;
    for (int p = 0; p < J.P; ++p) {
        float u = J.u0[p];
        if (J.x0map) {
            // (x0 - lb) / (ub - lb) in FP64, rounded once
            const double x = (double)J.x0map[(int64_t)p * J.n + v];
            const double ub = (double)J.lb[p] + (double)J.rng[p];
            u = (float)((x - (double)J.lb[p]) / (ub - (double)J.lb[p]));
            u = fminf(fmaxf(u, 0.f), 1.f);
        }
        J.u[(int64_t)p * J.n + v] = u;
        J.m[(int64_t)p * J.n + v] = 0.f;
        J.v[(int64_t)p * J.n + v] = 0.f;
    }
}

hipError_t fit_init(const FitJob* jobs, const BlkMap* map, int nblk, hipStream_t s) {
    hipLaunchKernelGGL(fit_init_kernel, dim3(nblk), dim3(kBlock), 0, s, jobs, map);
    return hipGetLastError();
}

// the same start in FP64: u = (x0 - lb) / (ub - lb) unrounded, clamped
__global__ __launch_bounds__(kBlock) void fit_init_f64_kernel(const FitJob* __restrict__ jobs,
                                                             const BlkMap* __restrict__ map) {
    const BlkMap bm = map[blockIdx.x];
    const FitJob& J = jobs[bm.job];
    const int64_t v = bm.lane0 + threadIdx.x;
    if (v >= J.n) return;
    for (int p = 0; p < J.P; ++p) {
        double u = J.u0d[p];
        if (J.x0map) {
            const double x = (double)J.x0map[(int64_t)p * J.n + v];
            const double ub = J.lbd[p] + J.rngd[p];
            u = fmin(fmax((x - J.lbd[p]) / (ub - J.lbd[p]), 0.0), 1.0);
        }
        J.ud[(int64_t)p * J.n + v] = u;
        J.md[(int64_t)p * J.n + v] = 0.0;
        J.vd[(int64_t)p * J.n + v] = 0.0;
    }
}

hipError_t fit_init_f64(const FitJob* jobs, const BlkMap* map, int nblk, hipStream_t s) {
    hipLaunchKernelGGL(fit_init_f64_kernel, dim3(nblk), dim3(kBlock), 0, s, jobs, map);
    return hipGetLastError();
}

// ----------------------------------------------------------------- fused
template <int KIND, int MAXM>
__global__ __launch_bounds__(kBlock) void fit_fused_kernel(const FitJob* __restrict__ jobs,
                                                          const BlkMap* __restrict__ map) {
    using Mdl = typename ModelOf<KIND, float>::T;
    constexpr int P = Mdl::P;
    constexpr bool CPLX = Mdl::kComplex;
    const BlkMap bm = map[blockIdx.x];
    const FitJob& J = jobs[bm.job];
    const int64_t n = J.n;
    const int64_t v = bm.lane0 + threadIdx.x;
    if (v >= n) return;
    float u[P], m[P], s2[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        u[p] = J.u[(int64_t)p * n + v];
        m[p] = J.m[(int64_t)p * n + v];
        s2[p] = J.v[(int64_t)p * n + v];
    }
    const float w = J.w ? J.w[v] : 1.f;
    float pmu[P], psg[P];
    if (J.prior_mask) {
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const bool on = (J.prior_mask >> p) & 1u;
            pmu[p] = on ? J.mu[(int64_t)p * n + v] : 0.f;
            psg[p] = on ? J.sigma[(int64_t)p * n + v] : 1.f;
        }
    }
    YReg<(MAXM > 0 ? MAXM : 1), CPLX> yr;
    if constexpr (MAXM > 0) {
#pragma unroll
        for (int k = 0; k < MAXM; ++k) {
            yr.r[k] = k < J.acq.M ? J.y[(int64_t)k * n + v] : 0.f;
            if (CPLX) yr.i[k] = k < J.acq.M ? J.y[(int64_t)(J.acq.M + k) * n + v] : 0.f;
        }
    }
    const YGlob yg{J.y, n, v, J.acq.M};
    double b1t = J.b1pow, b2t = J.b2pow;
    for (int t = J.t0; t <= J.t1; ++t) {
        // FP64 bias corrections, rounded once to FP32
        b1t *= J.beta1d;
        b2t *= J.beta2d;
        const float c1 = (float)(1.0 / (1.0 - b1t));
        const float c2 = (float)(1.0 / (1.0 - b2t));
        float gu[P];
        float lv;
        if constexpr (MAXM > 0) lv = data_grad<Mdl, MAXM>(J, u, yr, w, gu);
        else lv = data_grad<Mdl, 0>(J, u, yg, w, gu);
        if (J.prior_mask) lv += prior_at<P>(J, u, pmu, psg, gu);
        if (t == J.t_rec && J.loss_v) J.loss_v[v] = lv;
#pragma unroll
        for (int p = 0; p < P; ++p) u[p] = opt_update(J, u[p], gu[p], m[p], s2[p], c1, c2);
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
        J.u[(int64_t)p * n + v] = u[p];
        J.m[(int64_t)p * n + v] = m[p];
        J.v[(int64_t)p * n + v] = s2[p];
    }
}

template <int KIND, int MAXM>
static hipError_t fused_t(const FitJob* jobs, const BlkMap* map, int nblk, hipStream_t s) {
    GC_LAUNCH((fit_fused_kernel<KIND, MAXM>), dim3(nblk), dim3(kBlock), 0, s, jobs, map);
    return hipGetLastError();
}
template <int KIND, int A, int B, int C>
static hipError_t fused_pick(int maxm, const FitJob* jobs, const BlkMap* map, int nblk,
                             hipStream_t s) {
    if (maxm == A) return fused_t<KIND, A>(jobs, map, nblk, s);
    if (maxm == B) return fused_t<KIND, B>(jobs, map, nblk, s);
    if (maxm == C) return fused_t<KIND, C>(jobs, map, nblk, s);
    return fused_t<KIND, 0>(jobs, map, nblk, s);
}

hipError_t fit_fused(int kind, int maxm, const FitJob* jobs, const BlkMap* map, int nblk,
                     hipStream_t s) {
    switch (kind) {
        case MONOEXP_T2S: return fused_pick<MONOEXP_T2S, 12, 16, 32>(maxm, jobs, map, nblk, s);
        case MONOEXP_R2S: return fused_pick<MONOEXP_R2S, 12, 16, 32>(maxm, jobs, map, nblk, s);
        case GRE3: return fused_pick<GRE3, 12, 24, 32>(maxm, jobs, map, nblk, s);
        case DWI2: return fused_t<DWI2, 0>(jobs, map, nblk, s);
        case LINEAR3: return fused_pick<LINEAR3, 12, 16, 32>(maxm, jobs, map, nblk, s);
    }
    return hipErrorInvalidValue;
}

// ----------------------------------------------------------------- step
// One iteration for every voxel of every active job.  With xcd_remap the
// hardware block index is permuted so that each XCD (blocks are dealt
// round-robin over the 8 XCDs) processes a contiguous range of voxels and
// the TV neighbour reads of adjacent blocks hit the same L2.
//
// The neighbour indices are fetched before the model so that only the
// neighbour iterate gathers wait after it.  The data are read per use: a
// register copy of all 96 dwi2 measurements cuts occupancy to three waves per
// SIMD and measured 20 % slower at 64^3.
template <int KIND, typename R>
__global__ __launch_bounds__(kBlock) void fit_step_kernel(const FitJob* __restrict__ jobs,
                                                         const BlkMap* __restrict__ map,
                                                         int nblk, int xcd_remap) {
    using Mdl = typename ModelOf<KIND, R>::T;
    using F = FitR<R>;
    constexpr int P = Mdl::P;
    __shared__ R red[kBlock / 64];
    int b = blockIdx.x;
    if (xcd_remap) {
        // hardware block b runs on XCD x = b % 8; XCD x takes the contiguous
        // logical range [x q + min(x, r), ...) of q (+1 if x < r) blocks
        const int q = nblk / 8, r = nblk % 8, x = b % 8;
        b = x * q + (x < r ? x : r) + b / 8;
    }
    const BlkMap bm = map[b];
    const FitJob& J = jobs[bm.job];
    if (!J.active || (J.stop && J.stop[0] != 0)) return;   // uniform per block
    const int64_t n = J.n;
    const int64_t v = bm.lane0 + threadIdx.x;
    const bool live = v < n;
    R contrib = 0;
    if (live) {
        const R* uin = F::u_in(J);
        R u[P], m[P], s2[P], gu[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            u[p] = gload(uin)[(int64_t)p * n + v];
        }
        const R w = J.w ? (R)gload(J.w)[v] : (R)1;
        const bool grid_tv = J.tv_mask && J.tv_kind != 2;
        int32_t nb[6], dg[3][3];
        if (grid_tv) {
#pragma unroll
            for (int d = 0; d < 6; ++d) nb[d] = gload(J.nbr)[(int64_t)d * n + v];
            if (J.tv_kind == 1) {
#pragma unroll
                for (int d = 0; d < 3; ++d)
#pragma unroll
                    for (int e = 0; e < 3; ++e) {
                        const int32_t x = gload(J.nbr)[(int64_t)(2 * e + 1) * n +
                                                       (nb[2 * d] >= 0 ? nb[2 * d] : 0)];
                        dg[d][e] = (e != d && nb[2 * d] >= 0) ? x : -1;
                    }
            }
        }
        const YGlob yg{J.y, n, v, J.acq.M};
        contrib = data_grad<Mdl, 0, YGlob, R>(J, u, yg, w, gu);
        if (J.tv_mask && J.tv_kind == 0) {
            // every regularised map's neighbour values requested first, then
            // the subgradients in map order (measured 1 % faster than one
            // round trip per map; same operations in the same order)
            R Rtv = 0;
            R un[P][6];
#pragma unroll
            for (int p = 0; p < P; ++p)
                if ((J.tv_mask >> p) & 1u) tv_aniso_load<R>(uin + (int64_t)p * n, nb, un[p]);
#pragma unroll
            for (int p = 0; p < P; ++p)
                if ((J.tv_mask >> p) & 1u)
                    gu[p] += F::scale_tv(J) * tv_aniso_sub<R>(un[p], u[p], nb, Rtv);
            contrib += F::scale_tv(J) * Rtv;
        } else if (J.tv_mask && J.tv_kind == 2) {
            R Rtv = 0;
            GraphNb gn;
            graph_nb_load(J.g_rowptr, J.g_col, J.g_nnz, v, gn);
            R un[P][kGraphNb];
#pragma unroll
            for (int p = 0; p < P; ++p)
                if ((J.tv_mask >> p) & 1u) tv_graph_load<R>(uin + (int64_t)p * n, gn, un[p]);
#pragma unroll
            for (int p = 0; p < P; ++p)
                if ((J.tv_mask >> p) & 1u)
                    gu[p] += F::scale_tv(J) *
                             tv_graph_sub<R>(un[p], u[p], gn, uin + (int64_t)p * n, J.g_col, Rtv);
            contrib += F::scale_tv(J) * Rtv;
        } else if (J.tv_mask) {
            R Rtv = 0;
#pragma unroll
            for (int p = 0; p < P; ++p) {
                if (!((J.tv_mask >> p) & 1u)) continue;
                gu[p] += F::scale_tv(J) * tv_iso_at<R>(uin + (int64_t)p * n, u[p], nb, dg, Rtv);
            }
            contrib += F::scale_tv(J) * Rtv;
        }
        if (J.prior_mask) {
            R pmu[P], psg[P];
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const bool on = (J.prior_mask >> p) & 1u;
                pmu[p] = on ? (R)gload(J.mu)[(int64_t)p * n + v] : (R)0;
                psg[p] = on ? (R)gload(J.sigma)[(int64_t)p * n + v] : (R)1;
            }
            contrib += prior_at<P, R>(J, u, pmu, psg, gu);
        }
        // the optimiser state is read only now, so that it holds no registers
        // through the data term (84 instead of 96 VGPRs; measured 1 % faster
        // than reading it with the iterate, identical results)
        R* mm = F::m(J);
        R* vv = F::v(J);
#pragma unroll
        for (int p = 0; p < P; ++p) {
            m[p] = gload(mm)[(int64_t)p * n + v];
            s2[p] = gload(vv)[(int64_t)p * n + v];
        }
        R* uout = F::u_out(J);
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const R un = opt_update<R>(J, u[p], gu[p], m[p], s2[p], F::c1(J), F::c2(J));
            uout[(int64_t)p * n + v] = un;
            mm[(int64_t)p * n + v] = m[p];
            vv[(int64_t)p * n + v] = s2[p];
        }
    }
    if (J.record) {
        const R s = block_sum(contrib, red);
        if (threadIdx.x == 0) F::partial(J)[b - J.blk0] = s;
    }
}

hipError_t fit_step(int kind, const FitJob* jobs, const BlkMap* map, int nblk, int xcd_remap,
                    hipStream_t s) {
#define GC_STEP(K)                                                                      \
    case K:                                                                             \
        GC_LAUNCH((fit_step_kernel<K, float>), dim3(nblk), dim3(kBlock), 0, s, jobs, \
                           map, nblk, xcd_remap);                                       \
        break;
    switch (kind) {
        GC_STEP(MONOEXP_T2S)
        GC_STEP(MONOEXP_R2S)
        GC_STEP(GRE3)
        GC_STEP(DWI2)
        GC_STEP(LINEAR3)
        default: return hipErrorInvalidValue;
    }
#undef GC_STEP
    return hipGetLastError();
}

hipError_t fit_step_f64(int kind, const FitJob* jobs, const BlkMap* map, int nblk, int xcd_remap,
                        hipStream_t s) {
#define GC_STEP(K)                                                                      \
    case K:                                                                             \
        GC_LAUNCH((fit_step_kernel<K, double>), dim3(nblk), dim3(kBlock), 0, s, jobs, \
                           map, nblk, xcd_remap);                                       \
        break;
    switch (kind) {
        GC_STEP(MONOEXP_T2S)
        GC_STEP(MONOEXP_R2S)
        GC_STEP(GRE3)
        GC_STEP(DWI2)
        GC_STEP(LINEAR3)
        default: return hipErrorInvalidValue;
    }
#undef GC_STEP
    return hipGetLastError();
}

// ----------------------------------------------------------------- autograd
template <int KIND>
__global__ __launch_bounds__(kBlock) void forward_kernel(AcqDev a, const float* __restrict__ th_,
                                                        int64_t n, float* __restrict__ s) {
    using Mdl = typename ModelOf<KIND, float>::T;
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= n) return;
    float th[Mdl::P];
#pragma unroll
    for (int p = 0; p < Mdl::P; ++p) th[p] = th_[(int64_t)p * n + v];
    SOut o{s, n, v, a.M};
    Mdl::forward(th, a, o);
}

template <int KIND>
__global__ __launch_bounds__(kBlock) void vjp_kernel(AcqDev a, const float* __restrict__ th_,
                                                    int64_t n, const float* __restrict__ ds,
                                                    float* __restrict__ dth) {
    using Mdl = typename ModelOf<KIND, float>::T;
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= n) return;
    float th[Mdl::P], g[Mdl::P];
#pragma unroll
    for (int p = 0; p < Mdl::P; ++p) th[p] = th_[(int64_t)p * n + v];
    DGiven d{ds, n, v, a.M};
    Mdl::template grad<0>(th, d, a, g);
#pragma unroll
    for (int p = 0; p < Mdl::P; ++p) dth[(int64_t)p * n + v] = g[p];
}

template <int KIND>
__global__ __launch_bounds__(kBlock) void loss_vjp_kernel(AcqDev a, const float* __restrict__ th_,
                                                         const float* __restrict__ y,
                                                         const float* __restrict__ w, int64_t n,
                                                         int p, float scale,
                                                         float* __restrict__ loss,
                                                         float* __restrict__ dth) {
    using Mdl = typename ModelOf<KIND, float>::T;
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= n) return;
    float th[Mdl::P], g[Mdl::P];
#pragma unroll
    for (int q = 0; q < Mdl::P; ++q) th[q] = th_[(int64_t)q * n + v];
    const YGlob yg{y, n, v, a.M};
    const float wv = w ? w[v] : 1.f;
    float L, gs;
    if (p == 2) {
        DLoss<YGlob, 2> d{yg, 0.f};
        Mdl::template grad<0>(th, d, a, g);
        L = d.loss * (wv * wv);
        gs = -2.f * (wv * wv);
    } else {
        DLoss<YGlob, 1> d{yg, 0.f};
        Mdl::template grad<0>(th, d, a, g);
        L = d.loss * wv;
        gs = wv;
    }
#pragma unroll
    for (int q = 0; q < Mdl::P; ++q) dth[(int64_t)q * n + v] = g[q] * (gs * scale);
    if (loss) loss[v] = L * scale;
}

#define GC_DISPATCH(kind, CALL)                 \
    switch (kind) {                             \
        case MONOEXP_T2S: { constexpr int K = MONOEXP_T2S; CALL; break; } \
        case MONOEXP_R2S: { constexpr int K = MONOEXP_R2S; CALL; break; } \
        case GRE3: { constexpr int K = GRE3; CALL; break; }               \
        case DWI2: { constexpr int K = DWI2; CALL; break; }               \
        case LINEAR3: { constexpr int K = LINEAR3; CALL; break; }         \
        default: return hipErrorInvalidValue;   \
    }

hipError_t model_forward(int kind, const AcqDev& a, const float* theta, int64_t n, float* s,
                         hipStream_t st) {
    if (n == 0) return hipSuccess;
    const dim3 g((unsigned)((n + kBlock - 1) / kBlock));
    GC_DISPATCH(kind, hipLaunchKernelGGL((forward_kernel<K>), g, dim3(kBlock), 0, st, a, theta, n, s))
    return hipGetLastError();
}

hipError_t model_vjp(int kind, const AcqDev& a, const float* theta, int64_t n, const float* ds,
                     float* dtheta, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const dim3 g((unsigned)((n + kBlock - 1) / kBlock));
    GC_DISPATCH(kind, hipLaunchKernelGGL((vjp_kernel<K>), g, dim3(kBlock), 0, st, a, theta, n, ds,
                                         dtheta))
    return hipGetLastError();
}

hipError_t loss_vjp(int kind, const AcqDev& a, const float* theta, const float* y,
                    const float* w, int64_t n, int p, float scale, float* loss, float* dtheta,
                    hipStream_t st) {
    if (n == 0) return hipSuccess;
    const dim3 g((unsigned)((n + kBlock - 1) / kBlock));
    GC_DISPATCH(kind, hipLaunchKernelGGL((loss_vjp_kernel<K>), g, dim3(kBlock), 0, st, a, theta, y,
                                         w, n, p, scale, loss, dtheta))
    return hipGetLastError();
}

// ----------------------------------------------------------------- grid TV
// R = sum over masked forward pairs |u_b - u_a| (FP64 block partials);
// dR[a] = scale * subgradient, 0 outside the mask.
__global__ __launch_bounds__(kBlock) void tv_grid_kernel(int nx, int ny, int nz,
                                                        const uint8_t* __restrict__ mask,
                                                        const float* __restrict__ u, int dim,
                                                        float scale,
                                                        double* __restrict__ partial,
                                                        float* __restrict__ dR) {
    __shared__ double red[kBlock / 64];
    const int64_t G = (int64_t)nx * ny * nz;
    const int64_t a = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double r = 0.0;
    if (a < G) {
        float g = 0.f;
        if (!mask || mask[a]) {
            const int x = (int)(a % nx), y = (int)((a / nx) % ny), z = (int)(a / ((int64_t)nx * ny));
            const int64_t st[3] = {1, nx, (int64_t)nx * ny};
            const bool fw[3] = {x + 1 < nx, y + 1 < ny, dim == 3 && z + 1 < nz};
            const bool bw[3] = {x > 0, y > 0, dim == 3 && z > 0};
            const float ua = u[a];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                if (fw[d] && (!mask || mask[a + st[d]])) {
                    const float diff = u[a + st[d]] - ua;
                    r += fabs((double)diff);
                    g -= sgnf(diff);
                }
                if (bw[d] && (!mask || mask[a - st[d]])) g += sgnf(ua - u[a - st[d]]);
            }
        }
        if (dR) dR[a] = scale * g;
    }
    const double s = block_sum(r, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

hipError_t tv_grid(int nx, int ny, int nz, const uint8_t* mask, const float* u, int dim,
                   float scale, double* partial, int64_t nblk, float* dR, hipStream_t st) {
    hipLaunchKernelGGL(tv_grid_kernel, dim3((unsigned)nblk), dim3(kBlock), 0, st, nx, ny, nz, mask,
                       u, dim, scale, partial, dR);
    return hipGetLastError();
}

// Isotropic grid TV of one full-grid map: the same per-voxel function as the
// fit's step kernel, with neighbour indices taken from the grid and mask.
__global__ __launch_bounds__(kBlock) void tv_grid_iso_kernel(int nx, int ny, int nz,
                                                            const uint8_t* __restrict__ mask,
                                                            const float* __restrict__ u, int dim,
                                                            float scale,
                                                            double* __restrict__ partial,
                                                            float* __restrict__ dR) {
    __shared__ double red[kBlock / 64];
    const int64_t G = (int64_t)nx * ny * nz;
    const int64_t a = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double r = 0.0;
    if (a < G) {
        float g = 0.f;
        if (!mask || mask[a]) {
            const int c[3] = {(int)(a % nx), (int)((a / nx) % ny), (int)(a / ((int64_t)nx * ny))};
            const int ext[3] = {nx, ny, nz};
            const int64_t st[3] = {1, nx, (int64_t)nx * ny};
            // neighbour of grid voxel b (coordinates cb) along axis e in
            // direction dir, or -1 (outside the grid or mask; z only in 3D)
            auto at = [&](int64_t b, const int* cb, int e, int dir) -> int32_t {
                if (e == 2 && dim != 3) return -1;
                const int q = cb[e] + dir;
                if (q < 0 || q >= ext[e]) return -1;
                const int64_t k = b + dir * st[e];
                return (!mask || mask[k]) ? (int32_t)k : -1;
            };
            int32_t nb[6], dg[3][3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                nb[2 * d] = at(a, c, d, -1);
                nb[2 * d + 1] = at(a, c, d, +1);
            }
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                int cb[3] = {c[0], c[1], c[2]};
                cb[d] -= 1;
#pragma unroll
                for (int e = 0; e < 3; ++e)
                    dg[d][e] = (e != d && nb[2 * d] >= 0) ? at(nb[2 * d], cb, e, +1) : -1;
            }
            float R = 0.f;
            g = tv_iso_at(u, u[a], nb, dg, R);
            r = (double)R;
        }
        if (dR) dR[a] = scale * g;
    }
    const double s = block_sum(r, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

hipError_t tv_grid_iso(int nx, int ny, int nz, const uint8_t* mask, const float* u, int dim,
                       float scale, double* partial, int64_t nblk, float* dR, hipStream_t st) {
    hipLaunchKernelGGL(tv_grid_iso_kernel, dim3((unsigned)nblk), dim3(kBlock), 0, st, nx, ny, nz,
                       mask, u, dim, scale, partial, dR);
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void tv_graph_kernel(int64_t n,
                                                         const int64_t* __restrict__ rowptr,
                                                         const int32_t* __restrict__ col,
                                                         const float* __restrict__ u, float scale,
                                                         double* __restrict__ partial,
                                                         float* __restrict__ dR) {
    __shared__ double red[kBlock / 64];
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double r = 0.0;
    if (v < n) {
        float R = 0.f;
        const float g = tv_graph_at(u, u[v], rowptr, col, v, R);
        r = (double)R;
        if (dR) dR[v] = scale * g;
    }
    const double s = block_sum(r, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

hipError_t tv_graph(int64_t n, const int64_t* rowptr, const int32_t* col, const float* u,
                    float scale, double* partial, int64_t nblk, float* dR, hipStream_t st) {
    hipLaunchKernelGGL(tv_graph_kernel, dim3((unsigned)nblk), dim3(kBlock), 0, st, n, rowptr, col,
                       u, scale, partial, dR);
    return hipGetLastError();
}

// Adjacency check before any kernel follows it: row offsets start at 0, do
// not decrease and end at nnz; every neighbour index lies in [0, n).  The two
// checks read only rowptr[0..n] and col[0..nnz), whatever those hold.
__global__ __launch_bounds__(kBlock) void check_graph_rows_kernel(int64_t n, int64_t nnz,
                                                                 const int64_t* __restrict__ rowptr,
                                                                 int* __restrict__ flag) {
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v > n) return;
    const int64_t k = rowptr[v];
    bool bad = k < 0 || k > nnz || (v == 0 && k != 0) || (v == n && k != nnz);
    if (v < n && rowptr[v + 1] < k) bad = true;
    if (bad) atomicOr(flag, 1);
}

__global__ __launch_bounds__(kBlock) void check_graph_cols_kernel(int64_t nnz, int64_t n,
                                                                 const int32_t* __restrict__ col,
                                                                 int* __restrict__ flag) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= nnz) return;
    if (col[k] < 0 || (int64_t)col[k] >= n) atomicOr(flag, 1);
}

hipError_t check_graph(int64_t n, int64_t nnz, const int64_t* rowptr, const int32_t* col,
                       int* flag, hipStream_t st) {
    hipLaunchKernelGGL(check_graph_rows_kernel, dim3((unsigned)((n + kBlock) / kBlock)),
                       dim3(kBlock), 0, st, n, nnz, rowptr, flag);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nnz == 0) return e;
    hipLaunchKernelGGL(check_graph_cols_kernel, dim3((unsigned)((nnz + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, st, nnz, n, col, flag);
    return hipGetLastError();
}

}  // namespace gc

namespace gc {

// ----------------------------------------------------------------- stopping
// Loss of iteration t from the block partials (fixed order, FP64 with
// compensation), then the stopping rules of the fit:
//   reason 1: L_t < tol;   reason 2: |least-squares slope of the last W
//   losses against the iteration index| < conv, once t >= W.
// stop[0] = stopping iteration (0 while running), stop[1] = reason.  Once
// set, later iterations' kernels see stop[0] != 0 and do nothing.
template <typename T>
__global__ __launch_bounds__(kBlock) void fit_loss_stop_kernel(const T* __restrict__ partial,
                                                              int64_t count,
                                                              double* __restrict__ hist, int t,
                                                              double tol, double conv, int W,
                                                              int* __restrict__ stop) {
    if (stop[0] != 0) return;
    __shared__ double ss[kBlock], cc[kBlock];
    double s = 0.0, comp = 0.0;
    for (int64_t i = threadIdx.x; i < count; i += kBlock) {
        const double x = (double)partial[i];
        const double u = s + x;
        comp += fabs(s) >= fabs(x) ? (s - u) + x : (x - u) + s;
        s = u;
    }
    ss[threadIdx.x] = s;
    cc[threadIdx.x] = comp;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            const double a = ss[threadIdx.x], b = ss[threadIdx.x + o];
            const double u = a + b;
            cc[threadIdx.x] += cc[threadIdx.x + o] + (fabs(a) >= fabs(b) ? (a - u) + b : (b - u) + a);
            ss[threadIdx.x] = u;
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double L = ss[0] + cc[0];
    hist[t - 1] = L;
    if (L < tol) {
        stop[0] = t;
        stop[1] = 1;
        return;
    }
    if (conv > 0.0 && W > 1 && t >= W) {
        double mx = 0.0, my = 0.0;
        for (int i = 0; i < W; ++i) {
            mx += (double)(t - W + 1 + i);
            my += hist[t - W + i];
        }
        mx /= W;
        my /= W;
        double sxy = 0.0, sxx = 0.0;
        for (int i = 0; i < W; ++i) {
            const double dx = (double)(t - W + 1 + i) - mx;
            sxy += dx * (hist[t - W + i] - my);
            sxx += dx * dx;
        }
        if (fabs(sxy / sxx) < conv) {
            stop[0] = t;
            stop[1] = 2;
        }
    }
}

hipError_t fit_loss_stop(const float* partial, int64_t count, double* hist, int t, double tol,
                         double conv, int W, int* stop, hipStream_t s) {
    hipLaunchKernelGGL(fit_loss_stop_kernel<float>, dim3(1), dim3(kBlock), 0, s, partial, count,
                       hist, t, tol, conv, W, stop);
    return hipGetLastError();
}

hipError_t fit_loss_stop_f64(const double* partial, int64_t count, double* hist, int t,
                             double tol, double conv, int W, int* stop, hipStream_t s) {
    hipLaunchKernelGGL(fit_loss_stop_kernel<double>, dim3(1), dim3(kBlock), 0, s, partial, count,
                       hist, t, tol, conv, W, stop);
    return hipGetLastError();
}

// theta = lb + (ub - lb) u, compacted [P][n]
struct ThetaMap {
    int P;
    float lb[kMaxP], rng[kMaxP];
};
__global__ __launch_bounds__(kBlock) void fit_theta_kernel(ThetaMap tm, const float* __restrict__ u,
                                                          int64_t n, float* __restrict__ out) {
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= n) return;
    for (int p = 0; p < tm.P; ++p) out[(int64_t)p * n + v] = tm.lb[p] + tm.rng[p] * u[(int64_t)p * n + v];
}

hipError_t fit_theta(int P, const float* lb, const float* rng, const float* u, int64_t n,
                     float* out, hipStream_t s) {
    if (n == 0) return hipSuccess;
    ThetaMap tm{};
    tm.P = P;
    for (int p = 0; p < P; ++p) {
        tm.lb[p] = lb[p];
        tm.rng[p] = rng[p];
    }
    hipLaunchKernelGGL(fit_theta_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       s, tm, u, n, out);
    return hipGetLastError();
}

// theta = lb + (ub - lb) u from an FP64 iterate, rounded once to FP32
struct ThetaMapF64 {
    int P;
    double lb[kMaxP], rng[kMaxP];
};
__global__ __launch_bounds__(kBlock) void fit_theta_f64_kernel(ThetaMapF64 tm,
                                                              const double* __restrict__ u,
                                                              int64_t n, float* __restrict__ out) {
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= n) return;
    for (int p = 0; p < tm.P; ++p)
        out[(int64_t)p * n + v] = (float)(tm.lb[p] + tm.rng[p] * u[(int64_t)p * n + v]);
}

hipError_t fit_theta_f64(int P, const double* lb, const double* rng, const double* u, int64_t n,
                         float* out, hipStream_t s) {
    if (n == 0) return hipSuccess;
    ThetaMapF64 tm{};
    tm.P = P;
    for (int p = 0; p < P; ++p) {
        tm.lb[p] = lb[p];
        tm.rng[p] = rng[p];
    }
    hipLaunchKernelGGL(fit_theta_f64_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, s, tm, u, n, out);
    return hipGetLastError();
}

__global__ void f32_to_f64_kernel(const float* __restrict__ a, double* __restrict__ b, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) b[i] = (double)a[i];
}
hipError_t f32_to_f64(const float* a, double* b, int64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(f32_to_f64_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       s, a, b, n);
    return hipGetLastError();
}

}  // namespace gc
