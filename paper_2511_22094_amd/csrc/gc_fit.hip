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
template <class Y, int LP> struct DLoss {
    const Y& y;
    float loss;
    __device__ __forceinline__ float one(float ym, float s) {
        const float r = ym - s;
        if constexpr (LP == 2) {
            loss += r * r;
            return r;
        } else {
            loss += fabsf(r);
            return r > 0.f ? -1.f : (r < 0.f ? 1.f : 0.f);
        }
    }
    __device__ __forceinline__ float re(int m, float s) { return one(y.re(m), s); }
    __device__ __forceinline__ float im(int m, float s) { return one(y.im(m), s); }
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

// One optimiser update of one coordinate in u units, then the projection.
__device__ __forceinline__ float opt_update(const FitJob& J, float u, float g, float& m,
                                            float& v, float c1, float c2) {
    float un;
    if (J.optimizer == 0) {
        m = J.beta1 * m + J.omb1 * g;
        v = J.beta2 * v + J.omb2 * g * g;
        un = u - J.lr * (m * c1) / (sqrtf(v * c2) + J.eps);
    } else if (J.optimizer == 1) {
        m = J.momentum * m - J.lr * g;
        un = u + m;
    } else {
        v = J.rho * v + J.omrho * g * g;
        un = u - J.lr * g / (sqrtf(v) + J.eps);
    }
    return fminf(fmaxf(un, 0.f), 1.f);
}

// data term of one voxel: loss (scaled) and dL/du (scaled) at iterate u
template <class Mdl, int MAXM, class Y>
__device__ __forceinline__ float data_grad(const FitJob& J, const float* u, const Y& y, float w,
                                           float* gu) {
    constexpr int P = Mdl::P;
    float th[P], g[P];
#pragma unroll
    for (int p = 0; p < P; ++p) th[p] = J.lb[p] + J.rng[p] * u[p];
    float loss, gs;   // loss and gradient factors of the voxel weight
    if (J.loss_p == 2) {
        DLoss<Y, 2> d{y, 0.f};
        Mdl::template grad<MAXM>(th, d, J.acq, g);
        loss = d.loss * (w * w);
        gs = -2.f * (w * w);
    } else {
        DLoss<Y, 1> d{y, 0.f};
        Mdl::template grad<MAXM>(th, d, J.acq, g);
        loss = d.loss * w;
        gs = w;
    }
#pragma unroll
    for (int p = 0; p < P; ++p) gu[p] = J.rng[p] * (g[p] * (gs * J.scale_data));
    return loss * J.scale_data;
}

__device__ __forceinline__ float sgnf(float x) { return x > 0.f ? 1.f : (x < 0.f ? -1.f : 0.f); }

// Anisotropic grid TV at voxel v for one map up (iterate t-1): the pairs
// (v, forward neighbour) add |difference| to R; the subgradient collects the
// pairs in which v takes part.  nb = (x-, x+, y-, y+, z-, z+), -1 = none.
// Neighbour values are read unconditionally (a missing neighbour, index -1,
// reads element 0 and is then ignored) so that all reads of a voxel are in
// flight together instead of one conditional read waiting after another.
__device__ __forceinline__ float tv_aniso_at(const float* __restrict__ up, float uv,
                                             const int32_t (&nb)[6], float& R) {
    float un[6];
#pragma unroll
    for (int d = 0; d < 6; ++d) un[d] = gload(up)[nb[d] >= 0 ? nb[d] : 0];
    float g = 0.f;
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        const bool in = nb[d] >= 0;
        if (d & 1) {          // forward neighbour: pair (v, nb)
            const float diff = in ? un[d] - uv : 0.f;
            R += fabsf(diff);
            g -= sgnf(diff);
        } else {              // backward neighbour: pair (nb, v)
            g += in ? sgnf(uv - un[d]) : 0.f;
        }
    }
    return g;
}

// Isotropic grid TV at voxel v: R gains v's own norm G_v of its forward
// differences; the subgradient is -sum_d D_d / G_v from that norm plus, for
// each backward neighbour b, (u_v - u_b) / G_b from b's norm.  G_b needs b's
// other forward neighbours: dg[d][e] is the forward neighbour along axis e of
// the backward neighbour along axis d (dg[d][d] is v itself, unused).
__device__ __forceinline__ float tv_iso_at(const float* __restrict__ up, float uv,
                                           const int32_t (&nb)[6], const int32_t (&dg)[3][3],
                                           float& R) {
    // all neighbour values first (unconditional reads, see tv_aniso_at)
    float uf[3], ubk[3], ud[3][3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        uf[d] = gload(up)[nb[2 * d + 1] >= 0 ? nb[2 * d + 1] : 0];
        ubk[d] = gload(up)[nb[2 * d] >= 0 ? nb[2 * d] : 0];
#pragma unroll
        for (int e = 0; e < 3; ++e) ud[d][e] = gload(up)[dg[d][e] >= 0 ? dg[d][e] : 0];
    }
    float D[3], ss = 0.f;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        D[d] = nb[2 * d + 1] >= 0 ? uf[d] - uv : 0.f;
        ss += D[d] * D[d];
    }
    const float Gv = sqrtf(ss);
    R += Gv;
    float g = 0.f;
    if (Gv > 0.f) {
#pragma unroll
        for (int d = 0; d < 3; ++d) g -= D[d] / Gv;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (nb[2 * d] < 0) continue;
        const float ub = ubk[d];
        const float Dv = uv - ub;
        float sb = 0.f;
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            if (e == d) {
                sb += Dv * Dv;
            } else if (dg[d][e] >= 0) {
                const float t = ud[d][e] - ub;
                sb += t * t;
            }
        }
        const float Gb = sqrtf(sb);
        if (Gb > 0.f) g += Dv / Gb;
    }
    return g;
}

// Graph TV at vertex v: R gains sum_{j in N(v)} |u_v - u_j|; with a symmetric
// adjacency every edge also appears from j's side, so the subgradient is
// 2 sum_j sign(u_v - u_j).
__device__ __forceinline__ float tv_graph_at(const float* __restrict__ up, float uv,
                                             const int64_t* __restrict__ rowptr,
                                             const int32_t* __restrict__ col, int64_t v,
                                             float& R) {
    float g = 0.f;
    const int64_t k1 = rowptr[v + 1];
    for (int64_t k = rowptr[v]; k < k1; ++k) {
        const float diff = uv - up[col[k]];
        R += fabsf(diff);
        g += 2.f * sgnf(diff);
    }
    return g;
}

// Prior term (Eq. 6) of one voxel: scale_prior |(theta - mu) / sigma| summed
// over the parameters of prior_mask, added to the loss (returned) and its
// subgradient in u units to gu.
template <int P>
__device__ __forceinline__ float prior_at(const FitJob& J, const float* u, const float* mu,
                                          const float* sg, float* gu) {
    float R = 0.f;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        if (!((J.prior_mask >> p) & 1u)) continue;
        const float th = J.lb[p] + J.rng[p] * u[p];
        const float r = (th - mu[p]) / sg[p];
        R += fabsf(r);
        gu[p] += J.scale_prior * sgnf(r) * (J.rng[p] / sg[p]);
    }
    return J.scale_prior * R;
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
    hipLaunchKernelGGL((fit_fused_kernel<KIND, MAXM>), dim3(nblk), dim3(kBlock), 0, s, jobs, map);
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
template <int KIND>
__global__ __launch_bounds__(kBlock) void fit_step_kernel(const FitJob* __restrict__ jobs,
                                                         const BlkMap* __restrict__ map,
                                                         int nblk, int xcd_remap) {
    using Mdl = typename ModelOf<KIND, float>::T;
    constexpr int P = Mdl::P;
    __shared__ float red[kBlock / 64];
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
    float contrib = 0.f;
    if (live) {
        float u[P], m[P], s2[P], gu[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            u[p] = gload(J.u_in)[(int64_t)p * n + v];
        }
        const float w = J.w ? gload(J.w)[v] : 1.f;
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
        contrib = data_grad<Mdl, 0>(J, u, yg, w, gu);
        if (J.tv_mask) {
            float R = 0.f;
#pragma unroll
            for (int p = 0; p < P; ++p) {
                if (!((J.tv_mask >> p) & 1u)) continue;
                const float* up = J.u_in + (int64_t)p * n;
                float g;
                if (J.tv_kind == 0) g = tv_aniso_at(up, u[p], nb, R);
                else if (J.tv_kind == 1) g = tv_iso_at(up, u[p], nb, dg, R);
                else g = tv_graph_at(up, u[p], J.g_rowptr, J.g_col, v, R);
                gu[p] += J.scale_tv * g;
            }
            contrib += J.scale_tv * R;
        }
        if (J.prior_mask) {
            float pmu[P], psg[P];
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const bool on = (J.prior_mask >> p) & 1u;
                pmu[p] = on ? gload(J.mu)[(int64_t)p * n + v] : 0.f;
                psg[p] = on ? gload(J.sigma)[(int64_t)p * n + v] : 1.f;
            }
            contrib += prior_at<P>(J, u, pmu, psg, gu);
        }
        // the optimiser state is read only now, so that it holds no registers
        // through the data term (84 instead of 96 VGPRs; measured 1 % faster
        // than reading it with the iterate, identical results)
#pragma unroll
        for (int p = 0; p < P; ++p) {
            m[p] = gload(J.m)[(int64_t)p * n + v];
            s2[p] = gload(J.v)[(int64_t)p * n + v];
        }
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const float un = opt_update(J, u[p], gu[p], m[p], s2[p], J.c1, J.c2);
            J.u_out[(int64_t)p * n + v] = un;
            J.m[(int64_t)p * n + v] = m[p];
            J.v[(int64_t)p * n + v] = s2[p];
        }
    }
    if (J.record) {
        const float s = block_sum(contrib, red);
        if (threadIdx.x == 0) J.partial[b - J.blk0] = s;
    }
}

hipError_t fit_step(int kind, const FitJob* jobs, const BlkMap* map, int nblk, int xcd_remap,
                    hipStream_t s) {
#define GC_STEP(K)                                                                      \
    case K:                                                                             \
        hipLaunchKernelGGL((fit_step_kernel<K>), dim3(nblk), dim3(kBlock), 0, s, jobs, map, \
                           nblk, xcd_remap);                                            \
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
__global__ __launch_bounds__(kBlock) void fit_loss_stop_kernel(const float* __restrict__ partial,
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
    hipLaunchKernelGGL(fit_loss_stop_kernel, dim3(1), dim3(kBlock), 0, s, partial, count, hist, t,
                       tol, conv, W, stop);
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
