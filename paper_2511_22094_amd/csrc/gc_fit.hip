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
    __device__ __forceinline__ float re(int m) const { return y[(int64_t)m * n + v]; }
    __device__ __forceinline__ float im(int m) const { return y[(int64_t)(M + m) * n + v]; }
};

// dLoss/ds for |w (y - s)|^p per component; accumulates the unscaled loss.
template <class Y> struct DLoss {
    const Y& y;
    float w;
    int p;
    float loss;
    __device__ __forceinline__ float one(float ym, float s) {
        const float r = ym - s;
        if (p == 2) {
            const float wr = w * r;
            loss += wr * wr;
            return -2.f * w * wr;
        }
        loss += fabsf(w * r);
        return r > 0.f ? -w : (r < 0.f ? w : 0.f);
    }
    __device__ __forceinline__ float re(int m, float s) { return one(y.re(m), s); }
    __device__ __forceinline__ float im(int m, float s) { return one(y.im(m), s); }
};

// upstream gradient ds read from HBM (vector-Jacobian product)
struct DGiven {
    const float* ds;
    int64_t n, v;
    int M;
    __device__ __forceinline__ float re(int m, float) const { return ds[(int64_t)m * n + v]; }
    __device__ __forceinline__ float im(int m, float) const {
        return ds[(int64_t)(M + m) * n + v];
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
    DLoss<Y> d{y, w, J.loss_p, 0.f};
    Mdl::template grad<MAXM>(th, d, J.acq, g);
#pragma unroll
    for (int p = 0; p < P; ++p) gu[p] = J.rng[p] * (g[p] * J.scale_data);
    return d.loss * J.scale_data;
}

__device__ __forceinline__ float sgnf(float x) { return x > 0.f ? 1.f : (x < 0.f ? -1.f : 0.f); }

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

int fit_pick_maxm(int kind, int M) {
    if (kind == GRE3) return M <= 12 ? 12 : (M <= 24 ? 24 : (M <= 32 ? 32 : 0));
    if (kind == DWI2) return M <= 32 ? 32 : (M <= 64 ? 64 : (M <= 96 ? 96 : 0));
    return M <= 12 ? 12 : (M <= 16 ? 16 : (M <= 32 ? 32 : 0));
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
        case DWI2: return fused_pick<DWI2, 32, 64, 96>(maxm, jobs, map, nblk, s);
        case LINEAR3: return fused_pick<LINEAR3, 12, 16, 32>(maxm, jobs, map, nblk, s);
    }
    return hipErrorInvalidValue;
}

// ----------------------------------------------------------------- step
// One iteration for every voxel of every active job.  With xcd_remap the
// hardware block index is permuted so that each XCD (blocks are dealt
// round-robin over the 8 XCDs) processes a contiguous range of voxels and
// the TV neighbour reads of adjacent blocks hit the same L2.
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
            u[p] = J.u_in[(int64_t)p * n + v];
            m[p] = J.m[(int64_t)p * n + v];
            s2[p] = J.v[(int64_t)p * n + v];
        }
        const float w = J.w ? J.w[v] : 1.f;
        const YGlob yg{J.y, n, v, J.acq.M};
        contrib = data_grad<Mdl, 0>(J, u, yg, w, gu);
        if (J.tv_mask) {
            float R = 0.f;
#pragma unroll
            for (int p = 0; p < P; ++p) {
                if (!((J.tv_mask >> p) & 1u)) continue;
                const float* up = J.u_in + (int64_t)p * n;
                float g = 0.f;
#pragma unroll
                for (int d = 0; d < 6; ++d) {
                    const int32_t nb = J.nbr[(int64_t)d * n + v];
                    if (nb < 0) continue;
                    const float un = up[nb];
                    if (d & 1) {          // forward neighbour: pair (v, nb)
                        const float diff = un - u[p];
                        R += fabsf(diff);
                        g -= sgnf(diff);
                    } else {              // backward neighbour: pair (nb, v)
                        g += sgnf(u[p] - un);
                    }
                }
                gu[p] += J.scale_tv * g;
            }
            contrib += J.scale_tv * R;
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
    DLoss<YGlob> d{yg, w ? w[v] : 1.f, p, 0.f};
    Mdl::template grad<0>(th, d, a, g);
#pragma unroll
    for (int q = 0; q < Mdl::P; ++q) dth[(int64_t)q * n + v] = g[q] * scale;
    if (loss) loss[v] = d.loss * scale;
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
