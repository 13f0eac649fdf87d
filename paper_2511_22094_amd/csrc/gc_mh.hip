// Fused Metropolis-Hastings kernels (paper §2.2.2): one lane per (voxel,
// chain).  A launch runs a chunk of iterations entirely in registers --
// random draws, proposal, bounds test, forward model, likelihood, accept /
// reject, retention and FP64 Welford moments -- and leaves the chain state
// in HBM for the next chunk.  The same kernels serve one job or many (the
// block work-list maps blocks to jobs).
#include "gc_internal.hpp"
#include "gc_timing.hpp"

namespace gc {

namespace {

// measured data held in registers (compile-time indices only)
template <int MAXM, bool CPLX> struct YReg {
    float r[MAXM];
    float i[CPLX ? MAXM : 1];
    __device__ __forceinline__ float re(int m) const { return r[m]; }
    __device__ __forceinline__ float im(int m) const { return i[CPLX ? m : 0]; }
};

// measured data staged in LDS for the chains of one voxel (any measurement
// count): real parts, then imaginary parts
struct YShared {
    const float* p;
    int M;
    __device__ __forceinline__ float re(int m) const { return p[m]; }
    __device__ __forceinline__ float im(int m) const { return p[M + m]; }
};

// measured data read from HBM (any measurement count)
struct YGlob {
    const float* y;
    int64_t n;
    int64_t v;
    int M;
    __device__ __forceinline__ float re(int m) const { return gload(y)[(int64_t)m * n + v]; }
    __device__ __forceinline__ float im(int m) const { return gload(y)[(int64_t)(M + m) * n + v]; }
};

template <typename R> __device__ __forceinline__ R lbR(const MhJob& J, int p);
template <> __device__ __forceinline__ float lbR<float>(const MhJob& J, int p) { return J.lb[p]; }
template <> __device__ __forceinline__ double lbR<double>(const MhJob& J, int p) { return J.lbd[p]; }
template <typename R> __device__ __forceinline__ R ubR(const MhJob& J, int p);
template <> __device__ __forceinline__ float ubR<float>(const MhJob& J, int p) { return J.ub[p]; }
template <> __device__ __forceinline__ double ubR<double>(const MhJob& J, int p) { return J.ubd[p]; }
template <typename R> __device__ __forceinline__ R stepR(const MhJob& J, int p);
template <> __device__ __forceinline__ float stepR<float>(const MhJob& J, int p) { return J.step[p]; }
template <> __device__ __forceinline__ double stepR<double>(const MhJob& J, int p) { return J.stepd[p]; }
template <typename R> __device__ __forceinline__ R x0R(const MhJob& J, int p);
template <> __device__ __forceinline__ float x0R<float>(const MhJob& J, int p) { return J.x0c[p]; }
template <> __device__ __forceinline__ double x0R<double>(const MhJob& J, int p) { return J.x0cd[p]; }
template <typename R> __device__ __forceinline__ R inv2s2R(const MhJob& J);
template <> __device__ __forceinline__ float inv2s2R<float>(const MhJob& J) { return J.inv2s2; }
template <> __device__ __forceinline__ double inv2s2R<double>(const MhJob& J) { return J.inv2s2d; }

// First iteration t >= max(t0, burnin) with (t - burnin + 1) % thin == 0.
__device__ __forceinline__ int first_keep(int t0, int burnin, int thin) {
    int t = t0 > burnin ? t0 : burnin;
    int r = (t - burnin + 1) % thin;
    return r == 0 ? t : t + (thin - r);
}

}  // namespace

// --------------------------------------------------------------------------
// Initial state: midpoint / given constant, uniform in the box (Philox with
// purpose 1, iteration 0), or a per-voxel map; log-likelihood of the start.
// --------------------------------------------------------------------------
template <int KIND, typename R>
__global__ __launch_bounds__(kBlock) void mh_init_kernel(const MhJob* __restrict__ jobs,
                                                        const BlkMap* __restrict__ map) {
    using Mdl = typename ModelOf<KIND, R>::T;
    constexpr int P = Mdl::P;
    const BlkMap bm = map[blockIdx.x];
    const MhJob& J = jobs[bm.job];
    const int64_t n = J.n, NL = n * J.C;
    const int64_t L = bm.lane0 + threadIdx.x;
    if (L >= NL) return;
    const int64_t v = L % n;
    const int c = (int)(L / n);
    R th[P];
    if (J.init_state) {
#pragma unroll
        for (int p = 0; p < P; ++p) th[p] = (R)J.init_state[(int64_t)p * NL + L];
    } else if (J.x0_mode == 1) {
#pragma unroll
        for (int b = 0; b < (P + 3) / 4; ++b) {
            U4 o = philox4x32_10(U4{(uint32_t)v, (uint32_t)c | (1u << 16), 0u, (uint32_t)b},
                                 J.k0, J.k1);
            uint32_t w[4] = {o.x, o.y, o.z, o.w};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                int p = 4 * b + i;
                if (p < P)
                    th[p] = lbR<R>(J, p) + (ubR<R>(J, p) - lbR<R>(J, p)) * uniform01<R>(w[i]);
            }
        }
    } else if (J.x0map) {
#pragma unroll
        for (int p = 0; p < P; ++p) th[p] = (R)J.x0map[(int64_t)p * n + v];
    } else {
#pragma unroll
        for (int p = 0; p < P; ++p) th[p] = x0R<R>(J, p);
    }
    const R w = J.w ? (R)J.w[v] : (R)1;
    YGlob y{J.y, n, v, J.acq.M};
    // a resumed chain carries its log-likelihood over unchanged (bit for bit)
    const R ll = J.init_logl ? (R)J.init_logl[L]
                             : -(inv2s2R<R>(J) * w * w) * Mdl::template sse<0>(th, y, J.acq);
    R* TH = (R*)J.th;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        TH[(int64_t)p * NL + L] = th[p];
        if (J.mean) {
            J.mean[(int64_t)p * NL + L] = 0.0;
            J.m2[(int64_t)p * NL + L] = 0.0;
        }
    }
    ((R*)J.ll)[L] = ll;
    J.acc[L] = 0;
}

// --------------------------------------------------------------------------
// A chunk of MH iterations [t0, t1) for every (voxel, chain) lane.
//
// SHARED (data read from memory, chain count C dividing the block size): the
// block with lanes [lane0, lane0 + kBlock) takes instead the C chains of the
// kBlock / C consecutive voxels from lane0 / C on, chain fastest, and stages
// those voxels' data once in LDS, where the C chains of a voxel read them.
// Every (voxel, chain) pair is still run by exactly one lane of the launch,
// with the same state and random stream, so results do not depend on SHARED.
// --------------------------------------------------------------------------
template <int KIND, typename R, int MAXM, int EXACT = 0, int RECUR = kRecurRuntime,
          bool SHARED = false>
__global__ __launch_bounds__(kBlock) void mh_chunk_kernel(const MhJob* __restrict__ jobs,
                                                         const BlkMap* __restrict__ map) {
    using Mdl = typename ModelOf<KIND, R>::T;
    constexpr int P = Mdl::P;
    constexpr bool CPLX = Mdl::kComplex;
    const BlkMap bm = map[blockIdx.x];
    const MhJob& J = jobs[bm.job];
    const int64_t n = J.n, NL = n * J.C;
    int64_t L, v;
    int c;
    YShared ys{nullptr, J.acq.M};
    if constexpr (SHARED) {
        // [kBlock / C][Ms]: a voxel's Meff values, rows padded to an odd
        // length Ms so that the voxels a wave reads at one measurement index
        // fall in different LDS banks (an even row of 96 floats put all of
        // them in one bank)
        extern __shared__ float ysm[];
        const int C = J.C, vb = kBlock / C, Me = CPLX ? 2 * J.acq.M : J.acq.M;
        const int Ms = Me | 1;
        const int64_t v0 = bm.lane0 / C;
        for (int idx = threadIdx.x; idx < vb * Me; idx += kBlock) {
            const int j = idx / vb, a = idx % vb;   // row j, voxel v0 + a: coalesced
            ysm[a * Ms + j] = v0 + a < n ? gload(J.y)[(int64_t)j * n + v0 + a] : 0.f;
        }
        __syncthreads();
        v = v0 + threadIdx.x / C;
        c = (int)(threadIdx.x % C);
        if (v >= n) return;
        L = (int64_t)c * n + v;
        ys.p = ysm + (threadIdx.x / C) * Ms;
    } else {
        L = bm.lane0 + threadIdx.x;
        if (L >= NL) return;
        v = L % n;
        c = (int)(L / n);
    }
    const AcqDev acq = J.acq;

    // chain state
    R* TH = (R*)J.th;
    R th[P];
#pragma unroll
    for (int p = 0; p < P; ++p) th[p] = TH[(int64_t)p * NL + L];
    R ll = ((R*)J.ll)[L];
    int32_t acc = J.acc[L];
    double mu[P], m2[P];
    const bool welford = J.mean != nullptr;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        mu[p] = welford ? J.mean[(int64_t)p * NL + L] : 0.0;
        m2[p] = welford ? J.m2[(int64_t)p * NL + L] : 0.0;
    }
    R lo[P], hi[P], st[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        lo[p] = lbR<R>(J, p);
        hi[p] = ubR<R>(J, p);
        st[p] = stepR<R>(J, p);
        // keep the upper bounds in vector registers: the box test takes both
        // bounds in one instruction, which reads at most one scalar register
        if constexpr (sizeof(R) == 4) asm volatile("" : "+v"(hi[p]));
    }
    const R w = J.w ? (R)J.w[v] : (R)1;
    const R nscale = -(inv2s2R<R>(J) * w * w);

    // measured data
    YReg<(MAXM > 0 ? MAXM : 1), CPLX> yr;
    if constexpr (MAXM > 0) {
#pragma unroll
        for (int m = 0; m < MAXM; ++m) {
            const bool in = EXACT || m < acq.M;
            yr.r[m] = in ? J.y[(int64_t)m * n + v] : 0.f;
            if (CPLX) yr.i[m] = in ? J.y[(int64_t)((EXACT ? MAXM : acq.M) + m) * n + v] : 0.f;
        }
    }
    const YGlob yg{J.y, n, v, acq.M};

    const int t0 = J.t0, t1 = J.t1, B = J.burnin, thin = J.thin;
    int keep_t = first_keep(t0, B, thin);
    const uint32_t vv = (uint32_t)v, cc = (uint32_t)c;
    const uint32_t k0 = J.k0, k1 = J.k1;
    for (int t = t0; t < t1; ++t) {
        R z[P], u;
        mh_draws<R, P>(vv, cc, (uint32_t)t, k0, k1, z, u);
        R thp[P], the[P];
        bool inb = true;
#pragma unroll
        for (int p = 0; p < P; ++p) {
            thp[p] = th[p] + st[p] * z[p];
            inb &= in_box(thp[p], lo[p], hi[p]);
        }
        // out-of-box proposals are rejected; evaluate at the current state
        // instead of branching so the wave stays converged
#pragma unroll
        for (int p = 0; p < P; ++p) the[p] = inb ? thp[p] : th[p];
        R sse;
        if constexpr (MAXM > 0) sse = Mdl::template sse<MAXM, EXACT, RECUR>(the, yr, acq);
        else if constexpr (SHARED) sse = Mdl::template sse<0>(the, ys, acq);
        else sse = Mdl::template sse<0>(the, yg, acq);
        const R llp = nscale * sse;
        const bool a = inb && (Math<R>::ln(u) < llp - ll);
#pragma unroll
        for (int p = 0; p < P; ++p) th[p] = a ? thp[p] : th[p];
        ll = a ? llp : ll;
        acc += a ? 1 : 0;
        if (t == keep_t) {   // uniform across the job
            keep_t += thin;
            const int k = (t - B + 1) / thin - J.k_base;   // 1-based, this call
            const double inv = 1.0 / (double)k;
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const double x = (double)th[p];
                const double d = x - mu[p];
                mu[p] += d * inv;
                m2[p] += d * (x - mu[p]);
            }
            if (J.samples) {
                const int ks = (t - B + 1) / thin - J.s_base - 1;   // slot in the buffer
#pragma unroll
                for (int p = 0; p < P; ++p)
                    J.samples[(((int64_t)c * J.s_K + ks) * P + p) * n + v] = (float)th[p];
            }
        }
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
        TH[(int64_t)p * NL + L] = th[p];
        if (welford) {
            J.mean[(int64_t)p * NL + L] = mu[p];
            J.m2[(int64_t)p * NL + L] = m2[p];
        }
    }
    ((R*)J.ll)[L] = ll;
    J.acc[L] = acc;
}

// --------------------------------------------------------------------------
// Pool the chains of each voxel (equal sample counts K per chain):
//   mean = average of chain means,
//   M2   = sum of chain M2 + K sum_c (mean_c - mean)^2,  std = sqrt(M2/(C K - 1)).
// vmap blocks cover voxels (not lanes); outputs are compacted [P][n].
// --------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void mh_finalize_kernel(const MhJob* __restrict__ jobs,
                                                            const BlkMap* __restrict__ vmap,
                                                            double* __restrict__ out_mean,
                                                            double* __restrict__ out_std) {
    const BlkMap bm = vmap[blockIdx.x];
    const MhJob& J = jobs[bm.job];
    const int64_t n = J.n, NL = n * J.C;
    const int64_t v = bm.lane0 + threadIdx.x;
    if (v >= n) return;
    const int C = J.C, K = J.K, P = J.P;
    for (int p = 0; p < P; ++p) {
        double s = 0.0;
        for (int c = 0; c < C; ++c) s += J.mean[(int64_t)p * NL + (int64_t)c * n + v];
        const double mean = s / (double)C;
        double M2 = 0.0;
        for (int c = 0; c < C; ++c) {
            const double d = J.mean[(int64_t)p * NL + (int64_t)c * n + v] - mean;
            M2 += J.m2[(int64_t)p * NL + (int64_t)c * n + v] + (double)K * d * d;
        }
        out_mean[(int64_t)p * n + v] = mean;
        out_std[(int64_t)p * n + v] = sqrt(M2 / (double)(C * K - 1));
    }
}

// ---------------------------------------------------------------- dispatch
template <int KIND, typename R>
static hipError_t init_t(const MhJob* jobs, const BlkMap* map, int nblk, hipStream_t s) {
    hipLaunchKernelGGL((mh_init_kernel<KIND, R>), dim3(nblk), dim3(kBlock), 0, s, jobs, map);
    return hipGetLastError();
}

hipError_t mh_init(int kind, bool fp64, const MhJob* jobs, const BlkMap* map, int nblk,
                   hipStream_t s) {
#define GC_INIT(K)                                                              \
    case K:                                                                     \
        return fp64 ? init_t<K, double>(jobs, map, nblk, s) : init_t<K, float>(jobs, map, nblk, s);
    switch (kind) {
        GC_INIT(MONOEXP_T2S)
        GC_INIT(MONOEXP_R2S)
        GC_INIT(GRE3)
        GC_INIT(DWI2)
        GC_INIT(LINEAR3)
    }
#undef GC_INIT
    return hipErrorInvalidValue;
}

template <int KIND, typename R, int MAXM, int EXACT = 0, int RECUR = kRecurRuntime>
static hipError_t chunk_t(const MhJob* jobs, const BlkMap* map, int nblk, hipStream_t s) {
    GC_LAUNCH((mh_chunk_kernel<KIND, R, MAXM, EXACT, RECUR>), dim3(nblk), dim3(kBlock), 0,
                       s, jobs, map);
    return hipGetLastError();
}

// Data read from memory: shared through LDS by the chains of a voxel when
// lds > 0 (see mh_chunk_kernel), else read per use by every lane.
template <int KIND, typename R>
static hipError_t chunk_mem_t(const MhJob* jobs, const BlkMap* map, int nblk, size_t lds,
                              hipStream_t s) {
    if (lds == 0) return chunk_t<KIND, R, 0>(jobs, map, nblk, s);
    GC_LAUNCH((mh_chunk_kernel<KIND, R, 0, 0, kRecurRuntime, true>), dim3(nblk),
                       dim3(kBlock), lds, s, jobs, map);
    return hipGetLastError();
}

// variant code = MAXM | exact << 16 | recurrence << 17 (see mh_pick_variant)
template <int KIND, int A, int B, int C>
static hipError_t chunk_f32(int variant, const MhJob* jobs, const BlkMap* map, int nblk,
                            size_t lds, hipStream_t s) {
    constexpr bool kRec = KIND == MONOEXP_T2S || KIND == MONOEXP_R2S || KIND == GRE3;
    constexpr int kExactRecur = kRec ? kRecurOn : kRecurOff;
    const int maxm = variant & 0xFFFF;
    const bool exact = (variant >> 16) & 1;
    if (exact) {
        if (maxm == A) return chunk_t<KIND, float, A, 1, kExactRecur>(jobs, map, nblk, s);
        if (maxm == B) return chunk_t<KIND, float, B, 1, kExactRecur>(jobs, map, nblk, s);
        if (maxm == C) return chunk_t<KIND, float, C, 1, kExactRecur>(jobs, map, nblk, s);
    }
    if (maxm == A) return chunk_t<KIND, float, A>(jobs, map, nblk, s);
    if (maxm == B) return chunk_t<KIND, float, B>(jobs, map, nblk, s);
    if (maxm == C) return chunk_t<KIND, float, C>(jobs, map, nblk, s);
    return chunk_mem_t<KIND, float>(jobs, map, nblk, lds, s);
}

hipError_t mh_chunk(int kind, bool fp64, int maxm, const MhJob* jobs, const BlkMap* map,
                    int nblk, int chains, int meff, hipStream_t s) {
    // rows padded to an odd length, as the kernel lays them out (meff is at
    // least every job's own count, so meff | 1 covers each job's padded row)
    const size_t row = (size_t)(meff | 1) * sizeof(float);
    const bool share = chains > 0 && kBlock % chains == 0 && meff > 0 &&
                       (size_t)(kBlock / chains) * row <= kMhSharedData;
    const size_t lds = share ? (size_t)(kBlock / chains) * row : 0;
    if (fp64) {
        switch (kind) {
            case MONOEXP_T2S: return chunk_mem_t<MONOEXP_T2S, double>(jobs, map, nblk, lds, s);
            case MONOEXP_R2S: return chunk_mem_t<MONOEXP_R2S, double>(jobs, map, nblk, lds, s);
            case GRE3: return chunk_mem_t<GRE3, double>(jobs, map, nblk, lds, s);
            case DWI2: return chunk_mem_t<DWI2, double>(jobs, map, nblk, lds, s);
            case LINEAR3: return chunk_mem_t<LINEAR3, double>(jobs, map, nblk, lds, s);
        }
        return hipErrorInvalidValue;
    }
    switch (kind) {
        case MONOEXP_T2S: return chunk_f32<MONOEXP_T2S, 12, 16, 32>(maxm, jobs, map, nblk, lds, s);
        case MONOEXP_R2S: return chunk_f32<MONOEXP_R2S, 12, 16, 32>(maxm, jobs, map, nblk, lds, s);
        case GRE3: return chunk_f32<GRE3, 12, 24, 32>(maxm, jobs, map, nblk, lds, s);
        case DWI2: return chunk_mem_t<DWI2, float>(jobs, map, nblk, lds, s);   // see mh_pick_variant
        case LINEAR3: return chunk_f32<LINEAR3, 12, 16, 16>(maxm, jobs, map, nblk, lds, s);
    }
    return hipErrorInvalidValue;
}

hipError_t mh_finalize(bool /*fp64*/, const MhJob* jobs, const BlkMap* vmap, int nblk,
                       double* out_mean, double* out_std, hipStream_t s) {
    hipLaunchKernelGGL(mh_finalize_kernel, dim3(nblk), dim3(kBlock), 0, s, jobs, vmap, out_mean,
                       out_std);
    return hipGetLastError();
}

}  // namespace gc
