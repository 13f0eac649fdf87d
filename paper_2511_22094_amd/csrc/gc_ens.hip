// Affine-invariant ensemble sampler (paper §2.2.2; Goodman & Weare 2010,
// stretch move; parallel split into two half-ensembles as in Foreman-Mackey
// et al. 2013).  All K walkers of a voxel live in one block's LDS; each lane
// owns one walker of each half and updates it in the matching half-step, so
// no lane idles.  Per (voxel v, walker k, iteration t) the counter
// (v, k | 2 << 16, t, 0) gives: word 0 -> partner j in the other half
// (floor of its 23-bit uniform times K/2),
// word 1 -> stretch z = ((a-1) u + 1)^2 / a, word 2 -> acceptance uniform;
// accept iff log u < (P-1) log z + logL(Y) - logL(X_k), Y = X_j + z (X_k - X_j),
// proposals outside the box rejected.
//
// Stretch moves multiply walker differences by up to a per accepted move, so
// a last-bit difference in a walker grows exponentially along the chain.  The
// walker-state arithmetic is therefore written as separate IEEE operations
// (floating-point contraction off) and the start is exactly computable, which
// keeps the FP64 instantiation bit-identical to a plain FP64 evaluation of
// the same steps; only the log-likelihoods carry last-bit differences, and
// those matter only for acceptance decisions within rounding of a tie.
#include "gc_internal.hpp"
#include "gc_timing.hpp"

namespace gc {

namespace {

template <typename R> __device__ __forceinline__ R lbE(const MhJob& J, int p) {
    if constexpr (sizeof(R) == 8) return J.lbd[p]; else return J.lb[p];
}
template <typename R> __device__ __forceinline__ R ubE(const MhJob& J, int p) {
    if constexpr (sizeof(R) == 8) return J.ubd[p]; else return J.ub[p];
}
template <typename R> __device__ __forceinline__ R x0E(const MhJob& J, int p) {
    if constexpr (sizeof(R) == 8) return J.x0cd[p]; else return J.x0c[p];
}
template <typename R> __device__ __forceinline__ R inv2s2E(const MhJob& J) {
    if constexpr (sizeof(R) == 8) return J.inv2s2d; else return J.inv2s2;
}
template <typename R> __device__ __forceinline__ R stretchE(const MhJob& J) {
    if constexpr (sizeof(R) == 8) return J.stretchd; else return J.stretch;
}

struct YGlobE {
    const float* y;
    int64_t n, v;
    int M;
    __device__ __forceinline__ float re(int m) const { return gload(y)[(int64_t)m * n + v]; }
    __device__ __forceinline__ float im(int m) const { return gload(y)[(int64_t)(M + m) * n + v]; }
};

// One voxel's measurements staged in LDS: real parts, or (re, im) pairs.
template <bool CPLX> struct YLdsE {
    const float* p;
    __device__ __forceinline__ float re(int m) const { return p[CPLX ? 2 * m : m]; }
    __device__ __forceinline__ float im(int m) const { return p[2 * m + 1]; }
};

__host__ __device__ constexpr size_t align16(size_t b) { return (b + 15) / 16 * 16; }

// Staged row length for Me floats: odd for real data; for (re, im) pairs an
// odd number of pairs, so pairs stay 8-byte aligned.
__host__ __device__ constexpr int ens_row(int Me, bool cplx) {
    return cplx ? ((Me / 2) % 2 == 0 ? Me + 2 : Me) : (Me | 1);
}

__device__ __forceinline__ int first_keep_e(int t0, int burnin, int thin) {
    int t = t0 > burnin ? t0 : burnin;
    int r = (t - burnin + 1) % thin;
    return r == 0 ? t : t + (thin - r);
}

}  // namespace

template <typename R> __device__ __forceinline__ R ballE(const MhJob& J, int p) {
    if constexpr (sizeof(R) == 8) return J.balld[p]; else return J.ball[p];
}

// Walker start: x0 (midpoint / given / map) plus a uniform offset in
// [-r, r], r = 1 % of the box width (word p % 4 of counter
// (v, k | 1 << 16, 0, p / 4): x = x0 + r (2u - 1)), clamped to the box;
// x0_mode 1 = uniform in the box as for MH chains.  Lanes are (voxel,
// walker) with lane = k n + v, like MH chains.
template <int KIND, typename R>
__global__ __launch_bounds__(kBlock) void ens_init_kernel(const MhJob* __restrict__ jobs,
                                                         const BlkMap* __restrict__ map) {
#pragma clang fp contract(off)
    using Mdl = typename ModelOf<KIND, R>::T;
    constexpr int P = Mdl::P;
    const BlkMap bm = map[blockIdx.x];
    const MhJob& J = jobs[bm.job];
    const int64_t n = J.n, NL = n * J.C;
    const int64_t L = bm.lane0 + threadIdx.x;
    if (L >= NL) return;
    const int64_t v = L % n;
    const int k = (int)(L / n);
    R th[P];
#pragma unroll
    for (int b = 0; b < (P + 3) / 4; ++b) {
        U4 o = philox4x32_10(U4{(uint32_t)v, (uint32_t)k | (1u << 16), 0u, (uint32_t)b}, J.k0,
                             J.k1);
        const uint32_t w[4] = {o.x, o.y, o.z, o.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int p = 4 * b + i;
            if (p >= P) continue;
            const R u = uniform01<R>(w[i]);
            const R lo = lbE<R>(J, p), hi = ubE<R>(J, p);
            if (J.x0_mode == 1) {
                th[p] = lo + (hi - lo) * u;
            } else {
                const R c = J.x0map ? (R)J.x0map[(int64_t)p * n + v] : x0E<R>(J, p);
                const R x = c + ballE<R>(J, p) * ((R)2 * u - (R)1);
                th[p] = x < lo ? lo : (x > hi ? hi : x);
            }
        }
    }
    const R w = J.w ? (R)J.w[v] : (R)1;
    const YGlobE y{J.y, n, v, J.acq.M};
    const R ll = -(inv2s2E<R>(J) * w * w) * Mdl::template sse<0>(th, y, J.acq);
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

// A chunk of ensemble iterations.  Block b covers voxels [b*vpb, (b+1)*vpb)
// with vpb = kBlock / (K/2); thread (vl, i) owns walkers i and K/2 + i of voxel
// b*vpb + vl.  The block map's lane0 is the block's first voxel.  With YLDS
// the block's measurements are staged once in LDS after the walkers (the 25
// threads of a half-ensemble then read them there instead of through the
// vector-memory path: one LDS read per value, no address arithmetic).
template <int KIND, typename R, bool YLDS>
__global__ __launch_bounds__(kBlock) void ens_chunk_kernel(const MhJob* __restrict__ jobs,
                                                          const BlkMap* __restrict__ map) {
#pragma clang fp contract(off)
    using Mdl = typename ModelOf<KIND, R>::T;
    constexpr int P = Mdl::P;
    constexpr bool CPLX = Mdl::kComplex;
    extern __shared__ unsigned char smem[];
    const BlkMap bm = map[blockIdx.x];
    const MhJob& J = jobs[bm.job];
    const int K = J.C, hp = K / 2, vpb = kBlock / hp;
    const int64_t n = J.n, NL = n * K;
    const int vl = threadIdx.x / hp, i = threadIdx.x % hp;
    const int64_t v = bm.lane0 + vl;
    const bool live = vl < vpb && v < n;
    R* X = (R*)smem;                    // [vpb][K][P]
    R* LP = X + (size_t)vpb * K * P;     // [vpb][K]
    R* TH = (R*)J.th;
    R* LLg = (R*)J.ll;
    // [vpb][Ms] measurements (Me = M, or 2 M as (re, im) pairs), after the
    // walkers; rows padded to Ms so that the voxels a wave reads at one index
    // fall in different LDS banks
    const int Me = CPLX ? 2 * J.acq.M : J.acq.M;
    const int Ms = ens_row(Me, CPLX);
    float* Yl = (float*)(smem + align16((size_t)vpb * K * (P + 1) * sizeof(R)));
    if constexpr (YLDS) {
        // consecutive threads take consecutive voxels of one row: coalesced reads
        for (int idx = threadIdx.x; idx < vpb * Me; idx += kBlock) {
            const int j = idx / vpb, a = idx % vpb;
            const int64_t va = bm.lane0 + a;
            const int row = CPLX ? ((j & 1) ? J.acq.M + (j >> 1) : (j >> 1)) : j;
            Yl[a * Ms + j] = va < n ? gload(J.y)[(int64_t)row * n + va] : 0.f;
        }
    }
    // load the ensemble of every voxel of the block
    for (int idx = threadIdx.x; idx < vpb * K; idx += kBlock) {
        const int a = idx / K, k = idx % K;
        const int64_t va = bm.lane0 + a;
        if (va < n) {
            const int64_t L = (int64_t)k * n + va;
#pragma unroll
            for (int p = 0; p < P; ++p) X[((size_t)a * K + k) * P + p] = TH[(int64_t)p * NL + L];
            LP[(size_t)a * K + k] = LLg[L];
        }
    }
    // Welford state of the two owned walkers
    double mu[2][P], m2[2][P];
    int32_t acc[2] = {0, 0};
    const bool welford = J.mean != nullptr;
    if (live) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int64_t L = (int64_t)(h * hp + i) * n + v;
            acc[h] = J.acc[L];
#pragma unroll
            for (int p = 0; p < P; ++p) {
                mu[h][p] = welford ? J.mean[(int64_t)p * NL + L] : 0.0;
                m2[h][p] = welford ? J.m2[(int64_t)p * NL + L] : 0.0;
            }
        }
    }
    __syncthreads();
    const R a = stretchE<R>(J);
    const R wv = live && J.w ? (R)J.w[v] : (R)1;
    const R nscale = -(inv2s2E<R>(J) * wv * wv);
    const YGlobE y{J.y, n, live ? v : 0, J.acq.M};
    const int B = J.burnin, thin = J.thin;
    int keep_t = first_keep_e(J.t0, B, thin);
    R* Xv = X + (size_t)(live ? vl : 0) * K * P;
    R* LPv = LP + (size_t)(live ? vl : 0) * K;
    for (int t = J.t0; t < J.t1; ++t) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int k = h * hp + i;
            R Y[P];
            R llp = 0;
            bool accept = false;
            if (live) {
                U4 o = philox4x32_10(U4{(uint32_t)v, (uint32_t)k | (2u << 16), (uint32_t)t, 0u},
                                     J.k0, J.k1);
                // partner: floor(u hp) of the 23-bit uniform u = (2q+1)/2^24,
                // taken in integer arithmetic so every precision agrees
                const int jj = (int)((((uint64_t)(o.x >> 9) * 2u + 1u) * (uint64_t)hp) >> 24);
                const int j = (1 - h) * hp + jj;
                const R uz = uniform01<R>(o.y);
                const R zt = (a - (R)1) * uz + (R)1;
                const R z = zt * zt / a;
                bool inb = true;
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    const R xj = Xv[(size_t)j * P + p];
                    Y[p] = xj + z * (Xv[(size_t)k * P + p] - xj);
                    inb &= in_box(Y[p], lbE<R>(J, p), ubE<R>(J, p));
                }
                R ev[P];
#pragma unroll
                for (int p = 0; p < P; ++p) ev[p] = inb ? Y[p] : Xv[(size_t)k * P + p];
                if constexpr (YLDS)
                    llp = nscale * Mdl::template sse<0>(ev, YLdsE<CPLX>{Yl + vl * Ms}, J.acq);
                else
                    llp = nscale * Mdl::template sse<0>(ev, y, J.acq);
                const R lhs = Math<R>::ln(uniform01<R>(o.z));
                accept = inb && (lhs < (R)(P - 1) * Math<R>::ln(z) + llp - LPv[k]);
            }
            __syncthreads();   // every read of this half-step is done
            if (accept) {
#pragma unroll
                for (int p = 0; p < P; ++p) Xv[(size_t)k * P + p] = Y[p];
                LPv[k] = llp;
                acc[h] += 1;
            }
            __syncthreads();   // updates visible to the other half
        }
        if (t == keep_t) {
            keep_t += thin;
            const int kk = (t - B + 1) / thin;
            const double inv = 1.0 / (double)kk;
            if (live) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int k = h * hp + i;
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        const double x = (double)Xv[(size_t)k * P + p];
                        const double d = x - mu[h][p];
                        mu[h][p] += d * inv;
                        m2[h][p] += d * (x - mu[h][p]);
                        if (J.samples)
                            J.samples[(((int64_t)k * J.s_K + (kk - 1 - J.s_base)) * P + p) * n +
                                      v] = (float)x;
                    }
                }
            }
        }
    }
    if (live) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int k = h * hp + i;
            const int64_t L = (int64_t)k * n + v;
#pragma unroll
            for (int p = 0; p < P; ++p) {
                TH[(int64_t)p * NL + L] = Xv[(size_t)k * P + p];
                if (welford) {
                    J.mean[(int64_t)p * NL + L] = mu[h][p];
                    J.m2[(int64_t)p * NL + L] = m2[h][p];
                }
            }
            LLg[L] = LPv[k];
            J.acc[L] = acc[h];
        }
    }
}

template <int KIND, typename R>
static hipError_t ens_init_t(const MhJob* jobs, const BlkMap* map, int nblk, hipStream_t s) {
    hipLaunchKernelGGL((ens_init_kernel<KIND, R>), dim3(nblk), dim3(kBlock), 0, s, jobs, map);
    return hipGetLastError();
}

hipError_t ens_init(int kind, bool fp64, const MhJob* jobs, const BlkMap* map, int nblk,
                    hipStream_t s) {
#define GC_EI(K)                                                                              \
    case K:                                                                                   \
        return fp64 ? ens_init_t<K, double>(jobs, map, nblk, s) : ens_init_t<K, float>(jobs, map, nblk, s);
    switch (kind) {
        GC_EI(MONOEXP_T2S)
        GC_EI(MONOEXP_R2S)
        GC_EI(GRE3)
        GC_EI(DWI2)
        GC_EI(LINEAR3)
    }
#undef GC_EI
    return hipErrorInvalidValue;
}

// Launch for jobs whose walker count is `walkers` (the map covers voxels in
// groups of kBlock / (walkers / 2)) and whose effective measurement counts are
// at most `meff`; dynamic LDS = vpb * K * (P + 1) reals for the walkers, plus
// vpb rows of staged data (meff floats, padded: ens_row) when that fits in
// kEnsLdsData bytes.
constexpr size_t kEnsLdsData = 64 * 1024;
template <int KIND, typename R>
static hipError_t ens_chunk_t(const MhJob* jobs, const BlkMap* map, int nblk, int walkers,
                              int meff, hipStream_t s) {
    using Mdl = typename ModelOf<KIND, R>::T;
    const int hp = walkers / 2, vpb = kBlock / hp;
    const size_t lds = (size_t)vpb * walkers * (Mdl::P + 1) * sizeof(R);
    // meff is at least every job's own count, so its padded row covers theirs
    const size_t lds_y = align16(lds) + (size_t)vpb * ens_row(meff, Mdl::kComplex) * sizeof(float);
    if (meff > 0 && lds_y <= kEnsLdsData)
        GC_LAUNCH((ens_chunk_kernel<KIND, R, true>), dim3(nblk), dim3(kBlock), lds_y, s,
                           jobs, map);
    else
        GC_LAUNCH((ens_chunk_kernel<KIND, R, false>), dim3(nblk), dim3(kBlock), lds, s,
                           jobs, map);
    return hipGetLastError();
}

hipError_t ens_chunk_walkers(int kind, bool fp64, const MhJob* jobs, const BlkMap* map, int nblk,
                             int walkers, int meff, hipStream_t s) {
#define GC_EC(K)                                                                          \
    case K:                                                                               \
        return fp64 ? ens_chunk_t<K, double>(jobs, map, nblk, walkers, meff, s)           \
                    : ens_chunk_t<K, float>(jobs, map, nblk, walkers, meff, s);
    switch (kind) {
        GC_EC(MONOEXP_T2S)
        GC_EC(MONOEXP_R2S)
        GC_EC(GRE3)
        GC_EC(DWI2)
        GC_EC(LINEAR3)
    }
#undef GC_EC
    return hipErrorInvalidValue;
}

}  // namespace gc
