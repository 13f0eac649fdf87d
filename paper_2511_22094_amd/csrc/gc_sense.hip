// Image reconstruction with the askadam solver (paper §2.6.4, Eq. 7):
//   minimise 1/Nk sum_{e,c, sampled} l(M_e F2(C_c I_e) - k_ec) + lambda/Npix TV2(I)
// over the complex multi-echo image I [E][Ny][Nz], with F2 the unitary 2D DFT
// over the two phase-encoding axes, C_c the coil sensitivities, M_e the
// sampling mask of echo e, l = |Re r|^2 + |Im r|^2 (L2) or |Re r| + |Im r| (L1)
// and TV2 the anisotropic 2D total variation of the real and imaginary parts.
//
// The E x Nc coil images live in one buffer `buf` [E][Nc][Ny][Nz] that holds,
// between the two launches of an iteration, the coil images transformed
// along z only.  One iteration:
//   ycols  (block per (e, c, G columns)): DFT along y, residual against the
//          measured samples, loss partial, dl/dX, inverse DFT along y;
//   zrows  (block per (e, y) row, all coils): inverse DFT along z, times
//          conj(C_c), sum over coils = gradient; TV subgradient; optimiser
//          step; then x = C_c I_new and its DFT along z for the next
//          iteration.
// Each pass reads and writes `buf` once: four passes of 8 E Nc Ny Nz bytes
// per iteration.  Transforms are four-step team FFTs (gc_fft.hpp) with one
// LDS transpose each.  Sizes along y and z are powers of two up to
// kSenseMaxN, z at least kSenseMinNz.
#include "gc_fft.hpp"
#include "gc_sense.hpp"
#include "gc_timing.hpp"

namespace gc {

namespace {

typedef float v2f __attribute__((ext_vector_type(2)));
// complex sample loaded through the global address space as one 8-byte load
__device__ __forceinline__ float2 ld2(const float2* p, int64_t i) {
    const v2f t = gload((const v2f*)p)[i];
    return make_float2(t.x, t.y);
}
// The same from a block-uniform base with a 32-bit offset (one address
// register per load instead of two).
__device__ __forceinline__ float2 ld2u(const float2* p, uint32_t i) {
    const v2f t = gload((const v2f*)p)[i];
    return make_float2(t.x, t.y);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {   // a * conj(b)
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float sgnf(float d) { return d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f); }

// Blocks are dealt round-robin over the 8 XCDs; XCD x takes a contiguous
// range of logical blocks so that neighbouring tiles share its L2.
__device__ __forceinline__ int xcd_block(int b, int nblk) {
    const int q = nblk / 8, r = nblk % 8, x = b % 8;
    return x * q + (x < r ? x : r) + b / 8;
}

// Fixed-order block sum (result in thread 0) for a power-of-two block size.
__device__ __forceinline__ float block_sum_pow2(float v, float* red /*[4]*/) {
    const int W = blockDim.x < 64 ? (int)blockDim.x : 64;
    for (int o = W >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, W);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = v;
    __syncthreads();
    float r = 0.f;
    if (threadIdx.x == 0)
        for (int i = 0; i < ((int)blockDim.x + 63) / 64; ++i) r += red[i];
    return r;
}

// y pass geometry: G columns per block, a team of N2 threads per column.
template <int LOG> struct YGeo {
    using Sh = FftShape<LOG>;
    static constexpr int G = sense_tile_cols(LOG);
    static constexpr int THREADS = G * Sh::N2;
    static constexpr int RS = Sh::N2 * G + G;   // float2 per k1 row of the transpose (padded)
    static constexpr int LDS = Sh::N + Sh::N1 * RS;
};
// z pass geometry: TEAMS coil rows at a time, a team of N2 threads per row.
// 256-point rows take 8 teams, not 16: a block's LDS is then 21 KB instead of
// 39 KB, LDS no longer limits a CU to 4 blocks, and the 1,536 blocks of a
// 6-echo 256-row slice run in one round instead of 1.5 (measured 43.8 -> 42.0
// us per pass; 4 teams, 49.7 us).
template <int LOG> struct ZGeo {
    using Sh = FftShape<LOG>;
    static constexpr int T1 = 256 / Sh::N2, T2 = LOG == 8 ? 8 : (4096 >> LOG);
    static constexpr int TEAMS = T1 < T2 ? T1 : T2;
    static constexpr int THREADS = TEAMS * Sh::N2;
    static constexpr int RS = Sh::N2 + 1;        // float2 per k1 row of a team's transpose
    static constexpr int AREA = Sh::N1 * RS;     // >= N: reused for the coil sum
    static constexpr int LDS = 2 * Sh::N + TEAMS * AREA;
};

}  // namespace

// ------------------------------------------------------------------ y pass
// MODE 0: iteration (forward DFT_y, residual, dl/dX, inverse DFT_y; buf in place)
// MODE 1: operator tail (forward DFT_y of buf, zero outside the mask, to out)
// MODE 2: adjoint head (input r zeroed outside the mask, inverse DFT_y, to buf)
template <int LOGY, int MODE>
__global__ __launch_bounds__(256) void sense_ycols_kernel(SenseDev S, const float2* __restrict__ in,
                                                         float2* __restrict__ buf,
                                                         float2* __restrict__ out,
                                                         float* __restrict__ partial,
                                                         const int* __restrict__ stop) {
    using Sh = FftShape<LOGY>;
    using Geo = YGeo<LOGY>;
    constexpr int N = Sh::N, N1 = Sh::N1, N2 = Sh::N2, G = Geo::G;
    extern __shared__ float2 lds[];
    __shared__ float red[4];
    if (stop && stop[0] != 0) return;   // uniform
    const int nzg = S.Nz / G;
    const int t = threadIdx.x, j = t % G, p = t / G;
    float2* tw = lds;
    float2* T = lds + N + j;
    const uint32_t Nz = S.Nz;
    const int64_t isz = (int64_t)S.Ny * Nz;                  // one coil image
    const int tl = xcd_block(blockIdx.x, gridDim.x);          // tile: (e, c, z / G)
    float2 a[N1];
    const int ec = tl / nzg, z0 = (tl % nzg) * G;
    const int e = ec / S.Nc, c = ec % S.Nc;
    const int z = z0 + j;
    const int64_t img = (int64_t)ec * isz;                // this coil image (block-uniform)
    float2* bimg = buf + img;                             // element (y, z) at y Nz + z
    const uint32_t bit = 1u << j;
    const int64_t tile = (int64_t)e * nzg + z0 / G;
    const uint32_t* ti = S.tinfo + tile * S.Ny;           // row y of this tile at ti[y]
    // the tile's columns, row masks and (iterating) measured samples are
    // fetched up front, without branches, so that the loads overlap
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1)
        a[n1] = ld2u(MODE == 2 ? in + img : bimg, (p + N2 * n1) * Nz + z);
    uint32_t word[N1];
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) word[n1] = gload(ti)[p + N2 * n1];
    float2 kv[N1];
    if (MODE == 0) {
        const float2* kc = S.kc + (int64_t)c * S.S + gload(S.tbase)[tile];
#pragma unroll
        for (int n1 = 0; n1 < N1; ++n1) {   // unsampled entries read sample 0 and drop it
            const uint32_t s = (word[n1] & bit) ? (word[n1] >> 16) + __popc(word[n1] & (bit - 1u)) : 0u;
            kv[n1] = ld2u(kc, s);
        }
    }
    // twiddles to LDS while the column loads are in flight
    for (int i = t; i < N; i += Geo::THREADS) tw[i] = ld2(S.twy, i);
    __syncthreads();
    if (MODE == 2) {
#pragma unroll
        for (int n1 = 0; n1 < N1; ++n1)
            if (!(word[n1] & bit)) a[n1] = make_float2(0.f, 0.f);
    } else {
        fft_team<LOGY, false>(a, p, T, Geo::RS, G, tw);
    }
    const float sc = S.rsqrtNy;
    if (MODE == 1) {
#pragma unroll
        for (int n1 = 0; n1 < N1; ++n1) {
            const int y = p + N2 * n1;
            out[img + y * Nz + z] = (word[n1] & bit) ? make_float2(a[n1].x * sc, a[n1].y * sc)
                                                    : make_float2(0.f, 0.f);
        }
    } else {
        float lsum = 0.f;
        if (MODE == 0) {
            const float sd = S.scale_data;
#pragma unroll
            for (int n1 = 0; n1 < N1; ++n1) {
                float2 d = make_float2(0.f, 0.f);
                if (word[n1] & bit) {
                    const float rx = a[n1].x * sc - kv[n1].x, ry = a[n1].y * sc - kv[n1].y;
                    if (S.loss_p == 2) {
                        lsum += rx * rx + ry * ry;
                        d = make_float2(2.f * rx * sd, 2.f * ry * sd);
                    } else {
                        lsum += fabsf(rx) + fabsf(ry);
                        d = make_float2(sgnf(rx) * sd, sgnf(ry) * sd);
                    }
                }
                a[n1] = d;
            }
        }
        fft_team<LOGY, true>(a, p, T, Geo::RS, G, tw);
#pragma unroll
        for (int n1 = 0; n1 < N1; ++n1)
            bimg[(p + N2 * n1) * Nz + z] = make_float2(a[n1].x * sc, a[n1].y * sc);
        if (MODE == 0 && partial) {
            const float s = block_sum_pow2(lsum * S.scale_data, red);
            if (t == 0) partial[tl] = s;
        }
    }
}

// ------------------------------------------------------------------ z pass
// MODE 0: iteration (gradient from buf, TV, optimiser step img_in -> img_out;
//         with fwd, the next iteration's forward rows into buf)
// MODE 1: operator head (forward rows of img_in into buf)
// MODE 2: adjoint tail (sum over coils of conj(C_c) F_z^H(buf), to out)
// The kernel keeps the registers the compiler wants: for 256-point rows 136
// VGPRs, 3 waves per SIMD, which with 8 teams still holds a 6-echo slice's
// 1,536 blocks at once (capped at 4 waves per SIMD it spilled and measured
// slower: 42.1 against 40.3 us per pass).
template <int LOGZ, int MODE>
__global__ __launch_bounds__(256)
void sense_zrows_kernel(SenseDev S, SenseOpt O,
                                                         const float2* __restrict__ img_in,
                                                         float2* __restrict__ img_out,
                                                         float2* __restrict__ m,
                                                         float2* __restrict__ v,
                                                         float2* __restrict__ buf,
                                                         float2* __restrict__ out,
                                                         float* __restrict__ partial,
                                                         const int* __restrict__ stop, int fwd) {
    using Sh = FftShape<LOGZ>;
    using Geo = ZGeo<LOGZ>;
    constexpr int N = Sh::N, N1 = Sh::N1, N2 = Sh::N2, TEAMS = Geo::TEAMS;
    extern __shared__ float2 lds[];
    __shared__ float red[4];
    if (stop && stop[0] != 0) return;   // uniform
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int y = blk / S.E, e = blk % S.E;   // the echoes of one row are neighbours
    const int t = threadIdx.x, tau = t / N2, p = t % N2;
    const int Ny = S.Ny, Nc = S.Nc;
    float2* tw = lds;
    float2* U = lds + N;
    float2* T = lds + 2 * N;
    float2* Tt = T + tau * Geo::AREA;
    const int64_t row = ((int64_t)e * Ny + y) * N;   // image row (e, y), block-uniform
    const uint32_t cstride = (uint32_t)Ny * N;        // coil to coil within buf and the maps
    // A batch is TEAMS coil rows.  Teams past the last coil read the last
    // coil's row and drop it, so that every load is unconditional and all of
    // them overlap.
    float2 a[N1], cv[N1];
    auto load_batch = [&](int cb) {
        const int c = cb + tau;
        const float2* bb = buf + (((int64_t)e * Nc + cb) * Ny + y) * N;   // block-uniform
        const float2* cm = S.coils + ((int64_t)cb * Ny + y) * N;
        const uint32_t o = (uint32_t)((c < Nc ? c : Nc - 1) - cb) * cstride + p;
#pragma unroll
        for (int n1 = 0; n1 < N1; ++n1) {
            a[n1] = ld2u(bb, o + N2 * n1);
            cv[n1] = ld2u(cm, o + N2 * n1);
        }
    };
    float2 twv[(N + Geo::THREADS - 1) / Geo::THREADS];   // twiddles: loads issued first
#pragma unroll
    for (int k = 0; k * Geo::THREADS < N; ++k)
        twv[k] = ld2(S.twz, min(t + k * Geo::THREADS, N - 1));
    if (MODE != 1) load_batch(0);   // in flight while the twiddles are staged
#pragma unroll
    for (int k = 0; k * Geo::THREADS < N; ++k)
        if (t + k * Geo::THREADS < N) tw[t + k * Geo::THREADS] = twv[k];
    if (MODE == 1)
        for (int z = t; z < N; z += Geo::THREADS) U[z] = ld2u(img_in + row, z);
    __syncthreads();
    const float sc = S.rsqrtNz;
    float tvl = 0.f;
    if (MODE != 1) {
        float2 acc[N1];
#pragma unroll
        for (int n1 = 0; n1 < N1; ++n1) acc[n1] = make_float2(0.f, 0.f);
        for (int cb = 0; cb < Nc; cb += TEAMS) {   // uniform trip count (barriers inside)
            if (cb > 0) load_batch(cb);
            const bool live = cb + tau < Nc;
            fft_team<LOGZ, true>(a, p, Tt, Geo::RS, 1, tw);
#pragma unroll
            for (int n1 = 0; n1 < N1; ++n1) {
                const float2 q = cmulc(a[n1], cv[n1]);
                acc[n1].x += live ? q.x : 0.f;
                acc[n1].y += live ? q.y : 0.f;
            }
        }
        __syncthreads();   // every team is done with its transpose area
#pragma unroll
        for (int n1 = 0; n1 < N1; ++n1) Tt[p + N2 * n1] = acc[n1];
        __syncthreads();
        for (int z = t; z < N; z += Geo::THREADS) {
            float2 g = make_float2(0.f, 0.f);
            for (int k = 0; k < TEAMS; ++k) {   // fixed order
                const float2 q = T[k * Geo::AREA + z];
                g.x += q.x;
                g.y += q.y;
            }
            g.x *= sc;
            g.y *= sc;
            if (MODE == 2) {
                out[row + z] = g;
                continue;
            }
            const float2* irow = img_in + row;
            const float2 u = ld2u(irow, z);
            if (O.scale_tv != 0.f) {
                // neighbours read at clamped positions (a pixel on the border
                // reads itself: difference 0, and its pair does not count)
                const bool zf = z + 1 < N, yf = y + 1 < Ny, zb = z > 0, yb = y > 0;
                const float2 qzf = ld2u(irow, zf ? z + 1 : z);
                const float2 qyf = ld2u(irow + (yf ? N : 0), z);
                const float2 qzb = ld2u(irow, zb ? z - 1 : z);
                const float2 qyb = ld2u(irow - (yb ? N : 0), z);
                // forward pairs (u, q): |q - u| counts, -sign(q - u) on u
                const float R = (zf ? fabsf(qzf.x - u.x) + fabsf(qzf.y - u.y) : 0.f) +
                                (yf ? fabsf(qyf.x - u.x) + fabsf(qyf.y - u.y) : 0.f);
                // backward pairs (q, u): +sign(u - q) on u; sign(0) = 0 covers the borders
                const float gx = sgnf(u.x - qzb.x) + sgnf(u.x - qyb.x) - sgnf(qzf.x - u.x) -
                                 sgnf(qyf.x - u.x);
                const float gy = sgnf(u.y - qzb.y) + sgnf(u.y - qyb.y) - sgnf(qzf.y - u.y) -
                                 sgnf(qyf.y - u.y);
                g.x += O.scale_tv * gx;
                g.y += O.scale_tv * gy;
                tvl += O.scale_tv * R;
            }
            float2 mm = m[row + z], vv = v[row + z], un;
            auto step = [&](float uu, float gg, float& mk, float& vk) -> float {
                if (O.optimizer == 0) {
                    mk = O.beta1 * mk + O.omb1 * gg;
                    vk = O.beta2 * vk + O.omb2 * gg * gg;
                    return uu - O.lr * (mk * O.c1) / (sqrtf(vk * O.c2) + O.eps);
                } else if (O.optimizer == 1) {
                    mk = O.momentum * mk - O.lr * gg;
                    return uu + mk;
                }
                vk = O.rho * vk + O.omrho * gg * gg;
                return uu - O.lr * gg / (sqrtf(vk) + O.eps);
            };
            un.x = step(u.x, g.x, mm.x, vv.x);
            un.y = step(u.y, g.y, mm.y, vv.y);
            img_out[row + z] = un;
            m[row + z] = mm;
            v[row + z] = vv;
            U[z] = un;
        }
    }
    if (MODE == 2) return;
    if (MODE == 0 && partial) {
        const float s = block_sum_pow2(tvl, red);
        if (t == 0) partial[blockIdx.x] = s;
    }
    if (MODE == 1 || fwd) {
        __syncthreads();   // U complete
        for (int cb = 0; cb < Nc; cb += TEAMS) {
            const int c = cb + tau;
            const bool live = c < Nc;
            float2* bb = buf + (((int64_t)e * Nc + cb) * Ny + y) * N;   // block-uniform
            const float2* cm = S.coils + ((int64_t)cb * Ny + y) * N;
            const uint32_t o = (uint32_t)((live ? c : Nc - 1) - cb) * cstride + p;
            float2 a[N1];
#pragma unroll
            for (int n1 = 0; n1 < N1; ++n1) a[n1] = ld2u(cm, o + N2 * n1);
#pragma unroll
            for (int n1 = 0; n1 < N1; ++n1) a[n1] = fft_cmul(a[n1], U[p + N2 * n1]);
            fft_team<LOGZ, false>(a, p, Tt, Geo::RS, 1, tw);
            if (live) {
#pragma unroll
                for (int n1 = 0; n1 < N1; ++n1)
                    bb[o + N2 * n1] = make_float2(a[n1].x * sc, a[n1].y * sc);
            }
        }
    }
}

// -------------------------------------------------------- k-space packing
__global__ __launch_bounds__(kBlock) void sense_pack_kernel(SenseDev S, const float2* __restrict__ dense,
                                                           float2* __restrict__ kc) {
    const int64_t NN = (int64_t)S.Ny * S.Nz;
    const int64_t n = (int64_t)S.E * S.Nc * NN;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int z = (int)(i % S.Nz);
    const int y = (int)((i / S.Nz) % S.Ny);
    const int64_t ec = i / NN;
    const int c = (int)(ec % S.Nc), e = (int)(ec / S.Nc);
    const int64_t tile = (int64_t)e * (S.Nz / S.G) + z / S.G;
    const uint32_t word = gload(S.tinfo)[tile * S.Ny + y], bit = 1u << (z % S.G);
    if (!(word & bit)) return;
    const int64_t s = (int64_t)gload(S.tbase)[tile] + (word >> 16) + __popc(word & (bit - 1u));
    kc[(int64_t)c * S.S + s] = ld2(dense, i);
}

// ------------------------------------------------------------------ launchers
namespace {

template <int LOGY, int MODE>
hipError_t launch_y(const SenseDev& S, const float2* in, float2* buf, float2* out, float* partial,
                    const int* stop, hipStream_t s) {
    using Geo = YGeo<LOGY>;
    const int nblk = S.E * S.Nc * (S.Nz / Geo::G);
    GC_LAUNCH((sense_ycols_kernel<LOGY, MODE>), dim3(nblk), dim3(Geo::THREADS),
                       Geo::LDS * sizeof(float2), s, S, in, buf, out, partial, stop);
    return hipGetLastError();
}

template <int MODE>
hipError_t dispatch_y(const SenseDev& S, const float2* in, float2* buf, float2* out, float* partial,
                      const int* stop, hipStream_t s) {
    switch (S.logNy) {
#define GC_Y(L) \
    case L: return launch_y<L, MODE>(S, in, buf, out, partial, stop, s);
        GC_Y(1) GC_Y(2) GC_Y(3) GC_Y(4) GC_Y(5) GC_Y(6) GC_Y(7) GC_Y(8) GC_Y(9) GC_Y(10)
#undef GC_Y
    default: return hipErrorInvalidValue;
    }
}

template <int LOGZ, int MODE>
hipError_t launch_z(const SenseDev& S, const SenseOpt& O, const float2* img_in, float2* img_out,
                    float2* m, float2* v, float2* buf, float2* out, float* partial,
                    const int* stop, int fwd, hipStream_t s) {
    using Geo = ZGeo<LOGZ>;
    const int nblk = S.E * S.Ny;
    GC_LAUNCH((sense_zrows_kernel<LOGZ, MODE>), dim3(nblk), dim3(Geo::THREADS),
                       Geo::LDS * sizeof(float2), s, S, O, img_in, img_out, m, v, buf, out,
                       partial, stop, fwd);
    return hipGetLastError();
}

template <int MODE>
hipError_t dispatch_z(const SenseDev& S, const SenseOpt& O, const float2* img_in,
                      float2* img_out, float2* m, float2* v, float2* buf, float2* out,
                      float* partial, const int* stop, int fwd, hipStream_t s) {
    switch (S.logNz) {
#define GC_Z(L) \
    case L: return launch_z<L, MODE>(S, O, img_in, img_out, m, v, buf, out, partial, stop, fwd, s);
        GC_Z(4) GC_Z(5) GC_Z(6) GC_Z(7) GC_Z(8) GC_Z(9) GC_Z(10)
#undef GC_Z
    default: return hipErrorInvalidValue;
    }
}

int ycols_blocks(const SenseDev& S) { return S.E * S.Nc * (S.Nz / sense_tile_cols(S.logNy)); }

}  // namespace

hipError_t sense_pack_kspace(const SenseDev& S, const float2* dense, float2* kc, hipStream_t s) {
    const int64_t n = (int64_t)S.E * S.Nc * S.Ny * S.Nz;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(sense_pack_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock),
                       0, s, S, dense, kc);
    return hipGetLastError();
}

hipError_t sense_forward_rows(const SenseDev& S, const float2* img, float2* buf, hipStream_t s) {
    return dispatch_z<1>(S, SenseOpt{}, img, nullptr, nullptr, nullptr, buf, nullptr, nullptr,
                         nullptr, 1, s);
}

hipError_t sense_stage(int stage, const SenseDev& S, const SenseOpt& O, const float2* img_in,
                       float2* img_out, float2* m, float2* v, float2* buf, float* partial,
                       const int* stop, int fwd, hipStream_t s) {
    if (stage == 0) return dispatch_y<0>(S, nullptr, buf, nullptr, partial, stop, s);
    return dispatch_z<0>(S, O, img_in, img_out, m, v, buf, nullptr,
                         partial ? partial + ycols_blocks(S) : nullptr, stop, fwd, s);
}

int64_t sense_partials(const SenseDev& S) { return (int64_t)ycols_blocks(S) + (int64_t)S.E * S.Ny; }

hipError_t sense_forward_op(const SenseDev& S, const float2* img, float2* buf, float2* out,
                            hipStream_t s) {
    hipError_t e = sense_forward_rows(S, img, buf, s);
    if (e != hipSuccess) return e;
    return dispatch_y<1>(S, nullptr, buf, out, nullptr, nullptr, s);
}

hipError_t sense_adjoint_op(const SenseDev& S, const float2* r, float2* buf, float2* out,
                            hipStream_t s) {
    hipError_t e = dispatch_y<2>(S, r, buf, nullptr, nullptr, nullptr, s);
    if (e != hipSuccess) return e;
    return dispatch_z<2>(S, SenseOpt{}, nullptr, nullptr, nullptr, nullptr, buf, out, nullptr,
                         nullptr, 0, s);
}

}  // namespace gc
