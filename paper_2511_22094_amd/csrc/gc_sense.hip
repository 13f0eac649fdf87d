// Image reconstruction with the askadam solver (paper §2.6.4, Eq. 7):
//   minimise 1/Nk sum_{e,c, sampled} l(M_e F2(C_c I_e) - k_ec) + lambda/Npix TV2(I)
// over the complex multi-echo image I [E][Ny][Nz], with F2 the unitary 2D DFT
// over the two phase-encoding axes, C_c the coil sensitivities, M_e the
// sampling mask of echo e, l = |Re r|^2 + |Im r|^2 (L2) or |Re r| + |Im r| (L1)
// and TV2 the anisotropic 2D total variation of the real and imaginary parts.
//
// One iteration is four kernels over the E x Nc coil images:
//   rows_fwd   x = C_c I_e, DFT along z (LDS, radix 2)            -> buf
//   cols       DFT along y, residual against the measured samples,
//              loss partials, dl/dX, inverse DFT along y (in LDS) -> buf
//   rows_adj   inverse DFT along z, times conj(C_c)                -> buf
//   update     sum over coils + TV subgradient, optimiser step on Re and Im
// Sizes along y and z are powers of two up to kSenseMaxN (z at least
// kSenseCols); the y pass works on tiles of Ny x G columns, G = min(16, 4096/Ny).
#include "gc_sense.hpp"

namespace gc {

namespace {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {   // a * conj(b)
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
// complex sample loaded through the global address space as one 8-byte load
typedef float v2f __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 ld2(const float2* p, int64_t i) {
    const v2f t = gload((const v2f*)p)[i];
    return make_float2(t.x, t.y);
}
__device__ __forceinline__ unsigned bitrev(unsigned i, int logn) {
    return __brev(i) >> (32 - logn);
}

// In-place radix-2 decimation-in-time transform of `cnt` interleaved
// sequences held in LDS, element j of sequence s at x[j * cnt + s], the input
// already in bit-reversed order.  tw[k] = exp(-2 pi i k / N); inverse uses
// the conjugate twiddles.  All threads of the block take part.
template <bool INV>
__device__ __forceinline__ void fft_lds(float2* x, int N, int logn, int cnt,
                                        const float2* __restrict__ tw) {
    for (int s = 1; s <= logn; ++s) {
        const int half = 1 << (s - 1);
        const int stride = N >> s;   // twiddle index step
        __syncthreads();
        for (int i = threadIdx.x; i < (N >> 1) * cnt; i += blockDim.x) {
            const int seq = i % cnt, bf = i / cnt;
            const int k = bf & (half - 1);
            const int a = ((bf >> (s - 1)) << s) + k;
            const int b = a + half;
            float2 w = ld2(tw, k * stride);
            if (INV) w.y = -w.y;
            const float2 xb = x[b * cnt + seq], xa = x[a * cnt + seq];
            const float2 t = cmul(w, xb);
            x[a * cnt + seq] = make_float2(xa.x + t.x, xa.y + t.y);
            x[b * cnt + seq] = make_float2(xa.x - t.x, xa.y - t.y);
        }
    }
    __syncthreads();
}

}  // namespace

// ---------------------------------------------------------------- rows
// One block per (e, c, y) row.  MODE 0: forward pass, input C_c I_e; MODE 1:
// adjoint pass, input buf, output conj(C_c) IDFT_z(buf).
template <int MODE>
__global__ __launch_bounds__(kBlock) void sense_rows_kernel(SenseDev S, const float2* __restrict__ img,
                                                           float2* __restrict__ buf,
                                                           const int* __restrict__ stop) {
    extern __shared__ float2 lds[];
    if (stop && stop[0] != 0) return;
    const int Ny = S.Ny, Nz = S.Nz;
    const int row = blockIdx.x;                  // ((e Nc + c) Ny + y)
    const int y = row % Ny, ec = row / Ny;
    const int c = ec % S.Nc, e = ec / S.Nc;
    const float2* C = S.coils + ((int64_t)c * Ny + y) * Nz;
    float2* out = buf + (int64_t)row * Nz;
    for (int z = threadIdx.x; z < Nz; z += blockDim.x) {
        float2 v;
        if (MODE == 0) v = cmul(ld2(C, z), ld2(img, ((int64_t)e * Ny + y) * Nz + z));
        else v = out[z];
        lds[bitrev(z, S.logNz)] = v;
    }
    fft_lds<MODE == 1>(lds, Nz, S.logNz, 1, S.twz);
    const float sc = S.rsqrtNz;
    for (int z = threadIdx.x; z < Nz; z += blockDim.x) {
        float2 v = lds[z];
        v.x *= sc;
        v.y *= sc;
        if (MODE == 1) v = cmulc(v, ld2(C, z));
        out[z] = v;
    }
}

// ---------------------------------------------------------------- columns
// One block per (e, c, group of G columns).  Forward DFT along y;
// r = X - k on sampled entries; loss partial; dl/dX scaled by 1/Nk; inverse
// DFT along y; back to buf.
__global__ __launch_bounds__(kBlock) void sense_cols_kernel(SenseDev S, float2* __restrict__ buf,
                                                           float* __restrict__ partial,
                                                           const int* __restrict__ stop) {
    extern __shared__ float2 lds[];
    __shared__ float red[kBlock / 64];
    if (stop && stop[0] != 0) return;
    const int Ny = S.Ny, Nz = S.Nz, G = S.G;
    const int ngrp = Nz / G;
    const int ec = blockIdx.x / ngrp, z0 = (blockIdx.x % ngrp) * G;
    const int e = ec / S.Nc;
    float2* base = buf + (int64_t)ec * Ny * Nz;
    float2* A = lds;             // [Ny][G]
    for (int i = threadIdx.x; i < Ny * G; i += blockDim.x) {
        const int y = i / G, j = i % G;
        A[bitrev(y, S.logNy) * G + j] = base[(int64_t)y * Nz + z0 + j];
    }
    fft_lds<false>(A, Ny, S.logNy, G, S.twy);
    const float sc = S.rsqrtNy;
    const float2* K = S.ksp + (int64_t)ec * Ny * Nz;
    const uint8_t* Mk = S.mask + (int64_t)e * Ny * Nz;
    float lsum = 0.f;
    // residual and dl/dX in place (natural order) ...
    for (int i = threadIdx.x; i < Ny * G; i += blockDim.x) {
        const int y = i / G, j = i % G;
        const int64_t a = (int64_t)y * Nz + z0 + j;
        float2 d = make_float2(0.f, 0.f);
        if (gload(Mk)[a]) {
            const float2 X = A[i];
            const float2 k = ld2(K, a);
            const float rx = X.x * sc - k.x, ry = X.y * sc - k.y;
            if (S.loss_p == 2) {
                lsum += rx * rx + ry * ry;
                d = make_float2(2.f * rx * S.scale_data, 2.f * ry * S.scale_data);
            } else {
                lsum += fabsf(rx) + fabsf(ry);
                d = make_float2((rx > 0.f ? 1.f : (rx < 0.f ? -1.f : 0.f)) * S.scale_data,
                                (ry > 0.f ? 1.f : (ry < 0.f ? -1.f : 0.f)) * S.scale_data);
            }
        }
        A[i] = d;
    }
    // ... then into bit-reversed order by pairwise swaps, for the inverse DFT
    __syncthreads();
    for (int i = threadIdx.x; i < Ny * G; i += blockDim.x) {
        const int y = i / G, j = i % G;
        const int r = (int)bitrev(y, S.logNy);
        if (y < r) {
            const float2 t = A[y * G + j];
            A[y * G + j] = A[r * G + j];
            A[r * G + j] = t;
        }
    }
    fft_lds<true>(A, Ny, S.logNy, G, S.twy);
    for (int i = threadIdx.x; i < Ny * G; i += blockDim.x) {
        const int y = i / G, j = i % G;
        float2 v = A[i];
        v.x *= sc;
        v.y *= sc;
        base[(int64_t)y * Nz + z0 + j] = v;
    }
    const float s = block_sum(lsum * S.scale_data, red);
    if (threadIdx.x == 0 && partial) partial[blockIdx.x] = s;
}

// ---------------------------------------------------------------- update
// One thread per image pixel (e, y, z): gradient = sum over coils of buf +
// TV subgradient of Re and Im (forward differences along y and z within the
// echo image, lambda / Npix); optimiser step; TV loss partial.
__global__ __launch_bounds__(kBlock) void sense_update_kernel(SenseDev S, SenseOpt O,
                                                             const float2* __restrict__ img_in,
                                                             float2* __restrict__ img_out,
                                                             float2* __restrict__ m,
                                                             float2* __restrict__ v,
                                                             const float2* __restrict__ buf,
                                                             float* __restrict__ partial,
                                                             const int* __restrict__ stop) {
    __shared__ float red[kBlock / 64];
    if (stop && stop[0] != 0) return;
    const int Ny = S.Ny, Nz = S.Nz;
    const int64_t npix = (int64_t)S.E * Ny * Nz;
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    float tvl = 0.f;
    if (p < npix) {
        const int z = (int)(p % Nz), y = (int)((p / Nz) % Ny), e = (int)(p / ((int64_t)Ny * Nz));
        float2 g = make_float2(0.f, 0.f);
        for (int c = 0; c < S.Nc; ++c) {
            const float2 t = ld2(buf, (((int64_t)e * S.Nc + c) * Ny + y) * Nz + z);
            g.x += t.x;
            g.y += t.y;
        }
        const float2 u = ld2(img_in, p);
        if (O.scale_tv != 0.f) {
            float gx = 0.f, gy = 0.f, R = 0.f;
            auto sg = [](float d) { return d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f); };
            // forward neighbours: pairs (p, q)
            if (z + 1 < Nz) {
                const float2 q = ld2(img_in, p + 1);
                R += fabsf(q.x - u.x) + fabsf(q.y - u.y);
                gx -= sg(q.x - u.x);
                gy -= sg(q.y - u.y);
            }
            if (y + 1 < Ny) {
                const float2 q = ld2(img_in, p + Nz);
                R += fabsf(q.x - u.x) + fabsf(q.y - u.y);
                gx -= sg(q.x - u.x);
                gy -= sg(q.y - u.y);
            }
            // backward neighbours: pairs (q, p)
            if (z > 0) {
                const float2 q = ld2(img_in, p - 1);
                gx += sg(u.x - q.x);
                gy += sg(u.y - q.y);
            }
            if (y > 0) {
                const float2 q = ld2(img_in, p - Nz);
                gx += sg(u.x - q.x);
                gy += sg(u.y - q.y);
            }
            g.x += O.scale_tv * gx;
            g.y += O.scale_tv * gy;
            tvl = O.scale_tv * R;
        }
        float2 mm = m[p], vv = v[p], un;
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
        img_out[p] = un;
        m[p] = mm;
        v[p] = vv;
    }
    if (partial) {
        const float s = block_sum(tvl, red);
        if (threadIdx.x == 0) partial[blockIdx.x] = s;
    }
}

// Pure operators (autograd building blocks): forward A(I) and adjoint A^H(r).
__global__ __launch_bounds__(kBlock) void sense_mask_kernel(SenseDev S, float2* __restrict__ buf) {
    const int64_t n = (int64_t)S.E * S.Nc * S.Ny * S.Nz;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int64_t pix = i % ((int64_t)S.Ny * S.Nz);
    const int e = (int)(i / ((int64_t)S.Nc * S.Ny * S.Nz));
    if (!gload(S.mask)[(int64_t)e * S.Ny * S.Nz + pix]) buf[i] = make_float2(0.f, 0.f);
}

template <bool INV>
__global__ __launch_bounds__(kBlock) void sense_cols_plain_kernel(SenseDev S, float2* __restrict__ buf) {
    extern __shared__ float2 lds[];
    const int Ny = S.Ny, Nz = S.Nz, G = S.G;
    const int ngrp = Nz / G;
    const int ec = blockIdx.x / ngrp, z0 = (blockIdx.x % ngrp) * G;
    float2* base = buf + (int64_t)ec * Ny * Nz;
    for (int i = threadIdx.x; i < Ny * G; i += blockDim.x) {
        const int y = i / G, j = i % G;
        lds[bitrev(y, S.logNy) * G + j] = base[(int64_t)y * Nz + z0 + j];
    }
    fft_lds<INV>(lds, Ny, S.logNy, G, S.twy);
    for (int i = threadIdx.x; i < Ny * G; i += blockDim.x) {
        const int y = i / G, j = i % G;
        float2 v = lds[i];
        v.x *= S.rsqrtNy;
        v.y *= S.rsqrtNy;
        base[(int64_t)y * Nz + z0 + j] = v;
    }
}

// adjoint combine: out[e] = sum_c buf[e][c]
__global__ __launch_bounds__(kBlock) void sense_coil_sum_kernel(SenseDev S, const float2* __restrict__ buf,
                                                               float2* __restrict__ out) {
    const int64_t npix = (int64_t)S.E * S.Ny * S.Nz;
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= npix) return;
    const int64_t pix = p % ((int64_t)S.Ny * S.Nz);
    const int e = (int)(p / ((int64_t)S.Ny * S.Nz));
    float2 g = make_float2(0.f, 0.f);
    for (int c = 0; c < S.Nc; ++c) {
        const float2 t = ld2(buf, ((int64_t)e * S.Nc + c) * S.Ny * S.Nz + pix);
        g.x += t.x;
        g.y += t.y;
    }
    out[p] = g;
}

// ---------------------------------------------------------------- launchers
static size_t rows_lds(const SenseDev& S) { return (size_t)S.Nz * sizeof(float2); }
static size_t cols_lds(const SenseDev& S, int bufs) {
    return (size_t)bufs * S.Ny * S.G * sizeof(float2);
}

hipError_t sense_stage(int stage, const SenseDev& S, const SenseOpt& O, const float2* img_in,
                       float2* img_out, float2* m, float2* v, float2* buf, float* partial,
                       const int* stop, hipStream_t s) {
    const int nrow = S.E * S.Nc * S.Ny;
    const int ncol = S.E * S.Nc * (S.Nz / S.G);
    const int64_t npix = (int64_t)S.E * S.Ny * S.Nz;
    const int nupd = (int)((npix + kBlock - 1) / kBlock);
    switch (stage) {
    case 0:
        hipLaunchKernelGGL(sense_rows_kernel<0>, dim3(nrow), dim3(kBlock), rows_lds(S), s, S,
                           img_in, buf, stop);
        break;
    case 1:
        hipLaunchKernelGGL(sense_cols_kernel, dim3(ncol), dim3(kBlock), cols_lds(S, 1), s, S, buf,
                           partial, stop);
        break;
    case 2:
        hipLaunchKernelGGL(sense_rows_kernel<1>, dim3(nrow), dim3(kBlock), rows_lds(S), s, S,
                           nullptr, buf, stop);
        break;
    default:
        hipLaunchKernelGGL(sense_update_kernel, dim3(nupd), dim3(kBlock), 0, s, S, O, img_in,
                           img_out, m, v, buf, partial ? partial + ncol : nullptr, stop);
    }
    return hipGetLastError();
}

int64_t sense_partials(const SenseDev& S) {
    const int64_t npix = (int64_t)S.E * S.Ny * S.Nz;
    return (int64_t)S.E * S.Nc * (S.Nz / S.G) + (npix + kBlock - 1) / kBlock;
}

hipError_t sense_forward_op(const SenseDev& S, const float2* img, float2* out, hipStream_t s) {
    const int nrow = S.E * S.Nc * S.Ny;
    const int ncol = S.E * S.Nc * (S.Nz / S.G);
    const int64_t n = (int64_t)S.E * S.Nc * S.Ny * S.Nz;
    hipLaunchKernelGGL(sense_rows_kernel<0>, dim3(nrow), dim3(kBlock), rows_lds(S), s, S, img, out,
                       nullptr);
    hipLaunchKernelGGL(sense_cols_plain_kernel<false>, dim3(ncol), dim3(kBlock), cols_lds(S, 1), s,
                       S, out);
    hipLaunchKernelGGL(sense_mask_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock),
                       0, s, S, out);
    return hipGetLastError();
}

hipError_t sense_adjoint_op(const SenseDev& S, float2* buf /* in: r, clobbered */, float2* out,
                            hipStream_t s) {
    const int nrow = S.E * S.Nc * S.Ny;
    const int ncol = S.E * S.Nc * (S.Nz / S.G);
    const int64_t n = (int64_t)S.E * S.Nc * S.Ny * S.Nz;
    const int64_t npix = (int64_t)S.E * S.Ny * S.Nz;
    hipLaunchKernelGGL(sense_mask_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock),
                       0, s, S, buf);
    hipLaunchKernelGGL(sense_cols_plain_kernel<true>, dim3(ncol), dim3(kBlock), cols_lds(S, 1), s,
                       S, buf);
    hipLaunchKernelGGL(sense_rows_kernel<1>, dim3(nrow), dim3(kBlock), rows_lds(S), s, S, nullptr,
                       buf, nullptr);
    hipLaunchKernelGGL(sense_coil_sum_kernel, dim3((unsigned)((npix + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, s, S, buf, out);
    return hipGetLastError();
}

}  // namespace gc
