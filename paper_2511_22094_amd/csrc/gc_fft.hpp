// Power-of-two complex DFTs for a team of threads (four-step decomposition).
//
// A length-N transform, N = N1 * N2 (N1 = N2 or 2 N2), runs on a team of N2
// threads.  Thread p holds x[p + N2 n1], n1 < N1, in registers:
//   1. each thread: DFT of length N1 over n1 (registers, twiddles are
//      compile-time constants);
//   2. each thread: multiply entry k1 by w_N^(p k1);
//   3. transpose through LDS;
//   4. each thread: DFT(s) of length N2 over the team (registers).
// On return thread p holds X[p + N2 n1] in the same register slots, so a
// forward transform's output is directly the input of an inverse one.
// Forward: X[k] = sum_n x[n] exp(-2 pi i n k / N); inverse: exponent +.
// No scaling.
#pragma once
#include <hip/hip_runtime.h>

namespace gc {

// ------------------------------------------------- compile-time cos / sin
namespace fftct {
constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double sin_poly(double x) {   // |x| <= pi/4: Taylor series to 1e-17
    double x2 = x * x, term = x, sum = x;
    for (int n = 1; n < 12; ++n) {
        term *= -x2 / ((2.0 * n) * (2.0 * n + 1.0));
        sum += term;
    }
    return sum;
}
constexpr double cos_poly(double x) {
    double x2 = x * x, term = 1.0, sum = 1.0;
    for (int n = 1; n < 12; ++n) {
        term *= -x2 / ((2.0 * n - 1.0) * (2.0 * n));
        sum += term;
    }
    return sum;
}
// cos and sin of 2 pi k / L (L a power of two >= 1), reduced to the first
// octant exactly in integer arithmetic (8 k / L splits into octant + rest).
constexpr void cis(int k, int L, double* c, double* s) {
    k = ((k % L) + L) % L;
    if (L < 8) {   // multiples of pi/2 (L = 1, 2, 4) or pi/4 (handled below)
        const int q = (4 * k) / L;                 // exact when L | 4k
        if (4 * k == q * L) {
            const double cc[4] = {1.0, 0.0, -1.0, 0.0}, ss[4] = {0.0, 1.0, 0.0, -1.0};
            *c = cc[q];
            *s = ss[q];
            return;
        }
    }
    // angle = 2 pi k / L = (pi/4) (8k / L); octant o and remainder r in [0, L/8)
    const int o = (8 * k) / L;
    const double r = 2.0 * kPi * (double)(k - o * L / 8) / (double)L;   // [0, pi/4)
    const double sr = sin_poly(r), cr = cos_poly(r);
    const double h = 0.70710678118654752440084436210484903;            // cos(pi/4)
    // angle = o pi/4 + r
    double cb = 1.0, sb = 0.0;
    switch (o) {
    case 0: cb = 1.0; sb = 0.0; break;
    case 1: cb = h; sb = h; break;
    case 2: cb = 0.0; sb = 1.0; break;
    case 3: cb = -h; sb = h; break;
    case 4: cb = -1.0; sb = 0.0; break;
    case 5: cb = -h; sb = -h; break;
    case 6: cb = 0.0; sb = -1.0; break;
    default: cb = h; sb = -h; break;
    }
    *c = cb * cr - sb * sr;
    *s = sb * cr + cb * sr;
}
template <int L> struct Tab {
    float c[L > 0 ? L : 1], s[L > 0 ? L : 1];   // cos / sin (2 pi k / L)
    constexpr Tab() : c(), s() {
        for (int k = 0; k < L; ++k) {
            double cc = 0.0, ss = 0.0;
            cis(k, L, &cc, &ss);
            c[k] = (float)cc;
            s[k] = (float)ss;
        }
    }
};
}  // namespace fftct

__device__ __forceinline__ float2 fft_cmul(float2 a, float2 w) {
    return make_float2(a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x);
}

// In-register DFT of length L (a power of two <= 32) over a[0..L), in place,
// natural order in and out (iterative radix 2, decimation in time).
template <int L, bool INV>
__device__ __forceinline__ void dft_reg(float2* a) {
    if constexpr (L == 1) {
        return;
    } else {
        constexpr fftct::Tab<L> T{};
        constexpr int LOG = (L >= 32) ? 5 : (L >= 16) ? 4 : (L >= 8) ? 3 : (L >= 4) ? 2 : 1;
        // bit-reversal permutation: register renaming after unrolling
#pragma unroll
        for (int i = 0; i < L; ++i) {
            int r = 0;
#pragma unroll
            for (int b = 0; b < LOG; ++b) r |= ((i >> b) & 1) << (LOG - 1 - b);
            if (i < r) {
                const float2 t = a[i];
                a[i] = a[r];
                a[r] = t;
            }
        }
#pragma unroll
        for (int s = 1; s <= LOG; ++s) {
            const int m = 1 << s, h = m >> 1;
#pragma unroll
            for (int k = 0; k < h; ++k) {
                const int ti = k * (L / m);                  // w_m^k = w_L^(k L/m)
#pragma unroll
                for (int j = k; j < L; j += m) {
                    const float2 u = a[j], x = a[j + h];
                    float2 t;
                    if (ti == 0) {
                        t = x;
                    } else if (4 * ti == L) {                // w = -i (forward), +i (inverse)
                        t = INV ? make_float2(-x.y, x.x) : make_float2(x.y, -x.x);
                    } else {
                        const float2 w = make_float2(T.c[ti], INV ? T.s[ti] : -T.s[ti]);
                        t = fft_cmul(x, w);
                    }
                    a[j] = make_float2(u.x + t.x, u.y + t.y);
                    a[j + h] = make_float2(u.x - t.x, u.y - t.y);
                }
            }
        }
    }
}

template <int LOG> struct FftShape {
    static constexpr int N = 1 << LOG;
    static constexpr int N1 = 1 << ((LOG + 1) / 2);
    static constexpr int N2 = 1 << (LOG / 2);
};

// Team transform (see the top of this file).  `T` is this thread's view of
// the team's LDS transpose area: element (k1, n2) lives at
// T[k1 * rs + n2 * es] (rs, es in float2 units, chosen by the caller for
// bank spread).  `twN` holds w_N^k = exp(-2 pi i k / N), k < N (LDS).  Every
// thread of the block must call this the same number of times (it holds
// block barriers).
template <int LOG, bool INV>
__device__ __forceinline__ void fft_team(float2 (&a)[FftShape<LOG>::N1], int p, float2* T, int rs,
                                         int es, const float2* twN) {
    using Sh = FftShape<LOG>;
    constexpr int N = Sh::N, N1 = Sh::N1, N2 = Sh::N2;
    dft_reg<N1, INV>(a);
#pragma unroll
    for (int k1 = 1; k1 < N1; ++k1) {
        float2 w = twN[(p * k1) & (N - 1)];
        if (INV) w.y = -w.y;
        a[k1] = fft_cmul(a[k1], w);
    }
    __syncthreads();   // the previous use of T is finished
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) T[k1 * rs + p * es] = a[k1];
    __syncthreads();
    if constexpr (N1 == N2) {
#pragma unroll
        for (int n2 = 0; n2 < N2; ++n2) a[n2] = T[p * rs + n2 * es];
        dft_reg<N2, INV>(a);
    } else {   // N1 = 2 N2: entries k1 = p and p + N2, interleaved back into a[]
        float2 b0[N2], b1[N2];
#pragma unroll
        for (int n2 = 0; n2 < N2; ++n2) {
            b0[n2] = T[p * rs + n2 * es];
            b1[n2] = T[(p + N2) * rs + n2 * es];
        }
        dft_reg<N2, INV>(b0);
        dft_reg<N2, INV>(b1);
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) {
            a[2 * k2] = b0[k2];
            a[2 * k2 + 1] = b1[k2];
        }
    }
}

}  // namespace gc
