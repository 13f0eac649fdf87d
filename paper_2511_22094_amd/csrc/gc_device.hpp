// Device-side building blocks of the voxel-parallel fitting path:
// precision traits, the counter-based random stream, and the forward
// models of the registry with their hand-written adjoints.
//
// Everything here is instantiated twice: Real = float is the production
// path (fast hardware transcendentals, recurrences over uniformly spaced
// echoes), Real = double is the deterministic test path that mirrors the
// FP64 definition step by step.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gc {

constexpr int kMaxP = 9;          // widest model (3-pool GRE)
constexpr int kBlock = 256;       // threads per block for every voxel kernel

enum ModelKind { MONOEXP_T2S = 0, MONOEXP_R2S = 1, GRE3 = 2, DWI2 = 3, LINEAR3 = 4 };

// --------------------------------------------------------------------------
// Precision traits.  FP32 uses the hardware transcendental unit directly:
// v_exp_f32 / v_log_f32 work in base 2, v_sin_f32 / v_cos_f32 take their
// argument in revolutions (sin(2 pi x)), which is exactly the form the
// Box-Muller angle and the GRE phase 2 pi df TE already have.
// --------------------------------------------------------------------------
template <typename R> struct Math;

template <> struct Math<float> {
    static constexpr float kLog2e = 1.44269504088896341f;
    static __device__ __forceinline__ float exp(float x) {
        return __builtin_amdgcn_exp2f(x * kLog2e);
    }
    // 2^x: for exponents whose log2(e) factor is folded into a constant
    static __device__ __forceinline__ float exp2(float x) { return __builtin_amdgcn_exp2f(x); }
    static __device__ __forceinline__ float ln(float x) {
        return __builtin_amdgcn_logf(x) * 0.693147180559945309f;
    }
    static __device__ __forceinline__ float sin2pi(float rev) {
        return __builtin_amdgcn_sinf(rev);
    }
    static __device__ __forceinline__ float cos2pi(float rev) {
        return __builtin_amdgcn_cosf(rev);
    }
    static __device__ __forceinline__ float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    // -2 ln(u) for Box-Muller, straight from the base-2 logarithm
    static __device__ __forceinline__ float m2ln(float u) {
        return __builtin_amdgcn_logf(u) * -1.38629436111989062f;
    }
    // sine / cosine of an angle in radians
    static __device__ __forceinline__ float sin(float x) {
        return __builtin_amdgcn_sinf(x * 0.159154943091895336f);
    }
    static __device__ __forceinline__ float cos(float x) {
        return __builtin_amdgcn_cosf(x * 0.159154943091895336f);
    }
};

template <> struct Math<double> {
    static constexpr double kTwoPi = 6.28318530717958647692;
    static __device__ __forceinline__ double exp(double x) { return ::exp(x); }
    static __device__ __forceinline__ double ln(double x) { return ::log(x); }
    static __device__ __forceinline__ double sin2pi(double rev) { return ::sin(kTwoPi * rev); }
    static __device__ __forceinline__ double cos2pi(double rev) { return ::cos(kTwoPi * rev); }
    static __device__ __forceinline__ double sqrt(double x) { return ::sqrt(x); }
    static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
    static __device__ __forceinline__ double m2ln(double u) { return -2.0 * ::log(u); }
    static __device__ __forceinline__ double sin(double x) { return ::sin(x); }
    static __device__ __forceinline__ double cos(double x) { return ::cos(x); }
};

// --------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11).  The key (the job's seed) is the
// same for every lane, so the key schedule stays in scalar registers; each
// round costs two 32x32->64 multiplies and two three-way XORs per lane.
// --------------------------------------------------------------------------
struct U4 { uint32_t x, y, z, w; };

// a ^ b ^ c as one VALU instruction (gfx950 three-input bitwise op; the
// truth table of XOR3 over inputs 0xF0, 0xCC, 0xAA is 0x96)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        uint32_t nx = xor3((uint32_t)(p1 >> 32), c.y, k0);
        uint32_t nz = xor3((uint32_t)(p0 >> 32), c.w, k1);
        c.y = (uint32_t)p1;
        c.w = (uint32_t)p0;
        c.x = nx;
        c.z = nz;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// (2k+1) / 2^24 from the top 23 bits k: exact in both precisions, in (0,1).
// FP32: one funnel shift places k under the exponent of 1.0, giving
// x = 1 + k 2^-23 exactly; x - (1 - 2^-24) = (2k+1) 2^-24 is representable
// (24 significant bits), so the subtraction is exact as well.
template <typename R> __device__ __forceinline__ R uniform01(uint32_t w);
template <> __device__ __forceinline__ float uniform01<float>(uint32_t w) {
    const uint32_t bits = __builtin_amdgcn_alignbit(0x7Fu, w, 9);   // 0x3F800000 | w >> 9
    return __builtin_bit_cast(float, bits) - 0x1.fffffep-1f;        // 1 - 2^-24
}
template <> __device__ __forceinline__ double uniform01<double>(uint32_t w) {
    return ((double)(w >> 9) + 0.5) * 0x1p-23;
}

// lo <= x <= hi (x finite, lo <= hi).  FP32: the median of (x, lo, hi) is x
// exactly when x lies in the box -- one med3 and one compare per coordinate.
__device__ __forceinline__ bool in_box(float x, float lo, float hi) {
    return __builtin_amdgcn_fmed3f(x, lo, hi) == x;
}
__device__ __forceinline__ bool in_box(double x, double lo, double hi) {
    return x >= lo && x <= hi;
}

// Draws of one MH step: P normals (Box-Muller on consecutive word pairs) and
// the acceptance uniform (the word after the last pair).  Counter =
// (voxel, chain | purpose << 16, iteration, block).
template <int P> struct StepDraws {
    static constexpr int kPairs = (P + 1) / 2;
    static constexpr int kWords = 2 * kPairs + 1;
    static constexpr int kBlocks = (kWords + 3) / 4;
};

template <typename R, int P>
__device__ __forceinline__ void mh_draws(uint32_t v, uint32_t c, uint32_t t, uint32_t k0,
                                         uint32_t k1, R (&z)[P], R& u_acc) {
    constexpr int NB = StepDraws<P>::kBlocks;
    uint32_t w[4 * NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        U4 o = philox4x32_10(U4{v, c, t, (uint32_t)b}, k0, k1);
        w[4 * b + 0] = o.x;
        w[4 * b + 1] = o.y;
        w[4 * b + 2] = o.z;
        w[4 * b + 3] = o.w;
    }
#pragma unroll
    for (int i = 0; i < StepDraws<P>::kPairs; ++i) {
        R u1 = uniform01<R>(w[2 * i]);
        R u2 = uniform01<R>(w[2 * i + 1]);
        R r = Math<R>::sqrt(Math<R>::m2ln(u1));
        if (2 * i < P) z[2 * i] = r * Math<R>::cos2pi(u2);
        if (2 * i + 1 < P) z[2 * i + 1] = r * Math<R>::sin2pi(u2);
    }
    u_acc = uniform01<R>(w[StepDraws<P>::kWords - 1]);
}

// --------------------------------------------------------------------------
// Acquisition as seen by the kernels (device pointers, uniform across lanes).
// TE in ms; b already multiplied by 1e-3 (so b*D is dimensionless with D in
// um^2/ms); bvec [M][3].  `uniform` marks equally spaced echoes te0 + m*dte,
// which lets the FP32 path replace per-echo exponentials by recurrences.
// --------------------------------------------------------------------------
struct AcqDev {
    const float* te;
    const float* bval;
    const float* bvec;
    const double* te_d;
    const double* bval_d;
    const double* bvec_d;
    int M;
    int uniform;
    float te0, dte;
    double te0_d, dte_d;
    // runs of consecutive measurements with equal b (a shell, in acquisition
    // order): run r ends (exclusive) at run_end[r]; one run when there is no b
    const int* run_end;
    int nrun;
};

// Address-space views of device pointers.  Every buffer the kernels touch
// lives in device global memory; saying so lets the compiler use global
// (not flat) loads for per-lane data, and scalar loads through the scalar
// cache for the acquisition tables, which every lane reads at the same
// index and which no kernel writes.
template <class T> using gmem_cptr = const __attribute__((address_space(1))) T*;
template <class T> using cmem_cptr = const __attribute__((address_space(4))) T*;
template <class T> __device__ __forceinline__ gmem_cptr<T> gload(const T* p) {
    return (gmem_cptr<T>)p;
}
template <class T> __device__ __forceinline__ cmem_cptr<T> cload(const T* p) {
    return (cmem_cptr<T>)p;
}

template <typename R> struct AcqView;
template <> struct AcqView<float> {
    static __device__ __forceinline__ float te(const AcqDev& a, int m) { return cload(a.te)[m]; }
    static __device__ __forceinline__ float b(const AcqDev& a, int m) { return cload(a.bval)[m]; }
    static __device__ __forceinline__ float g(const AcqDev& a, int m, int k) {
        return cload(a.bvec)[3 * m + k];
    }
    static __device__ __forceinline__ float te0(const AcqDev& a) { return a.te0; }
    static __device__ __forceinline__ float dte(const AcqDev& a) { return a.dte; }
};
template <> struct AcqView<double> {
    static __device__ __forceinline__ double te(const AcqDev& a, int m) {
        return cload(a.te_d)[m];
    }
    static __device__ __forceinline__ double b(const AcqDev& a, int m) {
        return cload(a.bval_d)[m];
    }
    static __device__ __forceinline__ double g(const AcqDev& a, int m, int k) {
        return cload(a.bvec_d)[3 * m + k];
    }
    static __device__ __forceinline__ double te0(const AcqDev& a) { return a.te0_d; }
    static __device__ __forceinline__ double dte(const AcqDev& a) { return a.dte_d; }
};

// Recurrences over echoes are used only in FP32 with equally spaced echoes;
// FP64 always evaluates the closed forms echo by echo.
template <typename R> struct UseRecur { static constexpr bool value = false; };
template <> struct UseRecur<float> { static constexpr bool value = true; };

// Compile-time evaluation choices of a kernel instantiation:
//   MAXM  > 0: measurement loop fully unrolled up to MAXM (data can sit in
//              registers); 0: runtime loop.
//   EXACT = 1: the acquisition has exactly MAXM measurements (no guards).
//   RECUR = 1: echo recurrence on, 2: off, 0: decided at run time from the
//              acquisition (equally spaced echoes).
enum { kRecurRuntime = 0, kRecurOn = 1, kRecurOff = 2 };

template <typename R, int RECUR> __device__ __forceinline__ bool recur_on(const AcqDev& a) {
    if constexpr (!UseRecur<R>::value || RECUR == kRecurOff) return false;
    else if constexpr (RECUR == kRecurOn) return true;
    else return a.uniform != 0;
}

// Compile-time trip counts unroll fully; a run-time count unrolls by 8, so
// that the loads of 8 measurements are in flight together.  (The pragma
// names the template parameter MAXM of the enclosing function.)
#define GC_FOR_MEAS(m, MAXM, M)                                                 \
    _Pragma("unroll(MAXM > 0 ? MAXM : 8)")                                     \
    for (int m = 0; m < ((MAXM) > 0 ? (MAXM) : (M)); ++m)                      \
        if ((MAXM) == 0 || EXACT || m < (M))

// --------------------------------------------------------------------------
// Forward models.  Each provides
//   sse<MAXM>(th, Y, a)          sum_j (y_j - s_j)^2            (MH path)
//   grad<MAXM>(th, Y, D, a, g)   g = J^T d with d_j = D(j, s_j)  (fits, VJP)
//   forward(th, a, S)            S(j, s_j) for every component
// Y.re(m) / Y.im(m) return the measured real / imaginary part of
// measurement m (real models use .re only); D.re(m, s) / D.im(m, s) return
// dLoss/ds for that component (and may accumulate the loss itself); S.re /
// S.im receive forward values.  Component order in memory is the M real
// parts, then the M imaginary parts.
// --------------------------------------------------------------------------

// s = S0 exp(k TE) with k = -1/T2* (monoexp_t2s) or -R2* 1e-3 (monoexp_r2s)
template <typename R, int KIND> struct MonoExp {
    static constexpr int P = 2;
    static constexpr bool kComplex = false;
    static __device__ __forceinline__ R rate(const R* th) {
        if (KIND == MONOEXP_T2S) return -Math<R>::rcp(th[1]);
        return -th[1] * (R)1e-3;
    }
    template <int MAXM, int EXACT = 0, int RECUR = kRecurRuntime, class Y>
    static __device__ __forceinline__ R sse(const R* th, const Y& y, const AcqDev& a) {
        R k = rate(th);
        R acc0 = 0, acc1 = 0;
        if (recur_on<R, RECUR>(a)) {
            R e = th[0] * Math<R>::exp(k * AcqView<R>::te0(a));
            R q = Math<R>::exp(k * AcqView<R>::dte(a));
            GC_FOR_MEAS(m, MAXM, a.M) {
                R r = (R)y.re(m) - e;
                if (m & 1) acc1 += r * r; else acc0 += r * r;
                e *= q;
            }
        } else {
            GC_FOR_MEAS(m, MAXM, a.M) {
                R r = (R)y.re(m) - th[0] * Math<R>::exp(k * AcqView<R>::te(a, m));
                if (m & 1) acc1 += r * r; else acc0 += r * r;
            }
        }
        return acc0 + acc1;
    }
    template <int MAXM, int EXACT = 0, int RECUR = kRecurRuntime, class D>
    static __device__ __forceinline__ void grad(const R* th, D& d, const AcqDev& a, R* g) {
        R k = rate(th);
        R gs = 0, gk = 0;   // gk accumulates sum d * s * TE
        GC_FOR_MEAS(m, MAXM, a.M) {
            R te = AcqView<R>::te(a, m);
            R E = Math<R>::exp(k * te);
            R s = th[0] * E;
            R dj = d.re(m, s);
            gs += dj * E;
            gk += dj * s * te;
        }
        g[0] = gs;
        // ds/dT2 = S0 E TE / T2^2 ; ds/dR2 = -S0 E TE 1e-3
        if (KIND == MONOEXP_T2S) g[1] = gk * (k * k);
        else g[1] = -gk * (R)1e-3;
    }
    template <class S>
    static __device__ __forceinline__ void forward(const R* th, const AcqDev& a, S& out) {
        R k = rate(th);
        for (int m = 0; m < a.M; ++m) out.re(m, th[0] * Math<R>::exp(k * AcqView<R>::te(a, m)));
    }
};

// s = sum_k A_k exp(-TE / tau_k), tau = (10, 30, 80) ms: linear in A.
template <typename R> struct Linear3 {
    static constexpr int P = 3;
    static constexpr bool kComplex = false;
    static __device__ __forceinline__ R rk(int k) {
        return k == 0 ? (R)(-1.0 / 10.0) : (k == 1 ? (R)(-1.0 / 30.0) : (R)(-1.0 / 80.0));
    }
    template <int MAXM, int EXACT = 0, int RECUR = kRecurRuntime, class Y>
    static __device__ __forceinline__ R sse(const R* th, const Y& y, const AcqDev& a) {
        R acc = 0;
        GC_FOR_MEAS(m, MAXM, a.M) {
            R te = AcqView<R>::te(a, m);
            R s = th[0] * Math<R>::exp(rk(0) * te) + th[1] * Math<R>::exp(rk(1) * te) +
                  th[2] * Math<R>::exp(rk(2) * te);
            R r = (R)y.re(m) - s;
            acc += r * r;
        }
        return acc;
    }
    template <int MAXM, int EXACT = 0, int RECUR = kRecurRuntime, class D>
    static __device__ __forceinline__ void grad(const R* th, D& d, const AcqDev& a, R* g) {
        g[0] = g[1] = g[2] = 0;
        GC_FOR_MEAS(m, MAXM, a.M) {
            R te = AcqView<R>::te(a, m);
            R e0 = Math<R>::exp(rk(0) * te), e1 = Math<R>::exp(rk(1) * te),
              e2 = Math<R>::exp(rk(2) * te);
            R dj = d.re(m, th[0] * e0 + th[1] * e1 + th[2] * e2);
            g[0] += dj * e0;
            g[1] += dj * e1;
            g[2] += dj * e2;
        }
    }
    template <class S>
    static __device__ __forceinline__ void forward(const R* th, const AcqDev& a, S& out) {
        for (int m = 0; m < a.M; ++m) {
            R te = AcqView<R>::te(a, m);
            out.re(m, th[0] * Math<R>::exp(rk(0) * te) + th[1] * Math<R>::exp(rk(1) * te) +
                       th[2] * Math<R>::exp(rk(2) * te));
        }
    }
};

// Three-pool complex GRE: s = sum_k A_k exp(-TE/T2_k) exp(i 2 pi df_k TE 1e-3).
// Pool term u_k(TE) = exp(-TE/T2_k + i 2 pi df_k TE 1e-3) (unit amplitude).
// With equally spaced echoes, u_k(TE + dte) = u_k(TE) q_k: one complex
// multiply per echo and pool instead of exp + sin + cos.
template <typename R> struct Gre3 {
    static constexpr int P = 9;
    static constexpr bool kComplex = true;

    // per-pool decay rate -1/T2 and phase rate df 1e-3 (revolutions per ms)
    static __device__ __forceinline__ void rates(const R* th, R* kr, R* kp) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            kr[k] = -Math<R>::rcp(th[3 + k]);
            kp[k] = th[6 + k] * (R)1e-3;
        }
    }
    static __device__ __forceinline__ void cexp(R re_exp, R rev, R& cr, R& ci) {
        R mag = Math<R>::exp(re_exp);
        cr = mag * Math<R>::cos2pi(rev);
        ci = mag * Math<R>::sin2pi(rev);
    }

    template <int MAXM, int EXACT = 0, int RECUR = kRecurRuntime, class Y>
    static __device__ __forceinline__ R sse(const R* th, const Y& y, const AcqDev& a) {
        R kr[3], kp[3];
        rates(th, kr, kp);
        R accr = 0, acci = 0;
        if (recur_on<R, RECUR>(a)) {
            R te0 = AcqView<R>::te0(a), dte = AcqView<R>::dte(a);
            R zr[3], zi[3], qr[3], qi[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                cexp(kr[k] * dte, kp[k] * dte, qr[k], qi[k]);
                if (te0 == dte) {   // first echo one step after TE = 0: z = A q
                    zr[k] = th[k] * qr[k];
                    zi[k] = th[k] * qi[k];
                } else {
                    cexp(kr[k] * te0, kp[k] * te0, zr[k], zi[k]);
                    zr[k] *= th[k];
                    zi[k] *= th[k];
                }
            }
            GC_FOR_MEAS(m, MAXM, a.M) {
                R sr = zr[0] + zr[1] + zr[2];
                R si = zi[0] + zi[1] + zi[2];
                R rr = (R)y.re(m) - sr;
                R ri = (R)y.im(m) - si;
                accr += rr * rr;
                acci += ri * ri;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    R nr = zr[k] * qr[k] - zi[k] * qi[k];
                    R ni = zr[k] * qi[k] + zi[k] * qr[k];
                    zr[k] = nr;
                    zi[k] = ni;
                }
            }
        } else {
            GC_FOR_MEAS(m, MAXM, a.M) {
                R te = AcqView<R>::te(a, m);
                R sr = 0, si = 0;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    R cr, ci;
                    cexp(kr[k] * te, kp[k] * te, cr, ci);
                    sr += th[k] * cr;
                    si += th[k] * ci;
                }
                R rr = (R)y.re(m) - sr;
                R ri = (R)y.im(m) - si;
                accr += rr * rr;
                acci += ri * ri;
            }
        }
        return accr + acci;
    }

    template <int MAXM, int EXACT = 0, int RECUR = kRecurRuntime, class D>
    static __device__ __forceinline__ void grad(const R* th, D& d, const AcqDev& a, R* g) {
        R kr[3], kp[3];
        rates(th, kr, kp);
        R gA[3] = {0, 0, 0}, gT[3] = {0, 0, 0}, gF[3] = {0, 0, 0};
        const bool rec = recur_on<R, RECUR>(a);
        R ur[3], ui[3], qr[3], qi[3];
        if (rec) {
            R te0 = AcqView<R>::te0(a), dte = AcqView<R>::dte(a);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                cexp(kr[k] * dte, kp[k] * dte, qr[k], qi[k]);
                if (te0 == dte) {   // first echo one step after TE = 0: u = q
                    ur[k] = qr[k];
                    ui[k] = qi[k];
                } else {
                    cexp(kr[k] * te0, kp[k] * te0, ur[k], ui[k]);
                }
            }
        }
        GC_FOR_MEAS(m, MAXM, a.M) {
            R te = AcqView<R>::te(a, m);
            if (!rec) {
#pragma unroll
                for (int k = 0; k < 3; ++k) cexp(kr[k] * te, kp[k] * te, ur[k], ui[k]);
            }
            R sr = th[0] * ur[0] + th[1] * ur[1] + th[2] * ur[2];
            R si = th[0] * ui[0] + th[1] * ui[1] + th[2] * ui[2];
            R dr = d.re(m, sr);
            R di = d.im(m, si);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                R p = dr * ur[k] + di * ui[k];     // Re(conj(d) u_k)
                R q = di * ur[k] - dr * ui[k];     // Re(conj(d) i u_k)
                gA[k] += p;
                gT[k] += p * te;
                gF[k] += q * te;
            }
            if (rec) {
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    R nr = ur[k] * qr[k] - ui[k] * qi[k];
                    R ni = ur[k] * qi[k] + ui[k] * qr[k];
                    ur[k] = nr;
                    ui[k] = ni;
                }
            }
        }
        const R w = (R)6.283185307179586477e-3;   // 2 pi 1e-3
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            g[k] = gA[k];
            g[3 + k] = gT[k] * th[k] * (kr[k] * kr[k]);   // A TE / T2^2
            g[6 + k] = gF[k] * th[k] * w;
        }
    }
    template <class S>
    static __device__ __forceinline__ void forward(const R* th, const AcqDev& a, S& out) {
        R kr[3], kp[3];
        rates(th, kr, kp);
        for (int m = 0; m < a.M; ++m) {
            R te = AcqView<R>::te(a, m);
            R sr = 0, si = 0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                R cr, ci;
                cexp(kr[k] * te, kp[k] * te, cr, ci);
                sr += th[k] * cr;
                si += th[k] * ci;
            }
            out.re(m, sr);
            out.im(m, si);
        }
    }
};

// Stick + ball diffusion: s = f exp(-b Da (g.n)^2) + (1-f) exp(-b De),
// n = (sin th cos ph, sin th sin ph, cos th), b pre-scaled by 1e-3.
template <typename R> struct Dwi2 {
    static constexpr int P = 5;
    static constexpr bool kComplex = false;
    static __device__ __forceinline__ void dir(const R* th, R* n) {
        R st = Math<R>::sin(th[3]), ct = Math<R>::cos(th[3]);
        R sp = Math<R>::sin(th[4]), cp = Math<R>::cos(th[4]);
        n[0] = st * cp;
        n[1] = st * sp;
        n[2] = ct;
        n[3] = ct * cp;   // dn/dtheta
        n[4] = ct * sp;
        n[5] = -st;
        n[6] = -st * sp;  // dn/dphi (z component 0)
        n[7] = st * cp;
    }
    template <int MAXM, int EXACT = 0, int RECUR = kRecurRuntime, class Y>
    static __device__ __forceinline__ R sse(const R* th, const Y& y, const AcqDev& a) {
        R n[8];
        dir(th, n);
        R acc = 0;
        if constexpr (MAXM == 0) {
            // run-time loop: shell by shell, the ball term once per shell and
            // no branch in the measurement loop (same values as below)
            int m = 0;
            for (int r = 0; r < a.nrun; ++r) {
                const int mend = cload(a.run_end)[r];
                const R b = AcqView<R>::b(a, m);
                const R ball = ((R)1 - th[0]) * Math<R>::exp(-b * th[2]);
                if constexpr (sizeof(R) == 4) {
                    // FP32: log2(e) folded into the shell constant, one exp2
                    const R cb = -b * th[1] * Math<R>::kLog2e;
                    // as in grad(); unrolled by 4 (measured 5-6 % faster than 8
                    // for the MH kernels, whose eight-wide body waited longer
                    // on its scalar and LDS reads)
                    cmem_cptr<float> gp = cload(a.bvec) + 3 * m;
#pragma unroll 4
                    for (; m < mend; ++m, gp += 3) {
                        R x = gp[0] * n[0] + gp[1] * n[1] + gp[2] * n[2];
                        R s = th[0] * Math<R>::exp2(cb * x * x) + ball;
                        R rr = (R)y.re(m) - s;
                        acc += rr * rr;
                    }
                } else {
#pragma unroll 8
                    for (; m < mend; ++m) {
                        R x = AcqView<R>::g(a, m, 0) * n[0] + AcqView<R>::g(a, m, 1) * n[1] +
                              AcqView<R>::g(a, m, 2) * n[2];
                        R s = th[0] * Math<R>::exp(-b * th[1] * x * x) + ball;
                        R rr = (R)y.re(m) - s;
                        acc += rr * rr;
                    }
                }
            }
            return acc;
        }
        // the ball term depends on b only: on a shell (consecutive equal b,
        // a uniform test) it is reused instead of recomputed -- same values
        R bprev = (R)-1, ball = 0;
        GC_FOR_MEAS(m, MAXM, a.M) {
            R x = AcqView<R>::g(a, m, 0) * n[0] + AcqView<R>::g(a, m, 1) * n[1] +
                  AcqView<R>::g(a, m, 2) * n[2];
            R b = AcqView<R>::b(a, m);
            if (__builtin_expect(b != bprev, 0)) {   // uniform: a scalar branch
                ball = ((R)1 - th[0]) * Math<R>::exp(-b * th[2]);
                bprev = b;
            }
            R s = th[0] * Math<R>::exp(-b * th[1] * x * x) + ball;
            R r = (R)y.re(m) - s;
            acc += r * r;
        }
        return acc;
    }
    template <int MAXM, int EXACT = 0, int RECUR = kRecurRuntime, class D>
    static __device__ __forceinline__ void grad(const R* th, D& d, const AcqDev& a, R* g) {
        R n[8];
        dir(th, n);
        R gf = 0, gda = 0, gde = 0, gn0 = 0, gn1 = 0, gn2 = 0;
        if constexpr (MAXM == 0 && sizeof(R) == 4) {
            // Shell by shell with the shell constants b, Ee factored out of the
            // sums: per measurement q = d Ea, then
            //   gf  += q - Ee d,   gda += b q x^2,   gde += b Ee d,
            //   gn  += b q x g,
            // where the b and Ee products are applied once per shell.
            int m = 0;
            for (int r = 0; r < a.nrun; ++r) {
                const int mend = cload(a.run_end)[r];
                const R b = AcqView<R>::b(a, m);
                const R Ee = Math<R>::exp(-b * th[2]);
                const R cb = -b * th[1] * Math<R>::kLog2e;
                const R ball = ((R)1 - th[0]) * Ee;
                R sq = 0, sd = 0, sx = 0, s0 = 0, s1 = 0, s2 = 0;
                // the directions through one scalar pointer walked along the
                // run: the unrolled body then reads them with a few wide
                // scalar loads at constant offsets (measured 6 % faster per
                // Adam+TV iteration than an address computed per measurement)
                cmem_cptr<float> gp = cload(a.bvec) + 3 * m;
#pragma unroll 8
                for (; m < mend; ++m, gp += 3) {
                    const R g0 = gp[0], g1 = gp[1], g2 = gp[2];
                    R x = g0 * n[0] + g1 * n[1] + g2 * n[2];
                    R Ea = Math<R>::exp2(cb * x * x);
                    R dj = d.re(m, th[0] * Ea + ball);
                    R q = dj * Ea;
                    sq += q;
                    sd += dj;
                    R qx = q * x;
                    sx += qx * x;
                    s0 += qx * g0;
                    s1 += qx * g1;
                    s2 += qx * g2;
                }
                gf += sq - Ee * sd;
                gda += b * sx;
                gde += b * Ee * sd;
                gn0 += b * s0;
                gn1 += b * s1;
                gn2 += b * s2;
            }
        } else if constexpr (MAXM == 0) {
            int m = 0;
            for (int r = 0; r < a.nrun; ++r) {
                const int mend = cload(a.run_end)[r];
                const R b = AcqView<R>::b(a, m);
                const R Ee = Math<R>::exp(-b * th[2]);
#pragma unroll 8
                for (; m < mend; ++m) {
                    R g0 = AcqView<R>::g(a, m, 0), g1 = AcqView<R>::g(a, m, 1),
                      g2 = AcqView<R>::g(a, m, 2);
                    R x = g0 * n[0] + g1 * n[1] + g2 * n[2];
                    R Ea = Math<R>::exp(-b * th[1] * x * x);
                    R dj = d.re(m, th[0] * Ea + ((R)1 - th[0]) * Ee);
                    gf += dj * (Ea - Ee);
                    R t = dj * b * Ea;
                    gda += t * x * x;
                    gde += dj * b * Ee;
                    R tx = t * x;
                    gn0 += tx * g0;
                    gn1 += tx * g1;
                    gn2 += tx * g2;
                }
            }
        } else {
            R bprev = (R)-1, Ee = 0;   // ball term reused along a shell (see sse)
            GC_FOR_MEAS(m, MAXM, a.M) {
                R g0 = AcqView<R>::g(a, m, 0), g1 = AcqView<R>::g(a, m, 1),
                  g2 = AcqView<R>::g(a, m, 2);
                R b = AcqView<R>::b(a, m);
                R x = g0 * n[0] + g1 * n[1] + g2 * n[2];
                R Ea = Math<R>::exp(-b * th[1] * x * x);
                if (__builtin_expect(b != bprev, 0)) {   // uniform: a scalar branch
                    Ee = Math<R>::exp(-b * th[2]);
                    bprev = b;
                }
                R dj = d.re(m, th[0] * Ea + ((R)1 - th[0]) * Ee);
                gf += dj * (Ea - Ee);
                R t = dj * b * Ea;      // d * b * Ea
                gda += t * x * x;
                gde += dj * b * Ee;
                R tx = t * x;
                gn0 += tx * g0;
                gn1 += tx * g1;
                gn2 += tx * g2;
            }
        }
        g[0] = gf;
        g[1] = -th[0] * gda;
        g[2] = -((R)1 - th[0]) * gde;
        R c = (R)-2 * th[0] * th[1];
        g[3] = c * (gn0 * n[3] + gn1 * n[4] + gn2 * n[5]);
        g[4] = c * (gn0 * n[6] + gn1 * n[7]);
    }
    template <class S>
    static __device__ __forceinline__ void forward(const R* th, const AcqDev& a, S& out) {
        R n[8];
        dir(th, n);
        for (int m = 0; m < a.M; ++m) {
            R x = AcqView<R>::g(a, m, 0) * n[0] + AcqView<R>::g(a, m, 1) * n[1] +
                  AcqView<R>::g(a, m, 2) * n[2];
            R b = AcqView<R>::b(a, m);
            out.re(m, th[0] * Math<R>::exp(-b * th[1] * x * x) +
                       ((R)1 - th[0]) * Math<R>::exp(-b * th[2]));
        }
    }
};

template <int KIND, typename R> struct ModelOf;
template <typename R> struct ModelOf<MONOEXP_T2S, R> { using T = MonoExp<R, MONOEXP_T2S>; };
template <typename R> struct ModelOf<MONOEXP_R2S, R> { using T = MonoExp<R, MONOEXP_R2S>; };
template <typename R> struct ModelOf<GRE3, R> { using T = Gre3<R>; };
template <typename R> struct ModelOf<DWI2, R> { using T = Dwi2<R>; };
template <typename R> struct ModelOf<LINEAR3, R> { using T = Linear3<R>; };

// Effective measurement count for register arrays sized at compile time.
template <int KIND, int MAXM> struct MeasEff {
    static constexpr int value = (KIND == GRE3 ? 2 * MAXM : MAXM);
};

// --------------------------------------------------------------------------
// Wave / block reductions (wave64).
// --------------------------------------------------------------------------
template <typename T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over a block of kBlock threads in a fixed order; result valid in thread 0.
template <typename T> __device__ __forceinline__ T block_sum(T v, T* lds /*[kBlock/64]*/) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    T r = 0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < kBlock / 64; ++i) r += lds[i];
    }
    return r;
}

}  // namespace gc
