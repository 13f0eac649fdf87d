// Image reconstruction (gc_sense.hip): descriptors and launchers.
#pragma once
#include "gc_internal.hpp"

namespace gc {

constexpr int kSenseMinNz = 16;       // smallest z length (one y-pass tile of columns)
constexpr int kSenseMaxN = 1024;      // largest transform length along y or z
// Columns per y-pass tile: G = min(16, 4096 / Ny), so a tile holds at most
// 4096 complex values.
__host__ __device__ constexpr int sense_tile_cols(int logNy) {
    return (4096 >> logNy) < 16 ? (4096 >> logNy) : 16;
}
struct SenseDev {
    int E, Nc, Ny, Nz, logNy, logNz;
    int G;                            // columns per y-pass tile (sense_tile_cols)
    int64_t S;                        // sampled (e, y, z) entries over all echoes
    float rsqrtNy, rsqrtNz;           // unitary scaling of each 1D transform
    const float2* coils;              // [Nc][Ny][Nz]
    // Samples are numbered tile by tile: echo e, tile z / G, row y, column z % G.
    const float2* kc;                 // measured samples [Nc][S] in that order
    const uint32_t* tinfo;            // [E][Nz/G][Ny]: (index of the row's first sample
                                      //  within its tile) << 16 | G-bit mask of the row
    const int32_t* tbase;             // [E][Nz/G]: index of the tile's first sample
    const float2* twy;                // [Ny] exp(-2 pi i k / Ny)
    const float2* twz;                // [Nz]
    float scale_data;                 // 1 / Nk
    int loss_p;
};
struct SenseOpt {
    int optimizer;
    float lr, beta1, beta2, eps, momentum, rho, omb1, omb2, omrho;
    float c1, c2;                     // bias corrections of this iteration
    float scale_tv;                   // lambda / Npix
};

// Measured samples, dense [E][Nc][Ny][Nz] -> S.kc (needs S.tinfo, S.tbase).
hipError_t sense_pack_kspace(const SenseDev& S, const float2* dense, float2* kc, hipStream_t s);
// buf = F_z(C_c I_e) for every (e, c, y) row (the first half of the operator).
hipError_t sense_forward_rows(const SenseDev& S, const float2* img, float2* buf, hipStream_t s);
// One iteration, stage 0 (y pass: residual, data-loss partials, dl/dX back to
// the z-transformed domain) then stage 1 (z pass: gradient, TV, optimiser
// step; with `fwd` also the next iteration's forward rows).
constexpr int kSenseStages = 2;
hipError_t sense_stage(int stage, const SenseDev& S, const SenseOpt& O, const float2* img_in,
                       float2* img_out, float2* m, float2* v, float2* buf, float* partial,
                       const int* stop, int fwd, hipStream_t s);
int64_t sense_partials(const SenseDev& S);   // loss partials written per iteration
hipError_t sense_forward_op(const SenseDev& S, const float2* img, float2* buf, float2* out,
                            hipStream_t s);
hipError_t sense_adjoint_op(const SenseDev& S, const float2* r, float2* buf, float2* out,
                            hipStream_t s);

}  // namespace gc
