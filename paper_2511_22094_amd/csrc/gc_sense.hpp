// Image reconstruction (gc_sense.hip): descriptors and launchers.
#pragma once
#include "gc_internal.hpp"

namespace gc {

constexpr int kSenseCols = 16;        // most columns per block of the y-direction pass
constexpr int kSenseColElems = 4096;  // y-pass tile: Ny x G complex values (32 KiB of LDS)
constexpr int kSenseMaxN = 1024;      // largest transform length along y or z
struct SenseDev {
    int E, Nc, Ny, Nz, logNy, logNz;
    int G;                            // columns per y-pass block, min(16, 4096 / Ny)
    float rsqrtNy, rsqrtNz;           // unitary scaling of each 1D transform
    const float2* coils;              // [Nc][Ny][Nz]
    const float2* ksp;                // [E][Nc][Ny][Nz]
    const uint8_t* mask;              // [E][Ny][Nz]
    const float2* twy;                // [Ny/2] exp(-2 pi i k / Ny)
    const float2* twz;                // [Nz/2]
    float scale_data;                 // 1 / Nk
    int loss_p;
};
struct SenseOpt {
    int optimizer;
    float lr, beta1, beta2, eps, momentum, rho, omb1, omb2, omrho;
    float c1, c2;                     // bias corrections of this iteration
    float scale_tv;                   // lambda / Npix
};
// One iteration is kSenseStages launches, stage 0..3 in order (the loss
// partials of stage 1 and 3 land in disjoint parts of `partial`).
constexpr int kSenseStages = 4;
hipError_t sense_stage(int stage, const SenseDev& S, const SenseOpt& O, const float2* img_in,
                       float2* img_out, float2* m, float2* v, float2* buf, float* partial,
                       const int* stop, hipStream_t s);
int64_t sense_partials(const SenseDev& S);   // loss partials written per iteration
hipError_t sense_forward_op(const SenseDev& S, const float2* img, float2* out, hipStream_t s);
hipError_t sense_adjoint_op(const SenseDev& S, float2* buf, float2* out, hipStream_t s);

}  // namespace gc
