// Host-side choice of the kernel instantiation for a model and acquisition
// (register-resident measurement counts, straight-line forms).  Kept apart
// from the kernels so the host-only build of the scheduler uses the same
// rules.
#include "gc_internal.hpp"

namespace gc {

// Register-resident data sizes instantiated per model (measurement counts);
// anything else runs the HBM-read variant (MAXM = 0).
int mh_pick_maxm(int kind, int M) {
    static const int mono[] = {12, 16, 32};
    static const int gre[] = {12, 24, 32};
    if (kind == DWI2) return 0;
    const int* list = kind == GRE3 ? gre : mono;
    if (kind == LINEAR3) return M <= 12 ? 12 : (M <= 16 ? 16 : 0);
    for (int i = 0; i < 3; ++i)
        if (M <= list[i]) return list[i];
    return 0;
}

// The exact, straight-line instantiation is used when the acquisition has
// exactly MAXM measurements and -- for the exponential-decay models -- equally
// spaced echoes (the recurrence then applies unconditionally).
int mh_pick_variant(int kind, int M, int uniform) {
    // dwi2 reads its data from memory: with up to 96 measurements per lane in
    // registers (and the straight-line form's hoisted acquisition values) the
    // kernel runs at one or two waves per SIMD, which measured 1.2x (register
    // loop) to 5.8x (straight line) slower than the memory-read loop
    if (kind == DWI2) return 0;
    const int maxm = mh_pick_maxm(kind, M);
    const bool rec_model = kind == MONOEXP_T2S || kind == MONOEXP_R2S || kind == GRE3;
    const bool exact = maxm == M && (!rec_model || uniform);
    return maxm | (exact ? 1 << 16 : 0);
}

// Fits: register-resident measurement counts of the fused kernel.
int fit_pick_maxm(int kind, int M) {
    if (kind == GRE3) return M <= 12 ? 12 : (M <= 24 ? 24 : (M <= 32 ? 32 : 0));
    // dwi2: the shell-by-shell loop over data read per use measured 15 %
    // faster than 96 measurements held in registers (two waves per SIMD)
    if (kind == DWI2) return 0;
    return M <= 12 ? 12 : (M <= 16 ? 16 : (M <= 32 ? 32 : 0));
}

}  // namespace gc
