// Launch interface of the forward cross-section tile kernels.
#pragma once

#include "xs_internal.hpp"

namespace xs {

enum ProfileKind { kDoppler = 0, kGaussFixed = 1, kLorentz = 2, kVoigt = 3 };

struct FwdArgs {
    SortedLines L;
    Geometry G;
    TPParam tp;
    const double* Q;        // device Q(T) array, indexed by tp.iq
    const int* off;         // offsets table, nkeys + 1 entries
    void* sigma;            // float* (FP32 path) or double* (FP64 path), n_points values
    int n_tiles;
    int fast_ok;            // FP32 path: far-only / skip-only line ranges may bypass the codes
    double alpha_fixed;     // HWHM for the fixed Gaussian
    const Tables* tab;      // device quadrature tables
};

// Points per block tile for a given number of 64-point slices per wavefront.
inline int tile_points(int slices_per_wave) { return 256 * slices_per_wave; }

hipError_t launch_forward(int profile, int fp64, int slices_per_wave, const FwdArgs& a, hipStream_t s);

}  // namespace xs
