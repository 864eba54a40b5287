// Launch interface of the forward cross-section kernels (tile kernels and the
// double-precision Voigt core pre-pass of the FP32 path).
#pragma once

#include "xs_internal.hpp"

namespace xs {

enum ProfileKind { kDoppler = 0, kGaussFixed = 1, kLorentz = 2, kVoigt = 3, kGHSampled = 4, kGHBinned = 5 };

struct FwdArgs {
    SortedLines L;
    Geometry G;
    TPParam tp;
    const double* Q;        // device Q(T) array, indexed by tp.iq
    const int* off;         // offsets table, nkeys + 1 entries
    void* sigma;            // float* (FP32 path) or double* (FP64 path), n_points values
    int n_lines;            // kept (sorted) lines
    int n_tiles;
    int seg;                // FP32 path: per-wavefront line segments (needs 64P + rm < hmin)
    int xcd_contiguous;     // map consecutive tiles to one XCD (when no order is given)
    const int* tile_order;  // tiles by decreasing line count (heaviest dispatched first), or NULL
    double alpha_fixed;     // HWHM for the fixed Gaussian
    const Tables* tab;      // device quadrature tables
    // FP32 Voigt core pre-pass results (per sorted line)
    const int* core_rc;             // core radius in grid steps (-1: none)
    const long long* core_off;      // first value of the line in core_val
    const float* core_val;          // a * Re w at the line's core points
};

// Points per block tile: 64-point slices per wavefront x wavefronts per block
// (the FP64 kernel always uses 4 wavefronts).
inline int tile_points(int slices_per_wave, int waves) { return 64 * waves * slices_per_wave; }

hipError_t launch_forward(int profile, int fp64, int waves, int slices_per_wave, const FwdArgs& a,
                          hipStream_t s);

// Core pre-pass (FP32 Voigt): radius/count per line, per-256-line block totals.
struct CoreArgs {
    SortedLines L;
    Geometry G;
    TPParam tp;
    const double* Q;
    int n_lines;
    const Tables* tab;
    int* rc;                         // [n_lines]
    int* cnt;                        // [n_lines]
    unsigned long long* bsum;        // [ceil(n_lines/256)] block totals, then exclusive prefix
    long long* coff;                 // [n_lines]
    float* val;                      // [total]
    unsigned long long* scan_tmp;    // scratch for the block-total scan (>= 4096 + 16 entries)
};

hipError_t launch_core_count(const CoreArgs& a, hipStream_t s);
hipError_t launch_core_eval(const CoreArgs& a, hipStream_t s);
int64_t core_blocks(int64_t n_lines);

}  // namespace xs
