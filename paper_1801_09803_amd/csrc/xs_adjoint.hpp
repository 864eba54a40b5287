// Launch interface of the Voigt adjoint kernel.
#pragma once

#include "xs_internal.hpp"

namespace xs {

struct AdjArgs {
    SortedLines L;
    Geometry G;
    TPParam tp;
    double P0;
    const double* Q;       // device Q(T) (one temperature)
    const double* dQ;      // device dQ/dT
    const void* gbar;      // dL/dsigma on the grid: float (FP32 path) or double
    int n_lines;           // kept (sorted) lines
    const Tables* tab;
    void* dlnA;            // [caller lines] float (FP32 path) or double, or NULL
    void* dgref;
    void* dn;
    double* pT;            // [n_lines] per-line dL/dT terms
    double* pP;            // [n_lines] per-line dL/dP terms
    float* rec;            // FP32 path: [n_lines][kAdjRec] per-line wing records
    double* sums;          // FP32 path: [n_lines][6] core and wing window sums
};

constexpr int kAdjRec = 24;

// part: >= 512 doubles of scratch
hipError_t launch_adjoint(const AdjArgs& a, int fp64, int64_t n_caller_lines, double* part, double* dT,
                          double* dP, hipStream_t s);

}  // namespace xs
