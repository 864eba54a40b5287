// Launch interfaces of the partition-function and line-preparation kernels.
#pragma once

#include "xs_internal.hpp"

namespace xs {

// One prepared line in the caller's order (48 B, so the gather into sorted order reads
// one record per line instead of eight scattered arrays).
struct PrepRec {
    double nu;       // E_up - E_low
    double elow;     // lower-state energy
    double cA;       // g_up A / (8 pi c nu^2)
    float gref, nexp;
    int kc, klo, khi, pad;
};

struct PrepArgs {
    int64_t n;                 // transitions
    const int* upper;
    const int* lower;
    const float* A;
    const float* gref_line;    // per-line broadening (broad == 1)
    const float* nexp_line;
    const float* gref_tab;     // a0 table (broad == 2)
    const float* nexp_tab;
    int n_j;
    float gamma_const, n_const;  // broad == 0
    int broad;
    int index_base;
    int a_is_log;              // A holds ln A
    const double* E;
    const int* g;
    const int* J;
    int64_t n_states;
    Geometry geo;
    int* flag;
    // outputs, indexed by the caller's line index
    PrepRec* p_rec;
    uint32_t* keys;
    uint32_t* vals;
};

struct GatherArgs {
    int64_t n;
    int nkeys;
    const uint32_t* keys;
    const uint32_t* vals;
    const PrepRec* p_rec;
    double* nu;
    double* elow;
    double* cA;
    float* gref;
    float* nexp;
    int* kc;
    int* klo;
    int* khi;
    int* orig;
};

// Q(T) and dQ/dT per temperature; with Ev (vibrational energies, or NULL for LTE) the
// populations are non-LTE with vibrational temperatures Tv_dev[nT].
hipError_t launch_partition(const double* E, const int* g, const double* Ev, int64_t n, const double* T_dev,
                            const double* Tv_dev, int nT, double* part, int nb, double* Q, double* dQ,
                            hipStream_t s);
hipError_t launch_prep(const PrepArgs& a, hipStream_t s);
int64_t radix_hist_len(int64_t n);
int radix_passes(uint32_t max_key);
hipError_t launch_exclusive_scan(const uint32_t* x, int64_t m, uint32_t* y, uint32_t* tsum, hipStream_t s);
hipError_t launch_radix_sort(uint32_t* k1, uint32_t* v1, uint32_t* k2, uint32_t* v2, int64_t n,
                             uint32_t max_key, uint32_t* hist, uint32_t* hoff, uint32_t* tsum,
                             uint32_t** out_k, uint32_t** out_v, hipStream_t s);
hipError_t launch_gather(const GatherArgs& a, hipStream_t s);
hipError_t launch_offsets(const uint32_t* keys, int64_t n, int nkeys, int* off, hipStream_t s);

}  // namespace xs
