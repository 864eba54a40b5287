// Launch interfaces of the state reductions: partition-function moments and the specific
// heat, per-state sums over the transitions (radiative lifetimes), and the cooling function.
#pragma once

#include "xs_internal.hpp"

namespace xs {

// One pass over the transitions in the caller's order.  Per transition: the state
// indices are checked (kFlagIndex) and, when nu is needed, nu = E_up - E_low > 0
// (kFlagNu); then, per upper state, sum_A += A and power += A nu (FP64 atomics, each
// output optional).  Invalid transitions contribute nothing.
struct RateArgs {
    int64_t n;
    const int* upper;
    const int* lower;       // needed only for power
    const float* A;
    int index_base;
    int a_is_log;           // A holds ln A
    const double* E;
    int64_t n_states;
    int* flag;
    double* sum_A;          // [n_states] or NULL
    double* power;          // [n_states] or NULL
};

hipError_t launch_fill(double* x, int64_t n, double v, hipStream_t s);
hipError_t launch_rates(const RateArgs& a, hipStream_t s);

// The same per-state sums without global atomics: the transitions are counted and
// scattered into buckets of 2^kBucketBits consecutive upper states (a counting sort by
// bucket: per-4096-transition-block histograms, one exclusive scan, a scatter of 16-B
// records), then one workgroup per bucket adds its records into LDS and writes the
// bucket's sums.  Applies while the histogram has at most kMaxBucketHist entries
// (bucket_rates_fits); otherwise launch_rates is the path.  Workspace: hist and hoff of
// bucket_hist_len entries, tsum of 4096 entries, rec of 16 n bytes.
constexpr int kBucketBits = 12;
constexpr int64_t kMaxBucketHist = (int64_t)4096 * 4096;
bool bucket_rates_fits(int64_t n, int64_t n_states);
int64_t bucket_hist_len(int64_t n, int64_t n_states);
hipError_t launch_bucket_rates(const RateArgs& a, uint32_t* hist, uint32_t* hoff, uint32_t* tsum, void* rec,
                               hipStream_t s);
// tau_i = 1 / sum_A_i, +inf where no transition leaves state i
hipError_t launch_lifetimes(const double* sum_A, int64_t n, double* tau, hipStream_t s);
// Q, Q' = sum g x e^-x, Q'' = sum g x^2 e^-x (x = c2 E/T) and C_p per temperature; part:
// 3 nT nb doubles; every output optional.
hipError_t launch_moments(const double* E, const int* g, int64_t n, const double* T_dev, int nT, double* part,
                          int nb, double* Q, double* Q1, double* Q2, double* Cp, hipStream_t s);
// W(T) = h c sum_i g_i power_i exp(-c2 E_i/T) / (4 pi Q(T)); part: 2 nT nb doubles.
hipError_t launch_cooling(const double* E, const int* g, const double* power, int64_t n, const double* T_dev,
                          int nT, double* part, int nb, double* W, hipStream_t s);

// Non-LTE (Sec. "Treating non-local thermodynamic equilibrium"): E_vib of each state is
// the lowest energy among the states with its manifold label (labels in [0, n_labels),
// energies >= 0; otherwise kFlagIndex / kFlagNu and E_vib = 0).  vmin: n_labels words.
hipError_t launch_vib_energies(const double* E, const int* labels, int64_t n, int n_labels,
                               unsigned long long* vmin, double* Ev, int* flag, hipStream_t s);
// Per kept sorted line p < n: evl[p] / evu[p] = E_vib of its lower / upper state, through
// the caller's index arrays (n_lines entries) at orig[p] (0 for an index out of range).
hipError_t launch_vib_gather(int64_t n, const int* orig, int64_t n_lines, const int* upper, const int* lower,
                             int index_base, const double* Ev, int64_t n_states, double* evl, double* evu,
                             hipStream_t s);

}  // namespace xs
