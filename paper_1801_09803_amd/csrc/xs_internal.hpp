// Internal definitions shared by the HIP kernels and the host plan code of libxsec.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>
#include <string>

#include "../../include/xsec.h"

namespace xs {

// Physical constants: the 2019 SI exact values of h, c, k_B and the CODATA 2018
// atomic mass constant.  c2 = h c / k_B is the second radiation constant of Eq. 1/2.
constexpr double kH = 6.62607015e-34;        // J s
constexpr double kC_SI = 299792458.0;        // m / s
constexpr double kKB = 1.380649e-23;         // J / K
constexpr double kAMU = 1.66053906660e-27;   // kg
constexpr double kC_CGS = kC_SI * 100.0;     // cm / s
constexpr double kC2 = kH * kC_SI / kKB * 100.0;   // cm K
constexpr double kH_CGS = kH * 1.0e7;        // erg s
constexpr double kPI = 3.14159265358979323846;
constexpr double kLN2 = 0.69314718055994530942;
constexpr double kSQRT_LN2 = 0.83255461115769775635;        // sqrt(ln 2)
constexpr double kSQRT_LN2_PI = 0.46971863934982566689;     // sqrt(ln 2 / pi)
constexpr double kINV_SQRT_PI = 0.56418958354775628695;     // 1 / sqrt(pi)

// Device error flags (bitwise OR-ed by the line-prep kernel).
constexpr int kFlagIndex = 1;
constexpr int kFlagNu = 2;
constexpr int kFlagKey = 4;

// Lines sorted by centre (structure of arrays, plan-owned device memory).
struct SortedLines {
    const double* nu;      // transition wavenumber E_up - E_low
    const double* elow;    // lower-state energy
    const double* cA;      // g_up A / (8 pi c nu^2)  (the T-independent part of Eq. 1)
    const float* gref;     // gamma_ref (cm^-1 / P0)
    const float* nexp;     // temperature exponent n
    const int* kc;         // nearest grid index to the centre (may lie off the grid)
    const int* klo;        // first grid index of the cut-off window (clipped)
    const int* khi;        // last grid index of the cut-off window (clipped)
    const int* orig;       // index of the line in the caller's arrays
    // non-LTE populations: vibrational energies of the lower and upper states (NULL in LTE)
    const double* evl;
    const double* evu;
};

// Grid and window geometry shared by every kernel of a plan.
struct Geometry {
    double nu_a, dnu, cutoff;
    int n_points;
    int hmax;    // upper bound of |window edge - kc| in grid steps (key offset)
    int hmin;    // lower bound of the same (lines with |kc - k| <= hmin cover k)
    int nkeys;   // number of sort keys for kept lines; key == nkeys marks a dropped line
    // Vectorized Voigt: radius R (cm^-1) of the region where the line's own Voigt profile
    // is used, and bounds of |k - kc| at the region's edges in grid steps (every point
    // with |k - kc| <= rvmin is inside, every point with |k - kc| > rvmax outside)
    double vv_radius;
    int rvmin, rvmax;
};

// Per (T, P) scalars computed on the host (everything but Q(T), which stays on the device).
struct TPParam {
    double T, P;
    double Tv;            // vibrational temperature of non-LTE populations (T_rot = T)
    double c2_over_T;     // used in Eq. 1 exponents as (c2 * E) / T
    double beta;          // alpha_D / nu  (Eq. 16)
    double ln_T0_T;       // ln(T0 / T), for (T0/T)^n in Eq. 18
    double p_over_p0;     // P / P0
    double rm_scale;      // radius per cm^-1 of line wavenumber (grid steps, Doppler-width
                          // profiles; 0 when the radius does not grow with the wavenumber)
    int iq;               // index of T in the plan's device Q array
    int rm;               // bound on the mid/core radius in grid steps (FP32 Voigt fast path)
    int emission;         // 1: line intensities are emissivities (upper-state population)
};

// Gauss-Hermite pairs used by the wing formulas (positive nodes only).
constexpr int kMaxGHPairs = 16;
struct GHPairs {
    int n_pairs;
    int has_zero;                 // odd rule: node at 0 with weight w0
    double w0;
    double t[kMaxGHPairs];
    double w[kMaxGHPairs];
};

// Weideman (1994) rational approximation coefficients a_1..a_N (real) and L.
constexpr int kMaxWeideman = 48;
struct WeidemanCoef {
    int n;
    double L;
    double a[kMaxWeideman];       // a[n-1] is the leading coefficient in Horner order
};

// Dawson's function D(x) on [0, kDawsonIv / 2): one polynomial of degree kDawsonNc - 1 per
// interval [i/2, (i+1)/2), in u = 4 (x - (i/2 + 1/4)) in [-1, 1], coefficients ascending;
// Chebyshev interpolation of a reference sum, absolute error below 2e-15 (relative 1e-13
// above x = 0.5, where D grows past 0.4)
constexpr int kDawsonIv = 17;
constexpr int kDawsonNc = 13;

// All quadrature tables of a plan, kept in one device buffer and read by the kernels
// through a uniform pointer (scalar loads).
constexpr int kGHConvDefault = 30;   // nodes of the Gauss-Hermite convolution profiles ("usually 30")
constexpr int kMaxGHConv = 64;       // largest rule a plan may ask for
constexpr int kMaxGHPair = kMaxGHConv / 2 + 1;
struct Tables {
    WeidemanCoef w24;   // FP32 path core
    WeidemanCoef w40;   // FP64 path core
    double dawson[kDawsonIv * kDawsonNc];   // FP32 path core: D(x) on the real axis
    GHPairs gh2, gh4, gh6, gh12;
    // Gauss-Hermite rule of the convolution profiles (Eq. 30-31): nconv nodes ascending,
    // and its npair node pairs +-t (the zero node of an odd rule as a pair of half weight)
    int nconv, npair;
    double tconv[kMaxGHConv], wconv[kMaxGHConv];
    float tconvf[kMaxGHConv], wconvf[kMaxGHConv];
    double tpair[kMaxGHPair], wpair[kMaxGHPair];
    float tpairf[kMaxGHPair], wpairf[kMaxGHPair];
};

// Host helpers implemented in xs_quadrature.cpp.
void gauss_hermite_rule(int n, double* nodes, double* weights);
void weideman_coefficients(int n, WeidemanCoef* out);
void dawson_table(double* out);
void make_gh_pairs(int n, GHPairs* out);

// Plan internals for entry points outside the plan's source file (xs_api.cpp):
// the thread-local error text of xs_last_error, and the plan's states on the device.
xs_status set_error(xs_status s, const std::string& msg);
bool plan_states(const xs_plan* p, const double** E, const int** g, int64_t* n_states);

}  // namespace xs
