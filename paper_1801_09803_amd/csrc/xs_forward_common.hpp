// Device helpers shared by the forward, core and adjoint kernels.
#pragma once

#include "xs_forward.hpp"
#include "xs_voigt.hpp"

namespace xs {

__device__ __forceinline__ int off_at(const int* off, int64_t kc, const Geometry& G) {
    int64_t k = kc + G.hmax;
    k = k < 0 ? 0 : (k > G.nkeys ? G.nkeys : k);
    return off[k];
}

// Tile index for a block.  With an order table the heaviest tiles are dispatched
// first (longest-processing-time first), which balances the CUs when line density
// varies along the grid; the lightest tiles fill the tail.
__device__ __forceinline__ int tile_of_block(int bid, int n, int xcd_contiguous, const int* order) {
    if (order) return order[bid];
    if (!xcd_contiguous) return bid;
    // consecutive tiles on the same XCD (blocks reach the 8 XCDs round-robin)
    const int x = bid & 7, q = n >> 3, r = n & 7;
    return x * q + (x < r ? x : r) + (bid >> 3);
}

// Work item of workgroup blockIdx.x (uniform: scalar registers).
__device__ __forceinline__ WorkItem work_item(const FwdArgs& A) {
    const int per = A.n_tp * A.n_split;
    const int rank = (int)blockIdx.x / per;
    const int rem = (int)blockIdx.x - rank * per;
    WorkItem w;
    w.tile = tile_of_block(rank, A.n_tiles, A.xcd_contiguous, A.tile_order);
    w.tp = rem / A.n_split;
    w.part = rem - w.tp * A.n_split;
    return w;
}

// Per-line, per-(T,P) double-precision setup.
struct LineSetup {
    double nu, S, aD, gam;
    int kc, klo, khi;
};

__device__ __forceinline__ LineSetup line_setup(const SortedLines& L, const TPParam& tp, int g, double Q) {
    LineSetup o;
    o.nu = L.nu[g];
    const double el = L.elow[g];
    o.S = line_intensity(L, g, el, o.nu, tp, Q);   // Eq. 1, or the emissivity for emission
    o.aD = o.nu * tp.beta;                                                        // Eq. 16
    o.gam = (double)L.gref[g] * exp((double)L.nexp[g] * tp.ln_T0_T) * tp.p_over_p0;  // Eq. 18
    o.kc = L.kc[g];
    o.klo = L.klo[g];
    o.khi = L.khi[g];
    return o;
}

// Smallest |nu_k - nu| over grid points kA..kB (0 if the centre lies inside).
__device__ __forceinline__ double min_abs_delta(const Geometry& G, int kA, int kB, double nu) {
    const double dA = (G.nu_a + (double)kA * G.dnu) - nu;
    const double dB = (G.nu_a + (double)kB * G.dnu) - nu;
    if (dA <= 0.0 && dB >= 0.0) return 0.0;
    return fmin(fabs(dA), fabs(dB));
}

// Conservative radius (grid steps from kc) of the points with |x| < X, where
// x_j = j h + xc (h = s dnu, xc = s d): |j| <= floor((X + |xc|)/h) + 1.  -1 if X <= 0.
__device__ __forceinline__ int radius_steps(double X, double h, double xc) {
    if (!(X > 0.0)) return -1;
    const double r = floor((X + fabs(xc)) / h) + 1.0;
    return r > 1.0e9 ? 1000000000 : (int)r;
}

// erf(b) - erf(a) for a <= b without cancellation in the tails: a difference of
// complementary error functions of same-signed arguments there.
__device__ __forceinline__ double erf_diff64(double a, double b) {
    if (a >= 0.0) return erfc(a) - erfc(b);
    if (b <= 0.0) return erfc(-b) - erfc(-a);
    return erf(b) - erf(a);
}

// Core radius of the FP32 Voigt path: points with |z| < 8 are evaluated by the
// double-precision core pre-pass.
constexpr double kCoreR2 = 64.0;
constexpr double kMidR2 = 1600.0;
// Far-wing radius of the FP32 Voigt path: wing-only runs whose points all lie at
// |x| >= kFarX use the one-pole form (relative error <= 1/kFarX^2 = 1e-6).
constexpr double kFarX = 1000.0;

}  // namespace xs
