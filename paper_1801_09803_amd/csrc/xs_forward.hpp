// Launch interface of the forward cross-section kernels (tile kernels and the
// double-precision Voigt core pre-pass of the FP32 path).
#pragma once

#include "xs_internal.hpp"

namespace xs {

enum ProfileKind {
    kDoppler = 0, kGaussFixed = 1, kLorentz = 2, kVoigt = 3, kGHSampled = 4, kGHBinned = 5,
    kVVoigt = 6,          // Vectorized Voigt (the area-normalised form differs only in its intensities)
    kDopplerBinned = 7,   // bin-averaged Doppler Gaussian (difference of error functions)
    kLorentzBinned = 8,   // bin-averaged Lorentzian (difference of arctangents)
    kSuperLines = 9       // per-bin intensity sums (no profile)
};

// Line intensity of sorted line g at a (T, P) point from the stored T-independent factor
// cA = g_up A / (8 pi c nu^2), the lower-state energy and nu:
//   absorption (Eq. 1, cm/molecule): cA exp(-c2 E_low/T) (1 - exp(-c2 nu/T)) / Q;
//   emission (the emissivity, erg/s/sr/molecule): h c g_up A nu exp(-c2 E_up/T) / (4 pi Q),
//   which is 2 h c^2 nu^3 cA exp(-c2 E_up/T) / Q with E_up = E_low + nu.
// With non-LTE populations (Sec. "Treating non-local thermodynamic equilibrium") the
// Boltzmann factors become F = exp(-c2 E_vib/T_vib) exp(-c2 E_rot/T_rot): absorption
// cA (F_low - F_up)/Q, formed as F_low (1 - F_up/F_low) through expm1 of
// ln F_low - ln F_up = c2 [dE_vib/T_vib + dE_rot/T_rot] (negative when inverted), and
// emission 2 h c^2 nu^3 cA F_up/Q; Q is then Q(T_vib, T_rot).
__device__ __forceinline__ double line_intensity(const SortedLines& L, int g, double elow, double nu,
                                                 const TPParam& tp, double Q) {
    const double cA = L.cA[g];
    constexpr double k2hc2 = 2.0 * kH_CGS * kC_CGS * kC_CGS;
    if (L.evl) {
        const double evl = L.evl[g], evu = L.evu[g];
        const double dev = evu - evl;
        const double ln_fl = -(kC2 * evl) / tp.Tv - (kC2 * (elow - evl)) / tp.T;
        const double d = (kC2 * dev) / tp.Tv + (kC2 * (nu - dev)) / tp.T;
        if (tp.emission) return cA * (k2hc2 * (nu * nu * nu)) * exp(ln_fl - d) / Q;
        return cA * exp(ln_fl) * (-expm1(-d)) / Q;
    }
    if (tp.emission) return cA * (k2hc2 * (nu * nu * nu)) * exp(-(kC2 * (elow + nu)) / tp.T) / Q;
    return cA * exp(-(kC2 * elow) / tp.T) * (-expm1(-(kC2 * nu) / tp.T)) / Q;
}

struct FwdArgs {
    SortedLines L;
    Geometry G;
    const TPParam* tps;     // device array: the launch's block of (T, P) points
    const double* Q;        // device Q(T) array, indexed by TPParam::iq
    const int* off;         // offsets table, nkeys + 1 entries
    void* sigma;            // output of the first (T, P) of the block: float* (FP32) or double*
    void* part;             // n_split > 1: per-part sums, [n_tp][n_split][n_points] float2
                            // (FP32: sum, compensation) or double (FP64)
    int n_lines;            // kept (sorted) lines
    int n_tiles;
    int n_tp;               // (T, P) points in this launch (sigma has n_tp rows of n_points)
    int n_split;            // workgroups sharing one tile: workgroup q of a tile takes the LDS
                            // batches q, q + n_split, ... of its sorted lines (1: write sigma)
    int seg;                // FP32 path: per-wavefront line segments (needs 64P + rm < hmin)
    int xcd_contiguous;     // map consecutive tiles to one XCD (when no order is given)
    const int* tile_order;  // tiles by decreasing line count (heaviest dispatched first), or NULL
    double alpha_fixed;     // HWHM for the fixed Gaussian
    const Tables* tab;      // device quadrature tables
    // FP32 path: line records of record_kernel, one row of rec_stride lines per (T, P) of
    // the launch (8 floats hot, 16 words cold, 1 double scale per line)
    const float* hot;
    const int* cold;
    const double* xscale;
    // super-lines: per-line intensities of each (T, P) of the launch (rows of line_S_stride)
    double* line_S;
    int64_t line_S_stride;
    int64_t rec_stride;
    const float* core_val;          // FP32 Voigt: a * Re w at the lines' core points
    // FP64 Vectorized Voigt: per (line, T, P) {beta, intensity factor} rows of vv_stride
    // lines per (T, P) of the launch, or NULL (beta = 1, factor 1)
    const double2* vv;
    int64_t vv_stride;
    // intensity threshold: per (T, P) of the launch, the kept lines' sorted indices in
    // order (map, rows of map_stride) and their offsets table (offs, rows of offs_stride);
    // NULL: every sorted line, the plan's offsets table
    const int* map;
    int64_t map_stride;
    const int* offs;
    int64_t offs_stride;
    // FP32 Voigt segmented sweep: node-sampled far-wing sums, FP64 [n_tp][far_slots][n_points]:
    // slot 0 the interpolated node sums of far_kernel, slot 1 (with far_ends) ends_kernel's;
    // added by launch_combine.  NULL: the tile kernel sums every line
    double* far;
    // far_kernel's node totals per share, FP64 [n_tp][waves of the launch][16][far_share]
    double* far_nodes;
    int far_share;          // far_kernel wavefronts per tile wavefront
    int far_slots;
    // with far: the window-end runs (windows ending or starting inside a wavefront) are
    // node-sampled by ends_kernel (every such line lies beyond the far reach and the |z| < 40
    // radius of the wavefront); the tile kernel then sweeps only the lines centred near its tile
    int far_ends;
};

// Sorted line index of the launch's line g (through the threshold map when there is one).
__device__ __forceinline__ int line_of(const int* map, int g) { return map ? map[g] : g; }

// Per-(line, T, P) records of the FP32 path (record_kernel).
struct RecArgs {
    SortedLines L;
    Geometry G;
    const TPParam* tp;              // device: this (T, P)
    const double* Q;
    int n_lines;
    const Tables* tab;
    double alpha_fixed;
    const int* core_rc;             // Voigt: core radius per line (-1: none)
    const long long* core_off;      // Voigt: index in core_val of the line's first core value
    const double2* vv;              // Vectorized Voigt: {beta, intensity factor} per line, or NULL
    const int* map;                 // intensity threshold: kept lines' sorted indices, or NULL
    const unsigned long long* count;   // number of kept lines (device), with map
    float* hot;                     // [n_lines][8] ([n_lines][12] for the Vectorized Voigt), in
                                    // the order of map when there is one
    int* cold;                      // words 0-7 of the cold records, [n_lines][8]
    int* cold_b;                    // words 8-15, [n_lines][8] (not written for Voigt: the
                                    // kernels rebuild its 4-node coefficients from the hot record)
    double* xscale;                 // [n_lines]
};

// Vectorized Voigt pre-pass: per sorted line and (T, P), the continuity factor beta
// (1 unless requested) and the intensity factor (1, or for the area-normalised form
// 1 / (dnu x the sum of the line's profile values over its whole cut-off window)).
struct VVArgs {
    SortedLines L;
    Geometry G;
    const TPParam* tp;              // device: this (T, P)
    const Tables* tab;
    int n_lines;
    int use_beta;
    int normalise;
    int fp64;                       // sum the profile as the FP64 path evaluates it
    double2* out;                   // [n_lines]
};

hipError_t launch_vv_prep(const VVArgs& a, hipStream_t s);

// Intensity threshold (Sec. "Intensity thresholds") of one (T, P): lines with I >= I_cut(nu)
// are kept, compacted in sorted order (map), with their own offsets table (offs).
struct CullArgs {
    SortedLines L;
    Geometry G;
    const TPParam* tp;               // device: this (T, P)
    const double* Q;
    int n_lines;
    int mode;                        // 1 constant, 2 HITRAN's dynamic cut-off
    double i_crit, nu_crit;
    unsigned long long* bsum;        // [ceil(n_lines/256)] block counts, then exclusive prefix
    unsigned long long* scan_tmp;    // >= 4096 + 16 entries; scan_tmp[4096] = kept lines
    unsigned* pos;                   // [n_lines + 1] kept lines before each sorted line
    int* map;                        // [n_lines] compacted -> sorted index
    const int* off;                  // the plan's offsets table [nkeys + 1]
    int* offs;                       // this (T, P)'s offsets table [nkeys + 1]
};

hipError_t launch_cull(const CullArgs& a, hipStream_t s);
// exclusive scan of nb block totals in place; scan_tmp[4096] receives the total
hipError_t launch_scan64(unsigned long long* bsum, int64_t nb, unsigned long long* scan_tmp, hipStream_t s);

hipError_t launch_records(int profile, const RecArgs& a, hipStream_t s);

// Work item of one workgroup: tiles in dispatch order, each tile's n_tp * n_split
// workgroups consecutive (the same lines are read back to back from the caches).
struct WorkItem {
    int tile, tp, part;
};

// Points per block tile: 64-point slices per wavefront x wavefronts per block
// (the FP64 kernel always uses 4 wavefronts).
inline int tile_points(int slices_per_wave, int waves) { return 64 * waves * slices_per_wave; }

hipError_t launch_forward(int profile, int fp64, int waves, int slices_per_wave, const FwdArgs& a,
                          hipStream_t s);
// FP32 Voigt segmented sweep (a.far set): the node-sampled far wing of the lines the tile
// kernel leaves out, into a.far; launch after launch_forward, before launch_combine.
hipError_t launch_far(int waves, int P, const FwdArgs& a, hipStream_t s);
// Super-line histograms: sigma[t][k] = (sum of the intensities of the lines with kc == k) / dnu
// for the launch's (T, P) block (one thread per grid point; lines of a bin in sorted order).
hipError_t launch_superlines(int fp64, const FwdArgs& a, hipStream_t s);
// n_split > 1: sigma[t][k] = compensated sum over parts of part[t][*][k]; with far sums,
// sigma[t][k] (the parts' sum, or the tile kernel's value when n_split = 1) plus the sum over
// shares of far[t][*][k].  Nothing to do otherwise.
hipError_t launch_combine(int fp64, const FwdArgs& a, hipStream_t s);

// Streaming accumulators: acc holds n (sum, compensation) pairs, float2 (FP32) or
// double2 (FP64); add TwoSums x[i] into acc[i]; finish writes sum + compensation.
hipError_t launch_acc_zero(int fp64, void* acc, int64_t n, hipStream_t s);
hipError_t launch_acc_add(int fp64, const void* x, void* acc, int64_t n, hipStream_t s);
hipError_t launch_acc_finish(int fp64, const void* acc, void* out, int64_t n, hipStream_t s);

// Core pre-pass (FP32 Voigt): radius/count per line, per-256-line block totals.
struct CoreArgs {
    SortedLines L;
    Geometry G;
    const TPParam* tp;               // device: this (T, P)
    const double* Q;
    int n_lines;
    const Tables* tab;
    int* rc;                         // [n_lines]
    int* cnt;                        // [n_lines]
    unsigned long long* bsum;        // [ceil(n_lines/256)] block totals, then exclusive prefix
    long long* coff;                 // [n_lines] (absolute indices into val)
    float* val;                      // values of every (T, P) of the block
    long long val_base;              // first index of this (T, P) in val
    long long val_end;               // end of this (T, P)'s capacity in val (no write at or beyond)
    unsigned long long* scan_tmp;    // scratch for the block-total scan (>= 4096 + 16 entries);
                                     // scan_tmp[4096] receives the total count
    const double2* vv;               // Vectorized Voigt intensity factors (.y), or NULL
    const unsigned* kept_pos;        // intensity threshold: compacted positions [n_lines + 1] (line g
                                     // is kept iff kept_pos[g + 1] > kept_pos[g]), or NULL
};

hipError_t launch_core_count(const CoreArgs& a, hipStream_t s);
hipError_t launch_core_eval(const CoreArgs& a, hipStream_t s);
int64_t core_blocks(int64_t n_lines);
// Upper bound of the total core point count at temperature parameters tp, valid for
// any Lorentz widths and any temperature not above tp.T; the total goes to scan_tmp[4096].
hipError_t launch_core_bound(const CoreArgs& a, hipStream_t s);

}  // namespace xs
