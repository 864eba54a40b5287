// Geometry of the node-sampled Voigt far wing of the FP32 segmented sweep, shared by the
// tile kernel (which leaves those lines out) and the far-wing kernels (which sample them).
#pragma once

#include "xs_forward_common.hpp"

namespace xs {

// Node-sampled Voigt far wing (segmented sweep): lines whose centre lies at least R grid
// steps from every point of a wavefront of WW points, R = max(far_reach(WW), the |z| < 8
// radius), add their wing values (the 2-node rule, or the 4-node rule inside the |z| < 40
// radius) at kFarN nodes across it (far_kernel), interpolated to its points; the tile
// kernel leaves them out.  Such a wing is a smooth rational function of the position with
// its poles near the line centre.  The nodes are the Chebyshev points of the first kind on
// [0, WW - 1] and the interpolant is the degree-15 polynomial through all of them
// (barycentric form); with the nearest centre 0.57 (WW - 1) from the wavefront its error
// stays below 2e-8 relative.
constexpr int kFarN = 16;
constexpr int far_reach(int ww) { return (57 * (ww - 1) + 99) / 100; }

// Grid steps from w0 to node m of a wavefront of WW points, (WW - 1)(1 - cos(pi (2m + 1)/32))/2,
// rounded to float (the position the node values are computed at).
template <int WW>
__device__ __forceinline__ float node_pos(int m) {
    constexpr double u[kFarN] = {
        0.0024076366639015356, 0.021529832133895588, 0.059039367825822475, 0.1134947733186315,
        0.18280335791817726,   0.2643016315870011,   0.35485766137276886,  0.45099142983521961,
        0.54900857016478033,   0.64514233862723103,  0.73569836841299885,  0.81719664208182263,
        0.88650522668136844,   0.94096063217417747,  0.97847016786610441,  0.99759236333609835};
    return (float)((double)(WW - 1) * u[m]);
}

// Weights at point o (0 .. WW-1) of the polynomial through the node values: the barycentric
// form sum_m (c_m / (o - p_m)) f_m / sum_m (c_m / (o - p_m)) with c_m = 1 / prod_{k != m}
// (p_m - p_k) for the node positions p_m as rounded (a node hit exactly takes its value).
template <int WW>
__device__ __forceinline__ void far_weights(int o, double (&w)[kFarN]) {
    double c[kFarN];
#pragma unroll
    for (int m = 0; m < kFarN; ++m) {
        double pr = 1.0;
#pragma unroll
        for (int k = 0; k < kFarN; ++k)
            if (k != m) pr *= (double)node_pos<WW>(m) - (double)node_pos<WW>(k);
        c[m] = 1.0 / pr;
    }
    double den = 0.0;
    int hit = -1;
#pragma unroll
    for (int m = 0; m < kFarN; ++m) {
        const double d = (double)o - (double)node_pos<WW>(m);
        if (d == 0.0) hit = m;
        w[m] = c[m] / (d == 0.0 ? 1.0 : d);
        den += w[m];
    }
    const double inv = 1.0 / den;
#pragma unroll
    for (int m = 0; m < kFarN; ++m) w[m] = hit < 0 ? w[m] * inv : (m == hit ? 1.0 : 0.0);
}

// Radius (grid steps) of the |z| < 40 zone of the lines whose centre can lie near the
// wavefront [w0, w1]: their wavenumbers, hence Doppler widths, are bounded there.
__device__ __forceinline__ int wave_rm(const TPParam& tp, const Geometry& G, int w0, int w1) {
    int rm = tp.rm;
    if (tp.rm_scale > 0.0) {
        const double nlo = G.nu_a + ((double)w0 - rm - 1) * G.dnu;
        const double nhi = G.nu_a + ((double)w1 + rm + 1) * G.dnu;
        const double rw = ceil(tp.rm_scale * fmax(fabs(nlo), fabs(nhi))) + 2.0;
        if (rw < (double)rm) rm = __builtin_amdgcn_readfirstlane((int)rw);
    }
    return rm;
}

// Node-sampling radius of the wavefront [w0, w1]: the far reach, or the |z| < 8 radius of
// the lines centred within max(reach, rm) of it where that is larger (every point of a
// node-sampled line must lie outside its core).  At most tp.rm.
__device__ __forceinline__ int wave_far_r(const TPParam& tp, const Geometry& G, int w0, int w1, int reach) {
    int r8 = tp.rm;
    if (tp.rm_scale > 0.0) {
        const double span = (double)(reach > tp.rm ? reach : tp.rm) + 1.0;
        const double nlo = G.nu_a + ((double)w0 - span) * G.dnu;
        const double nhi = G.nu_a + ((double)w1 + span) * G.dnu;
        const double rw = ceil(0.2 * tp.rm_scale * fmax(fabs(nlo), fabs(nhi))) + 2.0;
        if (rw < (double)r8) r8 = (int)rw;
    }
    return __builtin_amdgcn_readfirstlane(r8 > reach ? r8 : reach);
}

// The lines whose window covers the wavefront [w0, w1] are [s1, s4) (w1 - hmin <= kc <=
// w0 + hmin); of them, [s1, hcl) (kc < w0 - R) and [hcr, s4) (kc > w1 + R) are
// node-sampled, R from wave_far_r, and of those [ml, hcl) and [hcr, mr) lie inside the
// |z| < 40 radius rm (the 4-node rule).
struct FarRange {
    int s1, hcl, hcr, s4, ml, mr;
};

__device__ __forceinline__ FarRange far_range(const int* off, const Geometry& G, int w0, int w1, int rm, int R) {
    const int64_t l0 = (int64_t)w1 - G.hmin, r1 = (int64_t)w0 + G.hmin + 1;
    const int64_t hl = (int64_t)w0 - R > l0 ? (int64_t)w0 - R : l0;
    const int64_t hr = (int64_t)w1 + R + 1 < r1 ? (int64_t)w1 + R + 1 : r1;
    int64_t ml = (int64_t)w0 - rm, mr = (int64_t)w1 + rm + 1;
    ml = ml < l0 ? l0 : (ml > hl ? hl : ml);
    mr = mr > r1 ? r1 : (mr < hr ? hr : mr);
    FarRange f;
    f.s1 = off_at(off, l0, G);
    f.s4 = off_at(off, r1, G);
    f.hcl = off_at(off, hl, G);
    f.hcr = off_at(off, hr, G);
    f.ml = off_at(off, ml, G);
    f.mr = off_at(off, mr, G);
    return f;
}

}  // namespace xs
