// Double-precision pre-pass of the FP32 Voigt path: every line's grid points with
// |z| < 8 (where the single-precision wing formulas lose accuracy) are evaluated once
// per (T, P), densely (one grid point per lane, points of consecutive lines packed
// together), and stored as f32 values a * Re w(z) for the tile kernel to add.
//
// core_count: per sorted line, the core radius r (grid steps from kc, conservative)
//   and the number of window points in [kc - r, kc + r]; per-256-line totals.  Under an
//   intensity threshold only kept lines count (the cull runs first).
// (exclusive scan of the totals)
// core_eval: per 256 lines, block-local offsets, then the block's points grouped by
//   evaluation path, each thread taking runs of 8 consecutive points (a binary search over
//   the group's block prefix for the first, a forward step for the rest).  Near the real axis (y < 0.2) each line takes only the
//   Taylor terms its y needs.
#include "xs_forward_common.hpp"
#include "xs_lineprep.hpp"

namespace xs {

namespace {

template <class T>
__device__ __forceinline__ T block_exclusive_scan_t(T v, T* lds4, T* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    T incl = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const T o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
    }
    __syncthreads();
    if (lane == 63) lds4[wave] = incl;
    __syncthreads();
    T wbase = 0;
    for (int w = 0; w < wave; ++w) wbase += lds4[w];
    *total = lds4[0] + lds4[1] + lds4[2] + lds4[3];
    return wbase + incl - v;
}

struct CoreLine {
    double s, nu, y, a;
    int lo, hi, r, kc;
};

__device__ __forceinline__ CoreLine core_line(const CoreArgs& A, const TPParam& tp, int g, double Q) {
    const LineSetup ls = line_setup(A.L, tp, g, Q);
    CoreLine c;
    c.s = kSQRT_LN2 / ls.aD;
    c.nu = ls.nu;
    c.y = ls.gam * c.s;
    c.a = ls.S * kSQRT_LN2_PI / ls.aD;
    c.r = -1;
    c.lo = 0;
    c.hi = -1;
    c.kc = ls.kc;
    const double y2 = c.y * c.y;
    if (y2 < kCoreR2) {
        const double d = (A.G.nu_a + (double)ls.kc * A.G.dnu) - ls.nu;
        c.r = radius_steps(sqrt(kCoreR2 - y2), c.s * A.G.dnu, c.s * d);
        const int64_t lo = (int64_t)ls.kc - c.r, hi = (int64_t)ls.kc + c.r;
        c.lo = (int)(lo > ls.klo ? lo : ls.klo);
        c.hi = (int)(hi < ls.khi ? hi : ls.khi);
    }
    return c;
}

__global__ __launch_bounds__(256) void core_count_kernel(const CoreArgs A) {
    __shared__ unsigned long long lds[4];
    const int g = blockIdx.x * 256 + threadIdx.x;
    const TPParam tp = *A.tp;
    unsigned long long c = 0;
    if (g < A.n_lines) {
        if (!A.kept_pos || A.kept_pos[g + 1] > A.kept_pos[g]) {
            const CoreLine cl = core_line(A, tp, g, A.Q[tp.iq]);
            c = cl.hi >= cl.lo ? (unsigned long long)(cl.hi - cl.lo + 1) : 0ull;
            A.rc[g] = cl.r;
        } else {
            A.rc[g] = -1;   // below the intensity threshold: no record reads its core values
        }
        A.cnt[g] = (int)c;
    }
    unsigned long long tot;
    block_exclusive_scan_t<unsigned long long>(c, lds, &tot);
    if (threadIdx.x == 0) A.bsum[blockIdx.x] = tot;
}

// exclusive scan of m u64 values in place (m <= 4096 * 4096); tmp[4096] gets the total
constexpr int kScanTile = 4096;

__global__ __launch_bounds__(256) void scan64_tiles_kernel(const unsigned long long* x, int64_t m,
                                                           unsigned long long* tsum) {
    __shared__ unsigned long long lds[4];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * 16;
    unsigned long long s = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) if (base + k < m) s += x[base + k];
    unsigned long long tot;
    block_exclusive_scan_t<unsigned long long>(s, lds, &tot);
    if (threadIdx.x == 0) tsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void scan64_small_kernel(unsigned long long* tsum, int64_t nt) {
    __shared__ unsigned long long lds[4];
    const int64_t base = (int64_t)threadIdx.x * 16;
    unsigned long long v[16], s = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) { v[k] = (base + k < nt) ? tsum[base + k] : 0ull; s += v[k]; }
    unsigned long long tot;
    unsigned long long pre = block_exclusive_scan_t<unsigned long long>(s, lds, &tot);
#pragma unroll
    for (int k = 0; k < 16; ++k) { if (base + k < nt) tsum[base + k] = pre; pre += v[k]; }
    if (threadIdx.x == 0) tsum[kScanTile] = tot;
}

__global__ __launch_bounds__(256) void scan64_apply_kernel(unsigned long long* x, int64_t m,
                                                           const unsigned long long* tsum) {
    __shared__ unsigned long long lds[4];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * 16;
    unsigned long long v[16], s = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) { v[k] = (base + k < m) ? x[base + k] : 0ull; s += v[k]; }
    unsigned long long tot;
    unsigned long long pre = block_exclusive_scan_t<unsigned long long>(s, lds, &tot) + tsum[blockIdx.x];
#pragma unroll
    for (int k = 0; k < 16; ++k) { if (base + k < m) x[base + k] = pre; pre += v[k]; }
}

__global__ __launch_bounds__(256) void core_eval_kernel(const CoreArgs A) {
    __shared__ unsigned long long lds4[4];
    __shared__ unsigned long long pre[256];       // exclusive prefix of the lines' points
    __shared__ unsigned long long gpre[3][256];   // the same per evaluation group
    __shared__ double ls_s[256], ls_nu[256], ls_y[256], ls_a[256];
    __shared__ int ls_lo[256], ls_ia[256], ls_ib[256], ls_nl[256], ls_k[256];
    __shared__ double ls_daw[kDawsonIv * kDawsonNc];   // Dawson table (real-axis Im w)
    const int t = threadIdx.x;
    const int g = blockIdx.x * 256 + t;
    const TPParam tp = *A.tp;
    const double Q = A.Q[tp.iq];
    // A line's points |k - kc| <= r - 2 lie inside |z| < 8 (r = floor((X + |xc|)/h) + 1),
    // so they take the Weideman rational (y >= 0.2, group 0) or the Taylor series (group 1);
    // its outer points (|k - kc| >= r - 1, group 2) may fall in the wing rules.  Each group's
    // points are evaluated together (fewer divergent paths per wavefront) and written to
    // the same place as before: the values do not change.
    unsigned long long c = 0, gc[3] = {0, 0, 0};
    if (g < A.n_lines) {
        c = (unsigned long long)A.cnt[g];
        if (c) {
            const CoreLine cl = core_line(A, tp, g, Q);
            ls_s[t] = cl.s; ls_nu[t] = cl.nu; ls_y[t] = cl.y; ls_lo[t] = cl.lo;
            ls_k[t] = core_taylor_terms(cl.y);
            ls_a[t] = A.vv ? cl.a * A.vv[g].y : cl.a;   // area-normalised Vectorized Voigt: I' = I x factor
            const int64_t ia = (int64_t)cl.kc - (cl.r - 2) > cl.lo ? (int64_t)cl.kc - (cl.r - 2) : cl.lo;
            const int64_t ib = (int64_t)cl.kc + (cl.r - 2) < cl.hi ? (int64_t)cl.kc + (cl.r - 2) : cl.hi;
            const unsigned long long cin = ib >= ia ? (unsigned long long)(ib - ia + 1) : 0ull;
            ls_ia[t] = (int)ia;
            ls_ib[t] = (int)ib;
            ls_nl[t] = cin ? (int)(ia - cl.lo) : (int)c;   // outer points left of the inner ones
            gc[cl.y >= 0.2 ? 0 : 1] = cin;
            gc[2] = c - cin;
        }
    }
    unsigned long long tot, gtot[3];
    const unsigned long long ex = block_exclusive_scan_t<unsigned long long>(c, lds4, &tot);
    pre[t] = ex;
#pragma unroll
    for (int q = 0; q < 3; ++q) gpre[q][t] = block_exclusive_scan_t<unsigned long long>(gc[q], lds4, &gtot[q]);
    for (int i = t; i < kDawsonIv * kDawsonNc; i += 256) ls_daw[i] = A.tab->dawson[i];
    const long long base = A.val_base + (long long)A.bsum[blockIdx.x];
    if (g < A.n_lines) A.coff[g] = base + (long long)ex;
    __syncthreads();
    // each thread takes runs of kRun consecutive points: a binary search for the run's first
    // point, then a forward step to the next line where the run crosses into it
    constexpr unsigned long long kRun = 8;
    for (unsigned long long it0 = (unsigned long long)t * kRun; it0 < tot; it0 += 256 * kRun) {
    const unsigned long long itn = it0 + kRun < tot ? it0 + kRun : tot;
    int j = 0, jg = -1;   // line of the previous point and its group
#pragma unroll 1
    for (unsigned long long it = it0; it < itn; ++it) {
        const int grp = it < gtot[0] ? 0 : (it < gtot[0] + gtot[1] ? 1 : 2);
        const unsigned long long li = grp == 0 ? it : (grp == 1 ? it - gtot[0] : it - gtot[0] - gtot[1]);
        const unsigned long long* gp = gpre[grp];
        if (grp != jg) {
            int lo = 0, hi = 255;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (gp[mid] <= li) lo = mid; else hi = mid - 1;
            }
            j = lo;
            jg = grp;
        } else {
            while (j < 255 && gp[j + 1] <= li) ++j;
        }
        const int loc = (int)(li - gp[j]);
        const int k = grp < 2 ? ls_ia[j] + loc : (loc < ls_nl[j] ? ls_lo[j] + loc : ls_ib[j] + 1 + (loc - ls_nl[j]));
        const double x = ls_s[j] * ((A.G.nu_a + (double)k * A.G.dnu) - ls_nu[j]);
        const double y = ls_y[j];
        const double z2 = __builtin_fma(x, x, y * y);
        double re;
        if (z2 < kCoreR2) re = voigt_core_re_k<24>(x, y, ls_k[j], A.tab->w24, ls_daw);
        else if (z2 < kMidR2) re = gh_wing_re(x * x, y, A.tab->gh4);
        else re = gh_wing_re(x * x, y, A.tab->gh2);
        const long long at = base + (long long)pre[j] + (long long)(k - ls_lo[j]);
        if (at < A.val_end) A.val[at] = (float)(ls_a[j] * re);
    }
    }
}

// Core points of a line: 2r + 1 with r = floor((X + |xc|)/h) + 1, X <= 8, |xc| <= h/2
// (kc is the nearest grid index), so at most 16/h + 4, h = sqrt(ln2) dnu / alpha_D;
// alpha_D grows with T, so the bound also holds at every lower temperature.
__global__ __launch_bounds__(256) void core_bound_kernel(const CoreArgs A) {
    __shared__ unsigned long long lds[4];
    const int g = blockIdx.x * 256 + threadIdx.x;
    unsigned long long c = 0;
    if (g < A.n_lines) {
        const int klo = A.L.klo[g], khi = A.L.khi[g];
        if (khi >= klo) {
            const double aD = A.L.nu[g] * A.tp->beta;
            const double inv_h = aD / (kSQRT_LN2 * A.G.dnu);
            const double b = floor(16.0 * inv_h) + 6.0;
            const double win = (double)(khi - klo + 1);
            c = (unsigned long long)(b < win ? b : win);
        }
    }
    unsigned long long tot;
    block_exclusive_scan_t<unsigned long long>(c, lds, &tot);
    if (threadIdx.x == 0) A.bsum[blockIdx.x] = tot;
}

}  // namespace

int64_t core_blocks(int64_t n_lines) { return (n_lines + 255) / 256; }

static hipError_t scan_block_sums(const CoreArgs& a, int64_t nb, hipStream_t s) {
    const int64_t nt = (nb + kScanTile - 1) / kScanTile;
    if (nt > kScanTile) return hipErrorInvalidValue;
    hipLaunchKernelGGL(scan64_tiles_kernel, dim3((unsigned)nt), dim3(256), 0, s, a.bsum, nb, a.scan_tmp);
    hipLaunchKernelGGL(scan64_small_kernel, dim3(1), dim3(256), 0, s, a.scan_tmp, nt);
    hipLaunchKernelGGL(scan64_apply_kernel, dim3((unsigned)nt), dim3(256), 0, s, a.bsum, nb, a.scan_tmp);
    return hipGetLastError();
}

hipError_t launch_scan64(unsigned long long* bsum, int64_t nb, unsigned long long* scan_tmp, hipStream_t s) {
    CoreArgs a{};
    a.bsum = bsum;
    a.scan_tmp = scan_tmp;
    return scan_block_sums(a, nb, s);
}

hipError_t launch_core_count(const CoreArgs& a, hipStream_t s) {
    const int64_t nb = core_blocks(a.n_lines);
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(core_count_kernel, dim3((unsigned)nb), dim3(256), 0, s, a);
    return scan_block_sums(a, nb, s);
}

hipError_t launch_core_bound(const CoreArgs& a, hipStream_t s) {
    const int64_t nb = core_blocks(a.n_lines);
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(core_bound_kernel, dim3((unsigned)nb), dim3(256), 0, s, a);
    return scan_block_sums(a, nb, s);
}

hipError_t launch_core_eval(const CoreArgs& a, hipStream_t s) {
    const int64_t nb = core_blocks(a.n_lines);
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(core_eval_kernel, dim3((unsigned)nb), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace xs
