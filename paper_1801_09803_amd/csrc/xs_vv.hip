// Vectorized Voigt pre-pass (Sec. "Vectorized Voigt approximation" and Sec. "Binned
// Vectorized Voigt with the line area preserved"): per sorted line and (T, P)
//   beta   = f_V(R) / f_ref(R), the continuity factor at the radius R (or 1), where f_ref is
//            the Voigt profile with the Doppler width of a line at 1 cm^-1 (alpha_ref =
//            alpha_D / nu) and the line's Lorentz width;
//   factor = 1, or for the area-normalised form 1 / (dnu S), S the sum of the line's V-V
//            profile values over its whole cut-off window on the extended grid.
//
// S = (core sum) + beta (wing sum).  Far from a centre (|z| >= 40 in the variables of the
// profile), a Voigt profile of widths (alpha, gamma) is its Lorentzian L(D) times
// 1 + (3 D^2 - gamma^2) / (2 s^2 (D^2 + gamma^2)^2) (s = sqrt(ln2)/alpha) to a relative
// ~4/|z|^4; the reference profile's whole wing is that far (x_ref = sqrt(ln2) R / alpha_ref
// >= 2e4, checked by the host).  Over a run of grid points the Lorentzian sums exactly
// to a difference of digamma functions,
//     sum_{m=0}^{M} 1/((u + m)^2 + b^2) = Im[psi(u + M + 1 - i b) - psi(u - i b)] / b,
// (u, b in grid steps), with psi from its asymptotic series once Re >= 16 (the first
// terms are added directly), and the correction term is integrated in closed form (the
// antiderivative of (3 D^2 - g^2)/(D^2 + g^2)^3 is -D/(D^2 + g^2)^2) by the midpoint rule.
// FP64 path: the core points are summed explicitly with its own zones, one wavefront
// per line.  FP32 path, one thread per line: the points within max(|z| < 40, 16 dnu)
// of the centre explicitly (double-precision core for |z| < 8, the single-precision
// 4-node rule beyond), the rest of the core region and the wings in closed form.
#include "xs_forward_common.hpp"

namespace xs {

namespace {

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return __shfl(v, 0, 64);
}

// Re w(x + iy) with the FP64 path's zones (relative accuracy ~1e-13).
__device__ __forceinline__ double re_w64(double x, double y, const Tables* tab) {
    const double u = x * x;
    const double z2 = u + y * y;
    if (z2 < 64.0) return voigt_core_re<40, 14>(x, y, tab->w40);
    if (z2 < 400.0) return gh_wing_re(u, y, tab->gh12);
    if (z2 < 3600.0) return gh_wing_re(u, y, tab->gh6);
    if (z2 < 4.84e6) return gh_wing_re(u, y, tab->gh4);
    return gh_wing_re(u, y, tab->gh2);
}

// Im psi(u - i b), u >= 16, b >= 0: Im ln z - Im 1/(2z) + even terms through z^-10.
__device__ __forceinline__ double im_psi(double u, double b) {
    const double d = __builtin_fma(u, u, b * b);
    const double ir = u / d, ii = b / d;               // 1/z
    const double wr = ir * ir - ii * ii, wi = 2.0 * ir * ii;   // 1/z^2
    const double c[5] = {-1.0 / 132.0, 1.0 / 240.0, -1.0 / 252.0, 1.0 / 120.0, -1.0 / 12.0};
    double pr = c[0], pi = 0.0;
#pragma unroll
    for (int j = 1; j < 5; ++j) {
        const double t = pr * wr - pi * wi + c[j];
        pi = pr * wi + pi * wr;
        pr = t;
    }
    const double qi = pr * wi + pi * wr;               // Im of w * (series in w)
    return atan2(-b, u) - 0.5 * ii + qi;
}

// sum_{m=0}^{M} 1 / ((u0 + m)^2 + b^2), u0 > 0, b > 0 (grid steps)
__device__ __forceinline__ double lorentz_steps_sum(double u0, double M, double b) {
    double acc = 0.0;
    double m = 0.0;
    for (; m <= M && u0 + m < 16.0; m += 1.0) {
        const double u = u0 + m;
        acc += 1.0 / __builtin_fma(u, u, b * b);
    }
    if (m > M) return acc;
    return acc + (im_psi(u0 + M + 1.0, b) - im_psi(u0 + m, b)) / b;
}

// sum over k in [klo, khi] of 1/((k - a)^2 + b^2), b > 0 (split at the centre a)
__device__ __forceinline__ double lorentz_range(double klo, double khi, double a, double b) {
    if (khi < klo) return 0.0;
    const double fa = floor(a);
    double acc = 0.0;
    const double l1 = fmin(khi, fa);   // k <= fa: distance a - k >= 0
    if (l1 >= klo) acc += lorentz_steps_sum(a - l1, l1 - klo, b);
    const double r0 = fmax(klo, fa + 1.0);
    if (khi >= r0) acc += lorentz_steps_sum(r0 - a, khi - r0, b);
    return acc;
}

// Profile sum over grid points [klo, khi] of a Voigt profile far from its centre:
// Lorentzian (exact sum) plus the integrated |z|^-2 correction.  s = sqrt(ln2)/alpha.
__device__ __forceinline__ double far_sum(double klo, double khi, double nu, double gam, double s, const Geometry& G) {
    if (khi < klo || !(gam > 0.0)) return 0.0;
    const double h = G.dnu;
    const double a = (nu - G.nu_a) / h;
    const double lor = gam / (kPI * h * h) * lorentz_range(klo, khi, a, gam / h);
    const double cg = gam / (2.0 * kPI * s * s);
    const double d1 = (G.nu_a + (khi + 0.5) * h) - nu, d0 = (G.nu_a + (klo - 0.5) * h) - nu;
    const double q1 = __builtin_fma(d1, d1, gam * gam), q0 = __builtin_fma(d0, d0, gam * gam);
    return lor + cg * (-d1 / (q1 * q1) + d0 / (q0 * q0)) / h;
}

// Re w from the single-precision 4-node rule (8 <= |z| < 40)
__device__ __forceinline__ float re_w_gh4f(float x, float y, const Tables* tab) {
    const float u = x * x, y2 = y * y;
    float acc = 0.0f;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const float t2 = (float)(tab->gh4.t[j] * tab->gh4.t[j]);
        const float p = u + y2 - t2;
        const float d = __builtin_fmaf(p, p, 4.0f * t2 * y2);
        acc = __builtin_fmaf(2.0f * (float)tab->gh4.w[j] * (p + 2.0f * t2), __builtin_amdgcn_rcpf(d), acc);
    }
    return acc * y * (float)(1.0 / kPI);
}

// FP32-path area factor of one line (thread per line)
__device__ __forceinline__ double vv_factor32(const VVArgs& A, double nu, double aD, double gam, double beta,
                                              double sr) {
    const Geometry& G = A.G;
    const double h = G.dnu, R = G.vv_radius;
    const double s = kSQRT_LN2 / aD, y = gam * s;
    const double kwl = ceil((nu - G.cutoff - G.nu_a) / h), kwh = floor((nu + G.cutoff - G.nu_a) / h);
    const double kvl = ceil((nu - R - G.nu_a) / h), kvh = floor((nu + R - G.nu_a) / h);
    const double c0 = fmax(kwl, kvl), c1 = fmin(kwh, kvh);
    // explicit zone: |z| < 40 or within 16 grid steps of the centre
    const double X = y < 40.0 ? sqrt(1600.0 - y * y) : 0.0;
    const double De = fmax(X / s, 16.0 * h);
    const double e0 = fmax(c0, ceil((nu - De - G.nu_a) / h)), e1 = fmin(c1, floor((nu + De - G.nu_a) / h));
    double ex = 0.0;
    for (double k = e0; k <= e1; k += 1.0) {
        const double x = s * ((G.nu_a + k * h) - nu);
        const double z2 = __builtin_fma(x, x, y * y);
        if (z2 < kCoreR2) ex += voigt_core_re<24, 8>(x, y, A.tab->w24);
        else if (z2 < kMidR2) ex += (double)re_w_gh4f((float)x, (float)y, A.tab);
        else {
            const float q = (float)z2, yf = (float)y, p = q - 0.5f;
            ex += (double)(yf * (float)kINV_SQRT_PI * (q + 0.5f) * __builtin_amdgcn_rcpf(__builtin_fmaf(p, p, 2.0f * yf * yf)));
        }
    }
    double tot = kSQRT_LN2_PI / aD * ex;
    tot += far_sum(c0, fmin(c1, e0 - 1.0), nu, gam, s, G);
    tot += far_sum(fmax(c0, e1 + 1.0), c1, nu, gam, s, G);
    tot += beta * (far_sum(kwl, kvl - 1.0, nu, gam, sr, G) + far_sum(kvh + 1.0, kwh, nu, gam, sr, G));
    return tot > 0.0 ? 1.0 / (h * tot) : 0.0;
}

template <bool F64, bool NORM>
__global__ __launch_bounds__(256) void vv_prep_kernel(const VVArgs A) {
    const Geometry G = A.G;
    const TPParam tp = *A.tp;
    const double R = G.vv_radius;
    const double ar = tp.beta;                        // alpha_D of a line at 1 cm^-1 (Eq. 16)
    const double sr = kSQRT_LN2 / ar;
    // FP64 normalisation: one wavefront per line (grid-stride); otherwise one thread per line
    constexpr bool WAVE = F64 && NORM;
    const int lane = WAVE ? (int)(threadIdx.x & 63) : 0;
    const int64_t first = WAVE ? ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6 : (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t stride = WAVE ? (int64_t)gridDim.x * 4 : (int64_t)gridDim.x * 256;
    for (int64_t gi = first; gi < A.n_lines; gi += stride) {
        const int g = (int)gi;
        const double nu = A.L.nu[g];
        const double aD = nu * tp.beta;                                                          // Eq. 16
        const double gam = (double)A.L.gref[g] * exp((double)A.L.nexp[g] * tp.ln_T0_T) * tp.p_over_p0;  // Eq. 18
        const double s = kSQRT_LN2 / aD, y = gam * s;
        double beta = 1.0;
        if (A.use_beta) {
            const double fv = kSQRT_LN2_PI / aD * re_w64(s * R, y, A.tab);
            const double xr = sr * R, yr = sr * gam;
            const double fr = kSQRT_LN2_PI / ar * gh_wing_re(xr * xr, yr, A.tab->gh2);
            if (fr > 0.0) beta = fv / fr;
        }
        double factor = 1.0;
        if (NORM && !F64) factor = vv_factor32(A, nu, aD, gam, beta, sr);
        if (WAVE) {
            const double h = G.dnu;
            // whole window and core region on the extended grid (indices as doubles)
            const double kwl = ceil((nu - G.cutoff - G.nu_a) / h), kwh = floor((nu + G.cutoff - G.nu_a) / h);
            const double kvl = ceil((nu - R - G.nu_a) / h), kvh = floor((nu + R - G.nu_a) / h);
            const double c0 = fmax(kwl, kvl), c1 = fmin(kwh, kvh);
            double part = 0.0;
            for (double k = c0 + (double)lane; k <= c1; k += 64.0) part += re_w64(s * ((G.nu_a + k * h) - nu), y, A.tab);
            double tot = kSQRT_LN2_PI / aD * wave_sum_d(part);
            tot += beta * (far_sum(kwl, kvl - 1.0, nu, gam, sr, G) + far_sum(kvh + 1.0, kwh, nu, gam, sr, G));
            factor = tot > 0.0 ? 1.0 / (h * tot) : 0.0;
        }
        if (lane == 0) A.out[g] = make_double2(beta, factor);
    }
}

}  // namespace

hipError_t launch_vv_prep(const VVArgs& a, hipStream_t s) {
    if (a.n_lines <= 0) return hipSuccess;
    if (a.normalise && a.fp64) {
        const int64_t want = ((int64_t)a.n_lines + 3) / 4;
        const dim3 grid((unsigned)(want < 16384 ? want : 16384)), block(256);
        hipLaunchKernelGGL((vv_prep_kernel<true, true>), grid, block, 0, s, a);
    } else {
        const dim3 grid((unsigned)(((int64_t)a.n_lines + 255) / 256)), block(256);
        if (a.normalise) hipLaunchKernelGGL((vv_prep_kernel<false, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((vv_prep_kernel<true, false>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace xs
