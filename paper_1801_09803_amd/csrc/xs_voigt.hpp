// Device evaluation of Re w(z), w the Faddeeva function, for the Voigt profile
//   f_V(D) = sqrt(ln2/pi)/alpha_D * Re w(x + i y),  x = sqrt(ln2) D/alpha_D,
//   y = sqrt(ln2) gamma/alpha_D
// (the normalised Doppler (x) Lorentz convolution the paper's Voigt equation
// describes, Sec. "Line profiles").
//
// The plane is split by |z| (y is fixed per line, so the choice is per line and
// per 64-point slice, never per lane):
//  * wings: n-point Gauss-Hermite quadrature of the convolution,
//        Re w(z) ~ (y/pi) sum_j w_j / ((x - t_j)^2 + y^2),
//    summed over node pairs +-t_j as 2 w_j q_j / d_j with
//        p_j = x^2 + y^2 - t_j^2,  d_j = p_j^2 + 4 t_j^2 y^2,  q_j = p_j + 2 t_j^2.
//    (n = 2 is the single rational term of Humlicek's far region.)  The error falls
//    like |z|^-(2n); the zone radii keep it below the precision's target.
//  * core |z| < 8: Weideman's rational approximation (SIAM J. Numer. Anal. 1994) for
//    y >= 0.2; for y < 0.2 a Taylor series in i*y about the real axis,
//        w(x + iy) = sum_k w^(k)(x) (iy)^k / k!,
//        w' = -2 z w + 2i/sqrt(pi),  w^(k+1) = -2 x w^(k) - 2k w^(k-1),
//    started from w(x) = exp(-x^2) + i Im w(x) (Weideman on the real axis), which
//    keeps relative accuracy in Re w where it is much smaller than |w|.
#pragma once

#include "xs_internal.hpp"

namespace xs {

struct cplx { double re, im; };

__device__ __forceinline__ double rcp64(double d) {
    double r = __builtin_amdgcn_rcp(d);
    double e = __builtin_fma(-d, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-d, r, 1.0);
    return __builtin_fma(r, e, r);
}

// w(z) ~ 2 p(Z)/(L - iz)^2 + (1/sqrt(pi))/(L - iz),  Z = (L + iz)/(L - iz).
// p has real coefficients, so p(Z) is the remainder c1 Z + c0 of p divided by
// (t - Z)(t - conj Z) = t^2 - 2 Re Z t + |Z|^2 (synthetic division: two FMA per
// coefficient instead of the four of a complex Horner step).
template <int N>
__device__ __forceinline__ cplx weideman_w(double x, double y, const WeidemanCoef& W) {
    static_assert(N >= 3, "Weideman order");
    const double L = W.L;
    const double dr = L + y, di = -x;      // L - iz
    const double nr = L - y, ni = x;       // L + iz
    const double inv = rcp64(__builtin_fma(dr, dr, di * di));
    const double zr = (nr * dr + ni * di) * inv;
    const double zi = (ni * dr - nr * di) * inv;
    const double r2 = 2.0 * zr, s2 = __builtin_fma(zr, zr, zi * zi);
    double b2 = W.a[N - 1];
    double b1 = __builtin_fma(r2, b2, W.a[N - 2]);
#pragma unroll
    for (int k = N - 3; k >= 1; --k) {
        const double b0 = __builtin_fma(r2, b1, __builtin_fma(-s2, b2, W.a[k]));
        b2 = b1;
        b1 = b0;
    }
    const double pr = __builtin_fma(zr, b1, __builtin_fma(-s2, b2, W.a[0]));
    const double pi = zi * b1;
    const double ir = dr * inv, ii = -di * inv;            // 1/(L - iz)
    const double i2r = ir * ir - ii * ii, i2i = 2.0 * ir * ii;
    cplx w;
    w.re = 2.0 * (pr * i2r - pi * i2i) + kINV_SQRT_PI * ir;
    w.im = 2.0 * (pr * i2i + pi * i2r) + kINV_SQRT_PI * ii;
    return w;
}

// Re w(x + iy) for |z| < 8 with relative accuracy (N Weideman terms, K Taylor terms).
template <int N, int K>
__device__ __forceinline__ double voigt_core_re(double x, double y, const WeidemanCoef& W) {
    if (y >= 0.2) return weideman_w<N>(x, y, W).re;
    // w^(0), w^(1) on the real axis
    double w0r = exp(-x * x);
    double w0i = weideman_w<N>(x, 0.0, W).im;
    double w1r = -2.0 * x * w0r;
    double w1i = -2.0 * x * w0i + 2.0 * kINV_SQRT_PI;
    double sum = w0r - w1i * y;            // k = 0, 1:  Re(w0) + Re(i y w1)
    double fac = y;                        // y^k / k!
#pragma unroll
    for (int k = 1; k < K; ++k) {
        const double w2r = -2.0 * x * w1r - 2.0 * k * w0r;
        const double w2i = -2.0 * x * w1i - 2.0 * k * w0i;
        fac *= y / (k + 1);
        // Re(w^(k+1) i^(k+1)):  (k+1) mod 4 = 0: re, 1: -im, 2: -re, 3: im
        const int m = (k + 1) & 3;
        const double term = (m == 0) ? w2r : (m == 1) ? -w2i : (m == 2) ? -w2r : w2i;
        sum = __builtin_fma(term, fac, sum);
        w0r = w1r; w0i = w1i; w1r = w2r; w1i = w2i;
    }
    return sum;
}

// Taylor terms about the real axis that keep Re w(x + iy) within 1e-10 relative over
// |z| < 8 for this y (the series' tail shrinks like y^(K+1); thresholds at half the y where
// K terms first reach that accuracy).
__device__ __forceinline__ int core_taylor_terms(double y) {
    return y < 1.0e-6 ? 1 : y < 1.7e-5 ? 2 : y < 7.0e-4 ? 3 : y < 3.7e-3 ? 4 : y < 9.8e-3 ? 5
         : y < 2.0e-2 ? 6 : y < 3.3e-2 ? 7 : y < 5.0e-2 ? 8 : y < 7.1e-2 ? 9 : y < 9.1e-2 ? 10 : 12;
}

// Im w(x) on the real axis, (2/sqrt(pi)) D(x) with Dawson's function D odd, from the
// piecewise polynomials of the table dt (|x| < kDawsonIv / 2; Horner in u)
__device__ __forceinline__ double im_w_real(double x, const double* dt) {
    const double ax = fabs(x);
    int iv = (int)(ax * 2.0);
    iv = iv < kDawsonIv - 1 ? iv : kDawsonIv - 1;
    const double u = (ax - (0.5 * iv + 0.25)) * 4.0;
    const double* c = dt + iv * kDawsonNc;
    double p = c[kDawsonNc - 1];
#pragma unroll
    for (int j = kDawsonNc - 2; j >= 0; --j) p = __builtin_fma(p, u, c[j]);
    return copysign(2.0 * kINV_SQRT_PI * p, x);
}

// voigt_core_re with the number of Taylor terms chosen per line (K from core_taylor_terms,
// at most 12) and the real-axis Im w from the Dawson table dt; the factorial weights use
// constant reciprocals.
template <int N>
__device__ __forceinline__ double voigt_core_re_k(double x, double y, int K, const WeidemanCoef& W,
                                                  const double* dt) {
    if (y >= 0.2) return weideman_w<N>(x, y, W).re;
    double w0r = exp(-x * x);
    double w0i = im_w_real(x, dt);
    double w1r = -2.0 * x * w0r;
    double w1i = -2.0 * x * w0i + 2.0 * kINV_SQRT_PI;
    double sum = w0r - w1i * y;
    double fac = y;
    // unrolled with constant weights; lanes past their line's K are masked off
#pragma unroll
    for (int k = 1; k < 12; ++k) {
        if (k < K) {
            const double w2r = -2.0 * x * w1r - 2.0 * k * w0r;
            const double w2i = -2.0 * x * w1i - 2.0 * k * w0i;
            fac *= y * (1.0 / (k + 1));
            const int m = (k + 1) & 3;
            const double term = (m == 0) ? w2r : (m == 1) ? -w2i : (m == 2) ? -w2r : w2i;
            sum = __builtin_fma(term, fac, sum);
            w0r = w1r; w0i = w1i; w1r = w2r; w1i = w2i;
        }
    }
    return sum;
}

// Re w from the n-point Gauss-Hermite rule (pairs + optional zero node), double.
__device__ __forceinline__ double gh_wing_re(double u, double y, const GHPairs& G) {
    const double y2 = y * y;
    double acc = G.has_zero ? G.w0 * rcp64(u + y2) : 0.0;
    for (int j = 0; j < G.n_pairs; ++j) {
        const double t2 = G.t[j] * G.t[j];
        const double p = u + y2 - t2;
        const double d = __builtin_fma(p, p, 4.0 * t2 * y2);
        acc = __builtin_fma(2.0 * G.w[j] * (p + 2.0 * t2), rcp64(d), acc);
    }
    return acc * y * (1.0 / kPI);
}

}  // namespace xs

namespace xs {

// Re w, Re w' and Im w' for |z| < 8 (same split as voigt_core_re).
template <int N, int K>
__device__ __forceinline__ void voigt_core_dw(double x, double y, const WeidemanCoef& W, double* re_w,
                                              double* re_dw, double* im_dw) {
    if (y >= 0.2) {
        const cplx w = weideman_w<N>(x, y, W);
        // w' = -2 z w + 2i/sqrt(pi)
        *re_w = w.re;
        *re_dw = -2.0 * (x * w.re - y * w.im);
        *im_dw = -2.0 * (x * w.im + y * w.re) + 2.0 * kINV_SQRT_PI;
        return;
    }
    // Taylor in iy about the real axis: w(z) = sum w^(k) (iy)^k/k!, w'(z) = sum w^(k+1) (iy)^k/k!
    double w0r = exp(-x * x);
    double w0i = weideman_w<N>(x, 0.0, W).im;
    double w1r = -2.0 * x * w0r;
    double w1i = -2.0 * x * w0i + 2.0 * kINV_SQRT_PI;
    double sr = w0r, dr = w1r, di = w1i;   // k = 0 terms
    double fac = 1.0;                      // y^k / k!
#pragma unroll
    for (int k = 0; k < K; ++k) {
        // w^(k+2) from w^(k+1), w^(k)
        const double w2r = -2.0 * x * w1r - 2.0 * (k + 1) * w0r;
        const double w2i = -2.0 * x * w1i - 2.0 * (k + 1) * w0i;
        fac *= y / (k + 1);
        const int m = (k + 1) & 3;   // i^(k+1)
        // w term: w^(k+1) i^(k+1); w' term: w^(k+2) i^(k+1)
        if (m == 0) { sr += w1r * fac; dr += w2r * fac; di += w2i * fac; }
        else if (m == 1) { sr -= w1i * fac; dr -= w2i * fac; di += w2r * fac; }
        else if (m == 2) { sr -= w1r * fac; dr -= w2r * fac; di -= w2i * fac; }
        else { sr += w1i * fac; dr += w2i * fac; di -= w2r * fac; }
        w0r = w1r; w0i = w1i; w1r = w2r; w1i = w2i;
    }
    *re_w = sr;
    *re_dw = dr;
    *im_dw = di;
}

// n-point Gauss-Hermite approximation V = Re w of the Voigt convolution and its
// derivatives: returns V, x dV/dx and dV/dy (double).  With u = x^2 and, per node pair,
// p = u + y^2 - t^2, q = p + 2 t^2, d = p^2 + 4 t^2 y^2 (V = (y/pi) sum c q/d):
//   x dV/dx = (y/pi) sum c 2u (1/d - 2 p q/d^2)
//   dV/dy   = (1/pi) sum c (q/d + 2 y^2 (1/d - 2 q^2/d^2))
__device__ __forceinline__ void gh_wing_dv(double u, double y, const GHPairs& G, double* v, double* xvx,
                                           double* vy) {
    const double y2 = y * y;
    double s0 = 0.0, sx = 0.0, sy = 0.0;
    const int np = G.n_pairs + (G.has_zero ? 1 : 0);
    for (int j = 0; j < np; ++j) {
        const bool zero = j == G.n_pairs;
        const double t2 = zero ? 0.0 : G.t[j] * G.t[j];
        const double c = zero ? G.w0 : 2.0 * G.w[j];
        const double p = u + y2 - t2;
        const double q = p + 2.0 * t2;
        const double r = rcp64(__builtin_fma(p, p, 4.0 * t2 * y2));
        const double qr = q * r;
        s0 = __builtin_fma(c, qr, s0);
        sx = __builtin_fma(c, __builtin_fma(-2.0 * p * qr, r, r), sx);
        sy = __builtin_fma(c, __builtin_fma(2.0 * y2, __builtin_fma(-2.0 * q * qr, r, r), qr), sy);
    }
    *v = s0 * y * (1.0 / kPI);
    *xvx = sx * 2.0 * u * y * (1.0 / kPI);
    *vy = sy * (1.0 / kPI);
}

}  // namespace xs
