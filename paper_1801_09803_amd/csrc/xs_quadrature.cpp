// Host-side generation of the quadrature tables used by the device Faddeeva code.
//
//  * Gauss-Hermite rules (weight exp(-t^2)): nodes are the zeros of the Hermite
//    polynomial H_n, located by a sign-change scan of the orthonormal three-term
//    recurrence and refined by bisection in long double; weights are the
//    Christoffel numbers 1 / sum_k p_k(t)^2 of the orthonormal polynomials.
//  * Weideman's rational approximation of w(z) (J.A.C. Weideman, SIAM J. Numer.
//    Anal. 31 (1994) 1497): with L = N^(1/2) 2^(-1/4), the coefficients a_n are the
//    cosine coefficients of f(theta) = exp(-t^2)(L^2 + t^2), t = L tan(theta/2),
//    sampled at theta_k = k pi / M, M = 2N, k = -M..M-1.
#include "xs_internal.hpp"

#include <cmath>
#include <vector>

namespace xs {

namespace {

// Orthonormal Hermite polynomials p_0..p_n at t (weight exp(-t^2)).
long double hermite_orthonormal(int n, long double t, long double* sum_sq_below_n) {
    const long double pi = 3.141592653589793238462643383279502884L;
    long double pm1 = 0.0L;
    long double p = 1.0L / std::sqrt(std::sqrt(pi));
    long double ss = 0.0L;
    for (int k = 0; k < n; ++k) {
        ss += p * p;
        long double pn = std::sqrt(2.0L / (k + 1)) * t * p - std::sqrt((long double)k / (k + 1)) * pm1;
        pm1 = p;
        p = pn;
    }
    if (sum_sq_below_n) *sum_sq_below_n = ss;
    return p;
}

}  // namespace

void gauss_hermite_rule(int n, double* nodes, double* weights) {
    // All zeros of H_n lie inside |t| < sqrt(2n + 1).
    const long double tmax = std::sqrt(2.0L * n + 1.0L) + 0.5L;
    const int steps = 200000;
    const long double dt = 2.0L * tmax / steps;
    int found = 0;
    long double a = -tmax;
    long double fa = hermite_orthonormal(n, a, nullptr);
    for (int i = 1; i <= steps && found < n; ++i) {
        long double b = -tmax + i * dt;
        long double fb = hermite_orthonormal(n, b, nullptr);
        // a root exactly at a scan point was taken with the interval that ended there
        if (fa != 0.0L && (fb == 0.0L || (fa < 0) != (fb < 0))) {
            long double lo = a, hi = b, flo = fa;
            for (int it = 0; it < 200; ++it) {
                long double mid = 0.5L * (lo + hi);
                if (mid == lo || mid == hi) break;
                long double fm = hermite_orthonormal(n, mid, nullptr);
                if ((fm < 0) == (flo < 0)) { lo = mid; flo = fm; } else { hi = mid; }
            }
            long double t = 0.5L * (lo + hi);
            long double ss;
            hermite_orthonormal(n, t, &ss);
            nodes[found] = (double)t;
            weights[found] = (double)(1.0L / ss);
            ++found;
        }
        a = b;
        fa = fb;
    }
    // symmetrise (the rule is exactly symmetric about 0)
    for (int i = 0; i < n / 2; ++i) {
        double t = 0.5 * (nodes[n - 1 - i] - nodes[i]);
        double w = 0.5 * (weights[n - 1 - i] + weights[i]);
        nodes[i] = -t; nodes[n - 1 - i] = t;
        weights[i] = w; weights[n - 1 - i] = w;
    }
    if (n % 2) nodes[n / 2] = 0.0;
}

void make_gh_pairs(int n, GHPairs* out) {
    std::vector<double> t(n), w(n);
    gauss_hermite_rule(n, t.data(), w.data());
    out->n_pairs = n / 2;
    out->has_zero = n % 2;
    out->w0 = (n % 2) ? w[n / 2] : 0.0;
    for (int i = 0; i < n / 2 && i < kMaxGHPairs; ++i) {
        out->t[i] = t[n - 1 - i];
        out->w[i] = w[n - 1 - i];
    }
}

// Dawson's function D(x) = exp(-x^2) int_0^x exp(t^2) dt by Rybicki's sum (G. B. Rybicki,
// Computers in Physics 3, 85 (1989)): D(x) = lim_{h->0} pi^-1/2 sum_{n odd} exp(-(x - n h)^2)/n,
// whose error at step h falls like exp(-(pi / 2h)^2) (below 1e-26 at h = 0.2); terms more
// than 20 from x are below exp(-400) and left out.
static long double dawson_ref(long double x) {
    const long double pi = 3.141592653589793238462643383279502884L;
    const long double h = 0.2L;
    const int n0 = (int)std::floor(x / h);
    long double s = 0.0L;
    for (int n = n0 - 101; n <= n0 + 101; ++n) {
        if (n % 2 == 0) continue;
        const long double d = x - n * h;
        s += std::exp(-d * d) / n;
    }
    return s / std::sqrt(pi);
}

void dawson_table(double* out) {
    // per interval: Chebyshev interpolation at kDawsonNc points of the first kind, its
    // Chebyshev series turned into powers of u (T_0 = 1, T_1 = u, T_{j+1} = 2u T_j - T_{j-1})
    const long double pi = 3.141592653589793238462643383279502884L;
    constexpr int M = kDawsonNc;
    for (int iv = 0; iv < kDawsonIv; ++iv) {
        const long double c = 0.5L * iv + 0.25L;
        long double f[M];
        for (int k = 0; k < M; ++k) f[k] = dawson_ref(c + 0.25L * std::cos(pi * (k + 0.5L) / M));
        long double cheb[M];
        for (int j = 0; j < M; ++j) {
            long double acc = 0.0L;
            for (int k = 0; k < M; ++k) acc += f[k] * std::cos(pi * j * (k + 0.5L) / M);
            cheb[j] = acc * (j == 0 ? 1.0L : 2.0L) / M;
        }
        long double poly[M] = {}, tm[M] = {}, t0[M] = {}, t1[M] = {};
        t0[0] = 1.0L;   // T_0
        t1[1] = 1.0L;   // T_1
        for (int i = 0; i < M; ++i) poly[i] += cheb[0] * t0[i] + (M > 1 ? cheb[1] * t1[i] : 0.0L);
        for (int j = 2; j < M; ++j) {
            for (int i = 0; i < M; ++i) tm[i] = -t0[i] + (i > 0 ? 2.0L * t1[i - 1] : 0.0L);
            for (int i = 0; i < M; ++i) {
                poly[i] += cheb[j] * tm[i];
                t0[i] = t1[i];
                t1[i] = tm[i];
            }
        }
        for (int i = 0; i < M; ++i) out[iv * M + i] = (double)poly[i];
    }
}

void weideman_coefficients(int n, WeidemanCoef* out) {
    const long double pi = 3.141592653589793238462643383279502884L;
    const int M = 2 * n;
    const long double L = std::sqrt((long double)n / std::sqrt(2.0L));
    out->n = n;
    out->L = (double)L;
    // f at theta_k, k = -M+1..M-1 (the k = -M sample, t = -inf, is zero)
    std::vector<long double> f(2 * M);
    for (int k = -M + 1; k <= M - 1; ++k) {
        long double th = k * pi / M;
        long double t = L * std::tan(0.5L * th);
        f[k + M] = std::exp(-t * t) * (L * L + t * t);
    }
    f[0] = 0.0L;
    for (int m = 1; m <= n; ++m) {
        long double acc = 0.0L;
        for (int k = -M; k <= M - 1; ++k) acc += f[k + M] * std::cos(m * k * pi / M);
        out->a[m - 1] = (double)(acc / (2 * M));
    }
}

}  // namespace xs
