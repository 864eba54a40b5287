// Adjoint of the sampled Voigt cross section (extension of the paper's method: the
// derivative of Eq. 1, 2, 16, 18 and the Voigt profile of Sec. "Line profiles").
//
// Given gbar_k = dL/dsigma_k on the grid, each line i needs three window sums
// (phi = N Re w(z), N = sqrt(ln2/pi)/alpha_D, z = x + iy, x = s D, y = s gamma,
// s = sqrt(ln2)/alpha_D, V = Re w):
//   A0 = sum gbar V,   Ax = sum gbar x dV/dx,   Ay = sum gbar dV/dy
// from which
//   R0 = sum gbar phi            = N A0
//   Rg = sum gbar dphi/dgamma    = N s Ay
//   Ra = sum gbar dphi/dalpha_D  = -(N/alpha_D) (A0 + Ax + y Ay)
//   dL/dln A_i     = S_i R0
//   dL/dgamma_ref  = S_i Rg gamma_i / gamma_ref_i
//   dL/dn_i        = S_i Rg gamma_i ln(T0/T)
//   dL/dT = sum_i S_i (tau_i R0 + Ra alpha_D/(2T) - Rg n_i gamma_i / T),
//           tau_i = c2 E''/T^2 - (c2 nu/T^2)/expm1(c2 nu/T) - (dQ/dT)/Q
//   dL/dP = sum_i S_i Rg gamma_i / P   (gamma_ref (T0/T)^n / P0 at P = 0)
// Profiles are recomputed, nothing is stored from the forward pass.  Wing points use
// the analytic derivatives of the Gauss-Hermite rules, |z| < 8 points the core with w'
// (Weideman / Taylor).  FP64 path: one wavefront per line walks its window 64 points at
// a time, all in double.  FP32 path: three passes (below) with single-precision wings
// (the forward kernel's power-of-two scaling) and double-precision core points and sums.
// Per-line results go to the caller's line order; dL/dT and dL/dP are reduced in a fixed
// order.
#include "xs_adjoint.hpp"
#include "xs_forward_common.hpp"

namespace xs {

namespace {

__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// single-precision Gauss-Hermite wing sums in scaled variables (see file header of
// xs_forward_f32.hip for the scaling): per pair j, p = x_s^2 + a_j, q = p + b_j,
// d = p^2 + e_j, r = 1/d; returns sum c q r, sum c u (r - 2 p q r^2), sum c (q r + 2 y_s^2 (r - 2 q^2 r^2))
template <int NP>
__device__ __forceinline__ void wing_dv_f32(float xs, const float* a, const float* b, const float* e,
                                            const float* c, float ys2, float* sv, float* sx, float* sy) {
    const float u = xs * xs;
    float v0 = 0.f, v1 = 0.f, v2 = 0.f;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const float p = u + a[j];
        const float q = p + b[j];
        const float r = __builtin_amdgcn_rcpf(__builtin_fmaf(p, p, e[j]));
        const float qr = q * r;
        v0 = __builtin_fmaf(c[j], qr, v0);
        v1 = __builtin_fmaf(c[j], r * __builtin_fmaf(-2.0f * p, qr, 1.0f), v1);
        v2 = __builtin_fmaf(c[j], __builtin_fmaf(2.0f * ys2, r * __builtin_fmaf(-2.0f * q, qr, 1.0f), qr), v2);
    }
    *sv = v0;
    *sx = v1 * u;
    *sy = v2;
}

// FP64 path: one wavefront per line, every window point in double precision.
__global__ __launch_bounds__(256) void adjoint64_kernel(const AdjArgs A) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int nwaves = gridDim.x * 4;
    const Geometry G = A.G;
    const double T = A.tp.T;
    const double Q = A.Q[0], dQ = A.dQ[0];
    const Tables* tab = A.tab;
    const double* gbar = static_cast<const double*>(A.gbar);

    for (int g = blockIdx.x * 4 + wave; g < A.n_lines; g += nwaves) {
        const LineSetup ls = line_setup(A.L, A.tp, g, Q);
        const double s = kSQRT_LN2 / ls.aD;
        const double y = ls.gam * s;
        const double Nn = kSQRT_LN2_PI / ls.aD;
        const double y2 = y * y;
        double c0 = 0.0, cx = 0.0, cy = 0.0;
        for (int k = ls.klo + lane; k <= ls.khi; k += 64) {
            const double gb = gbar[k];
            const double x = s * ((G.nu_a + (double)k * G.dnu) - ls.nu);
            const double u = x * x;
            const double z2 = u + y2;
            double v, xvx, vy;
            if (z2 < kCoreR2) {
                double rw, rdw, idw;
                voigt_core_dw<40, 14>(x, y, tab->w40, &rw, &rdw, &idw);
                v = rw; xvx = x * rdw; vy = -idw;
            } else if (z2 < 400.0) {
                gh_wing_dv(u, y, tab->gh12, &v, &xvx, &vy);
            } else if (z2 < 3600.0) {
                gh_wing_dv(u, y, tab->gh6, &v, &xvx, &vy);
            } else if (z2 < 4.84e6) {
                gh_wing_dv(u, y, tab->gh4, &v, &xvx, &vy);
            } else {
                gh_wing_dv(u, y, tab->gh2, &v, &xvx, &vy);
            }
            c0 = __builtin_fma(gb, v, c0);
            cx = __builtin_fma(gb, xvx, cx);
            cy = __builtin_fma(gb, vy, cy);
        }
        c0 = wave_sum64(c0); cx = wave_sum64(cx); cy = wave_sum64(cy);
        if (lane == 0) {
            const double R0 = Nn * c0;
            const double Rg = Nn * s * cy;
            const double Ra = -(Nn / ls.aD) * (c0 + cx + y * cy);
            const double S = ls.S;
            const double gref = (double)A.L.gref[g];
            const double nexp = (double)A.L.nexp[g];
            const int o = A.L.orig[g];
            if (A.dlnA) static_cast<double*>(A.dlnA)[o] = S * R0;
            if (A.dgref) static_cast<double*>(A.dgref)[o] = gref > 0.0 ? S * Rg * ls.gam / gref : 0.0;
            if (A.dn) static_cast<double*>(A.dn)[o] = S * Rg * ls.gam * A.tp.ln_T0_T;
            const double x2 = (kC2 * ls.nu) / T;
            const double tau = (kC2 * A.L.elow[g]) / (T * T) - ((kC2 * ls.nu) / (T * T)) / expm1(x2) - dQ / Q;
            A.pT[g] = S * (tau * R0 + Ra * ls.aD / (2.0 * T) - Rg * nexp * ls.gam / T);
            const double dgam_dP = A.tp.P > 0.0 ? ls.gam / A.tp.P
                                                : gref * exp(nexp * A.tp.ln_T0_T) / A.P0;
            A.pP[g] = S * Rg * dgam_dP;
        }
    }
}

// ------------------------------------------------------------ FP32 path, three passes
// 1. adj32_prep: one thread per line: the double-precision setup reduced to a record of
//    scaled single-precision wing coefficients and index ranges, and the window sums over
//    the line's core points [kcl, kch] (the forward core pre-pass's range: every point with
//    |z| < 8 lies inside it) in double precision (core with w', or the 4- / 2-node rule).
// 2. adj32_wing: one wavefront per line: the window sums over the other points with the
//    single-precision Gauss-Hermite derivatives, by index runs: the 2-node rule beyond the
//    line's |z| = 40 radius, the 4-node rule inside it (the core excluded), 8-point
//    single-precision partials folded into double.
// 3. adj32_final: one thread per line: R0, R_gamma, R_alpha and the gradients.
enum : int { J_HS = 0, J_XCS = 1, J_YS2 = 2, J_Z1S = 3, J_A2 = 4, J_B2 = 5, J_E2 = 6, J_C2 = 7,
             J_A4 = 8, J_B4 = 10, J_E4 = 12, J_C4 = 14, J_KLO = 16, J_KHI = 17, J_KC = 18, J_KCL = 19,
             J_KCH = 20, J_RAD = 21 };

// scaling of the single-precision wing variables: x_s = x sc keeps x_s^4 in range
__device__ __forceinline__ double wing_scale(double s, const Geometry& G) {
    const double xmax = s * (G.cutoff + 2.0 * G.dnu) + 1.0;
    int ex;
    frexp(xmax, &ex);
    ex = ex > 31 ? ex - 31 : 0;
    return ldexp(1.0, -ex);
}

__global__ __launch_bounds__(256) void adj32_prep_kernel(const AdjArgs A) {
    const int g = blockIdx.x * 256 + threadIdx.x;
    if (g >= A.n_lines) return;
    const Geometry G = A.G;
    const Tables* tab = A.tab;
    const LineSetup ls = line_setup(A.L, A.tp, g, A.Q[0]);
    const double s = kSQRT_LN2 / ls.aD;
    const double y = ls.gam * s, y2 = y * y;
    const double d = (G.nu_a + (double)ls.kc * G.dnu) - ls.nu;
    const double sc = wing_scale(s, G), sc2 = sc * sc;
    float f[kAdjRec];
    int* fi = reinterpret_cast<int*>(f);
#pragma unroll
    for (int i = 0; i < kAdjRec; ++i) f[i] = 0.0f;
    f[J_HS] = (float)(s * G.dnu * sc);
    f[J_XCS] = (float)(s * d * sc);
    f[J_YS2] = (float)(y2 * sc2);
    f[J_Z1S] = (float)(kMidR2 * sc2);
    {
        const double t2 = tab->gh2.t[0] * tab->gh2.t[0];
        f[J_A2] = (float)((y2 - t2) * sc2);
        f[J_B2] = (float)(2.0 * t2 * sc2);
        f[J_E2] = (float)(4.0 * t2 * y2 * sc2 * sc2);
        f[J_C2] = (float)(2.0 * tab->gh2.w[0]);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const double t2 = tab->gh4.t[j] * tab->gh4.t[j];
        f[J_A4 + j] = (float)((y2 - t2) * sc2);
        f[J_B4 + j] = (float)(2.0 * t2 * sc2);
        f[J_E4 + j] = (float)(4.0 * t2 * y2 * sc2 * sc2);
        f[J_C4 + j] = (float)(2.0 * tab->gh4.w[j]);
    }
    int kcl = 0, kch = -1;
    if (y2 < kCoreR2) {
        const int r = radius_steps(sqrt(kCoreR2 - y2), s * G.dnu, s * d);
        const int64_t lo = (int64_t)ls.kc - r, hi = (int64_t)ls.kc + r;
        kcl = (int)(lo > ls.klo ? lo : ls.klo);
        kch = (int)(hi < ls.khi ? hi : ls.khi);
    }
    // points beyond rad steps from kc have |z| >= 40 (the 2-node rule's zone)
    fi[J_RAD] = y2 < kMidR2 ? radius_steps(sqrt(kMidR2 - y2), s * G.dnu, s * d) : -1;
    fi[J_KLO] = ls.klo;
    fi[J_KHI] = ls.khi;
    fi[J_KC] = ls.kc;
    fi[J_KCL] = kcl;
    fi[J_KCH] = kch;
    float4* ro = reinterpret_cast<float4*>(A.rec + (int64_t)g * kAdjRec);
#pragma unroll
    for (int q = 0; q < kAdjRec / 4; ++q) ro[q] = make_float4(f[4 * q], f[4 * q + 1], f[4 * q + 2], f[4 * q + 3]);
    // core points in double precision
    const float* gbar = static_cast<const float*>(A.gbar);
    double c0 = 0.0, cx = 0.0, cy = 0.0;
    for (int k = kcl; k <= kch; ++k) {
        const double x = s * ((G.nu_a + (double)k * G.dnu) - ls.nu);
        const double u = x * x, z2 = u + y2;
        double v, xvx, vy;
        if (z2 < kCoreR2) {
            double rw, rdw, idw;
            voigt_core_dw<24, 8>(x, y, tab->w24, &rw, &rdw, &idw);
            v = rw; xvx = x * rdw; vy = -idw;
        } else if (z2 < kMidR2) {
            gh_wing_dv(u, y, tab->gh4, &v, &xvx, &vy);
        } else {
            gh_wing_dv(u, y, tab->gh2, &v, &xvx, &vy);
        }
        const double gb = (double)gbar[k];
        c0 = __builtin_fma(gb, v, c0);
        cx = __builtin_fma(gb, xvx, cx);
        cy = __builtin_fma(gb, vy, cy);
    }
    double* sm = A.sums + (int64_t)g * 6;
    sm[0] = c0;
    sm[1] = cx;
    sm[2] = cy;
}

// Window sums over the points kA..kB of one line (lanes over consecutive points, partials
// in single precision over 8 passes of 64 points, then folded into double).  TWO: the
// 2-node rule (one node pair) written out, with its weight c applied per fold; otherwise
// the 4-node rule through wing_dv_f32.
template <bool TWO>
__device__ __forceinline__ void adj_run(int kA, int kB, int kc, int lane, const float* __restrict__ gbar, float hs,
                                        float xcs, float ys2, const float* a, const float* b, const float* e,
                                        const float* c, double* s0, double* sx, double* sy) {
    if (kB < kA) return;
    const int niter = (kB - kA + 64) / 64;
    const float ys2x2 = 2.0f * ys2;
    float jf = (float)(kA + lane - kc);    // exact: |k - kc| < 2^24
    for (int it0 = 0; it0 < niter; it0 += 8) {
        const int ite = it0 + 8 < niter ? it0 + 8 : niter;
        float p0 = 0.0f, px = 0.0f, py = 0.0f;
        for (int it = it0; it < ite; ++it) {
            const int k = kA + 64 * it + lane;
            const float gb = k <= kB ? gbar[k] : 0.0f;
            const float xsv = __builtin_fmaf(jf, hs, xcs);
            jf += 64.0f;
            if constexpr (TWO) {
                // p = x^2 + a, q = p + b, r = 1/(p^2 + e): V ~ q r, x dV/dx ~ x^2 r (1 - 2 p q r),
                // dV/dy ~ q r + 2 y^2 r (1 - 2 q q r)
                const float u = xsv * xsv;
                const float pp = u + a[0];
                const float q = pp + b[0];
                const float r = __builtin_amdgcn_rcpf(__builtin_fmaf(pp, pp, e[0]));
                const float qr = q * r;
                const float m2 = -2.0f * qr;
                p0 = __builtin_fmaf(gb, qr, p0);
                px = __builtin_fmaf(gb * (u * r), __builtin_fmaf(pp, m2, 1.0f), px);
                py = __builtin_fmaf(gb, __builtin_fmaf(ys2x2, r * __builtin_fmaf(q, m2, 1.0f), qr), py);
            } else {
                float sv, ssx, ssy;
                wing_dv_f32<2>(xsv, a, b, e, c, ys2, &sv, &ssx, &ssy);
                p0 = __builtin_fmaf(gb, sv, p0);
                px = __builtin_fmaf(gb, ssx, px);
                py = __builtin_fmaf(gb, ssy, py);
            }
        }
        const double w = TWO ? (double)c[0] : 1.0;
        *s0 += w * (double)p0;
        *sx += w * (double)px;
        *sy += w * (double)py;
    }
}

__global__ __launch_bounds__(256) void adj32_wing_kernel(const AdjArgs A) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int nwaves = gridDim.x * 4;
    const float* gbar = static_cast<const float*>(A.gbar);
    for (int g = blockIdx.x * 4 + wave; g < A.n_lines; g += nwaves) {
        const float* r = A.rec + (int64_t)g * kAdjRec;
        const int* ri = reinterpret_cast<const int*>(r);
        const float hs = r[J_HS], xcs = r[J_XCS], ys2 = r[J_YS2];
        const float a2[1] = {r[J_A2]}, b2[1] = {r[J_B2]}, e2[1] = {r[J_E2]}, c2[1] = {r[J_C2]};
        const float a4[2] = {r[J_A4], r[J_A4 + 1]}, b4[2] = {r[J_B4], r[J_B4 + 1]};
        const float e4[2] = {r[J_E4], r[J_E4 + 1]}, c4[2] = {r[J_C4], r[J_C4 + 1]};
        const int klo = __builtin_amdgcn_readfirstlane(ri[J_KLO]);
        const int khi = __builtin_amdgcn_readfirstlane(ri[J_KHI]);
        const int kc = __builtin_amdgcn_readfirstlane(ri[J_KC]);
        const int kcl = __builtin_amdgcn_readfirstlane(ri[J_KCL]);
        const int kch = __builtin_amdgcn_readfirstlane(ri[J_KCH]);
        const int rad = __builtin_amdgcn_readfirstlane(ri[J_RAD]);
        double s0 = 0.0, sxa = 0.0, sya = 0.0;
        if (rad < 0) {
            adj_run<true>(klo, khi, kc, lane, gbar, hs, xcs, ys2, a2, b2, e2, c2, &s0, &sxa, &sya);
        } else {
            // [klo, kml) and (kmh, khi]: 2-node; [kml, kmh] without the core [kcl, kch]: 4-node
            // (the core lies inside: its radius is that of |z| < 8)
            const int64_t ml = (int64_t)kc - rad, mh = (int64_t)kc + rad;
            const int kml = (int)(ml > klo ? ml : klo), kmh = (int)(mh < khi ? mh : khi);
            adj_run<true>(klo, (kml - 1 < khi ? kml - 1 : khi), kc, lane, gbar, hs, xcs, ys2, a2, b2, e2, c2, &s0,
                          &sxa, &sya);
            if (kcl > kch) {
                adj_run<false>(kml, kmh, kc, lane, gbar, hs, xcs, ys2, a4, b4, e4, c4, &s0, &sxa, &sya);
            } else {
                adj_run<false>(kml, (kcl - 1 < kmh ? kcl - 1 : kmh), kc, lane, gbar, hs, xcs, ys2, a4, b4, e4, c4,
                               &s0, &sxa, &sya);
                adj_run<false>((kch + 1 > kml ? kch + 1 : kml), kmh, kc, lane, gbar, hs, xcs, ys2, a4, b4, e4, c4,
                               &s0, &sxa, &sya);
            }
            adj_run<true>((kmh + 1 > klo ? kmh + 1 : klo), khi, kc, lane, gbar, hs, xcs, ys2, a2, b2, e2, c2, &s0,
                          &sxa, &sya);
        }
        s0 = wave_sum64(s0);
        sxa = wave_sum64(sxa);
        sya = wave_sum64(sya);
        if (lane == 0) {
            double* sm = A.sums + (int64_t)g * 6;
            sm[3] = s0;
            sm[4] = sxa;
            sm[5] = sya;
        }
    }
}

__global__ __launch_bounds__(256) void adj32_final_kernel(const AdjArgs A) {
    const int g = blockIdx.x * 256 + threadIdx.x;
    if (g >= A.n_lines) return;
    const double T = A.tp.T;
    const double Q = A.Q[0], dQ = A.dQ[0];
    const LineSetup ls = line_setup(A.L, A.tp, g, Q);
    const double s = kSQRT_LN2 / ls.aD;
    const double y = ls.gam * s;
    const double Nn = kSQRT_LN2_PI / ls.aD;
    const double sc = wing_scale(s, A.G), sc2 = sc * sc;
    const double* sm = A.sums + (int64_t)g * 6;
    // scaled sums carry a factor c^2 = 1/sc^2 (x_s = x sc): V = (y sc^2/pi) sum c q_s r_s, ...
    const double kv = y * sc2 / kPI, ky = sc2 / kPI;
    const double A0 = kv * sm[3] + sm[0];
    const double Ax = 2.0 * kv * sm[4] + sm[1];
    const double Ay = ky * sm[5] + sm[2];
    const double R0 = Nn * A0;
    const double Rg = Nn * s * Ay;
    const double Ra = -(Nn / ls.aD) * (A0 + Ax + y * Ay);
    const double S = ls.S;
    const double gref = (double)A.L.gref[g];
    const double nexp = (double)A.L.nexp[g];
    const int o = A.L.orig[g];
    // double outputs: a loss on cross sections of ~1e-20 cm^2 has per-line gradients far
    // below the float range (stored as float they would lose their digits as subnormals)
    if (A.dlnA) static_cast<double*>(A.dlnA)[o] = S * R0;
    if (A.dgref) static_cast<double*>(A.dgref)[o] = gref > 0.0 ? S * Rg * ls.gam / gref : 0.0;
    if (A.dn) static_cast<double*>(A.dn)[o] = S * Rg * ls.gam * A.tp.ln_T0_T;
    const double x2 = (kC2 * ls.nu) / T;
    const double tau = (kC2 * A.L.elow[g]) / (T * T) - ((kC2 * ls.nu) / (T * T)) / expm1(x2) - dQ / Q;
    A.pT[g] = S * (tau * R0 + Ra * ls.aD / (2.0 * T) - Rg * nexp * ls.gam / T);
    const double dgam_dP = A.tp.P > 0.0 ? ls.gam / A.tp.P : gref * exp(nexp * A.tp.ln_T0_T) / A.P0;
    A.pP[g] = S * Rg * dgam_dP;
}

template <class R>
__global__ __launch_bounds__(256) void fill_zero_kernel(void* a, void* b, void* c, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    if (a) static_cast<R*>(a)[i] = R(0);
    if (b) static_cast<R*>(b)[i] = R(0);
    if (c) static_cast<R*>(c)[i] = R(0);
}

// fixed-order sum of two double arrays: 256 blocks x 256 threads of strided partials,
// then one block over the 256 partials
__global__ __launch_bounds__(256) void sum2_partial_kernel(const double* a, const double* b, int64_t n,
                                                           double* part) {
    __shared__ double la[4], lb[4];
    double sa = 0.0, sb = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        sa += a[i];
        sb += b[i];
    }
    sa = wave_sum64(sa);
    sb = wave_sum64(sb);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) { la[wave] = sa; lb[wave] = sb; }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[blockIdx.x] = (la[0] + la[1]) + (la[2] + la[3]);
        part[gridDim.x + blockIdx.x] = (lb[0] + lb[1]) + (lb[2] + lb[3]);
    }
}

__global__ __launch_bounds__(256) void sum2_final_kernel(const double* part, int nb, double* outa, double* outb) {
    __shared__ double la[4], lb[4];
    double sa = 0.0, sb = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) { sa += part[i]; sb += part[nb + i]; }
    sa = wave_sum64(sa);
    sb = wave_sum64(sb);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) { la[wave] = sa; lb[wave] = sb; }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (outa) *outa = (la[0] + la[1]) + (la[2] + la[3]);
        if (outb) *outb = (lb[0] + lb[1]) + (lb[2] + lb[3]);
    }
}

}  // namespace

hipError_t launch_adjoint(const AdjArgs& a, int fp64, int64_t n_caller_lines, double* part, double* dT,
                          double* dP, hipStream_t s) {
    if (n_caller_lines > 0) {
        const dim3 g((unsigned)((n_caller_lines + 255) / 256));
        hipLaunchKernelGGL(fill_zero_kernel<double>, g, dim3(256), 0, s, a.dlnA, a.dgref, a.dn, n_caller_lines);
    }
    if (a.n_lines > 0) {
        const int blocks = 2048;
        if (fp64) {
            hipLaunchKernelGGL(adjoint64_kernel, dim3(blocks), dim3(256), 0, s, a);
        } else {
            const dim3 gl((unsigned)((a.n_lines + 255) / 256));
            hipLaunchKernelGGL(adj32_prep_kernel, gl, dim3(256), 0, s, a);
            hipLaunchKernelGGL(adj32_wing_kernel, dim3(4096), dim3(256), 0, s, a);
            hipLaunchKernelGGL(adj32_final_kernel, gl, dim3(256), 0, s, a);
        }
    }
    hipLaunchKernelGGL(sum2_partial_kernel, dim3(256), dim3(256), 0, s, a.pT, a.pP, (int64_t)a.n_lines, part);
    hipLaunchKernelGGL(sum2_final_kernel, dim3(1), dim3(256), 0, s, part, 256, dT, dP);
    return hipGetLastError();
}

}  // namespace xs
