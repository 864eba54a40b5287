// FP64 forward tile kernel: the plain double-precision path (profiles, wings and
// sums all in double).  Same tile ownership and sorted-line ranges as the FP32
// kernel; every line carries per-slice codes (skip / zone / window mask), and the
// Voigt zones use Gauss-Hermite rules of 2, 4, 6 and 12 nodes for |z| >= 2200, 60,
// 20 and 8, and the Weideman/Taylor core (40 terms / 14 terms) inside |z| < 8.
// Vectorized Voigt: the same Voigt inside the radius R; beyond it beta times the reference
// profile (Doppler width of a line at 1 cm^-1), evaluated with the 2-node rule in the
// reference's own variables (relative error 1/(2 |z_ref|^4), |z_ref| >= 2e4).
#include "xs_forward_common.hpp"

namespace xs {

namespace {

constexpr int kRec = 32;
constexpr int kBatch = 256;
enum : int { D_NU = 0, D_S = 1, D_Y = 2, D_A = 3, D_CODE = 4, D_KLIM = 5, D_AD = 6, D_W = 7, D_SR = 8, D_KV = 9 };

// Re w from the plain path's zones, chosen per lane (slices that touch |z| < 8).
__device__ __forceinline__ double re_w_zones(double x, double y, const Tables* tab) {
    const double u = x * x;
    const double z2 = u + y * y;
    if (z2 < 64.0) return voigt_core_re<40, 14>(x, y, tab->w40);
    if (z2 < 400.0) return gh_wing_re(u, y, tab->gh12);
    if (z2 < 3600.0) return gh_wing_re(u, y, tab->gh6);
    if (z2 < 4.84e6) return gh_wing_re(u, y, tab->gh4);
    return gh_wing_re(u, y, tab->gh2);
}

// ============================================================== FP64 path
template <int PROF, int P>
__global__ __launch_bounds__(256) void fwd_f64_kernel(const FwdArgs A) {
    constexpr int W = 256 * P;
    constexpr int NS = 4 * P;
    __shared__ double rec[kBatch * (kRec / 2)];

    const Geometry G = A.G;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const WorkItem wi = work_item(A);
    const TPParam tp = A.tps[wi.tp];
    const int t0 = wi.tile * W, t1 = t0 + W - 1;
    // intensity threshold: this (T, P)'s kept lines and offsets table
    const int* map = A.map ? A.map + (int64_t)wi.tp * A.map_stride : nullptr;
    const int* off = A.offs ? A.offs + (int64_t)wi.tp * A.offs_stride : A.off;
    // lines overlapping the tile; this workgroup takes every n_split-th batch of them
    const int b0 = off_at(off, (int64_t)t0 - G.hmax, G);
    const int b5 = off_at(off, (int64_t)t1 + G.hmax + 1, G);
    const double Q = A.Q[tp.iq];

    int kk[P];
    double nuk[P], acc[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        kk[p] = t0 + 64 * (wave * P + p) + lane;
        nuk[p] = G.nu_a + (double)kk[p] * G.dnu;
        acc[p] = 0.0;
    }
    const int cshift = 4 * (wave * P);   // NS <= 16 slices, 64-bit code

    for (int bs = b0 + kBatch * wi.part; bs < b5; bs += kBatch * A.n_split) {
        const int g = bs + tid;
        if (g < b5) {
            double* r = rec + tid * (kRec / 2);
            const int gs = line_of(map, g);
            const LineSetup ls = line_setup(A.L, tp, gs, Q);
            double s, y = 0.0;
            r[D_NU] = ls.nu;
            if (PROF == kVoigt || PROF == kVVoigt) {
                s = kSQRT_LN2 / ls.aD;
                y = ls.gam * s;
                r[D_A] = ls.S * kSQRT_LN2_PI / ls.aD;
                if (PROF == kVVoigt) {
                    const double2 vv = A.vv ? A.vv[(int64_t)wi.tp * A.vv_stride + gs] : make_double2(1.0, 1.0);
                    const double sr = kSQRT_LN2 / tp.beta;   // reference: alpha_D of a line at 1 cm^-1
                    r[D_A] *= vv.y;
                    r[D_W] = vv.x * vv.y * ls.S * kSQRT_LN2_PI / tp.beta;
                    r[D_SR] = sr;
                    r[D_AD] = sr * ls.gam;
                    const double kvl = ceil((ls.nu - G.vv_radius - G.nu_a) / G.dnu);
                    const double kvh = floor((ls.nu + G.vv_radius - G.nu_a) / G.dnu);
                    int* kv = reinterpret_cast<int*>(r + D_KV);
                    kv[0] = (int)fmin(fmax(kvl, -1.0), (double)G.n_points);
                    kv[1] = (int)fmin(fmax(kvh, -1.0), (double)G.n_points);
                }
            } else if (PROF == kLorentz) {
                s = ls.gam > 0.0 ? 1.0 / ls.gam : 0.0;
                r[D_A] = ls.S * s * (1.0 / kPI);
            } else if (PROF == kLorentzBinned) {
                // bin average of Eq. 17 in wavenumber units (x = D, y = gamma)
                s = 1.0;
                y = ls.gam;
                r[D_A] = ls.S / (kPI * G.dnu);
            } else if (PROF == kDopplerBinned) {
                // bin average of Eq. 15 with the Doppler HWHM
                s = kSQRT_LN2 / ls.aD;
                r[D_A] = ls.S / (2.0 * G.dnu);
            } else if (PROF == kGHSampled || PROF == kGHBinned) {
                // Gauss-Hermite convolution in wavenumber units (x = D, y = gamma)
                s = 1.0;
                y = ls.gam;
                r[D_AD] = ls.aD / kSQRT_LN2;
                r[D_A] = (PROF == kGHSampled) ? ls.S * ls.gam / (kPI * 1.7724538509055160273)
                                              : ls.S / (kPI * 1.7724538509055160273 * G.dnu);
            } else {
                const double alpha = (PROF == kDoppler) ? ls.aD : A.alpha_fixed;
                s = kSQRT_LN2 / alpha;
                r[D_A] = ls.S * kSQRT_LN2_PI / alpha;
            }
            r[D_S] = s;
            r[D_Y] = y;
            int* kl = reinterpret_cast<int*>(r + D_KLIM);
            kl[0] = ls.klo;
            kl[1] = ls.khi;
            unsigned long long code = 0;
#pragma unroll
            for (int sl = 0; sl < NS; ++sl) {
                const int kA = t0 + 64 * sl, kB = kA + 63;
                unsigned long long c = 0;
                if (!(kB < ls.klo || kA > ls.khi)) {
                    const bool full = (kA >= ls.klo && kB <= ls.khi);
                    const double mx = min_abs_delta(G, kA, kB, ls.nu) * s;
                    unsigned zone = 1;
                    if (PROF == kVoigt || PROF == kVVoigt) {
                        const double z2 = mx * mx + y * y;
                        zone = z2 < 64.0 * 1.0001 ? 5u : z2 < 400.0 * 1.0001 ? 4u
                             : z2 < 3600.0 * 1.0001 ? 3u : z2 < 4.84e6 * 1.0001 ? 2u : 1u;
                        if (PROF == kVVoigt) {
                            // 7: every point beyond R; 6: R falls inside the slice
                            const int* kv = reinterpret_cast<const int*>(r + D_KV);
                            if (kB < kv[0] || kA > kv[1]) zone = 7u;
                            else if (!(kA >= kv[0] && kB <= kv[1])) zone = 6u;
                        }
                    } else if (PROF == kLorentz || PROF == kGHSampled) {
                        zone = ls.gam > 0.0 ? 1u : 0u;
                    } else if (PROF == kGHBinned || PROF == kLorentzBinned) {
                        zone = 1u;
                    } else if (PROF == kDopplerBinned) {
                        const double e = mx - 0.5 * s * G.dnu;   // nearest bin edge, scaled
                        zone = (e < 0.0 || e * e < 745.0) ? 1u : 0u;
                    } else {
                        zone = (mx * mx < 745.0) ? 1u : 0u;   // exp(-x^2) underflows beyond
                    }
                    c = zone ? (zone | (full ? 0u : 8u)) : 0u;
                }
                code |= c << (4 * sl);
            }
            reinterpret_cast<unsigned long long*>(r)[D_CODE] = code;
        }
        __syncthreads();
        const int be = bs + kBatch < b5 ? bs + kBatch : b5;
        for (int l = bs; l < be; ++l) {
            const double* r = rec + (l - bs) * (kRec / 2);
            const unsigned long long code64 = reinterpret_cast<const unsigned long long*>(r)[D_CODE];
            const unsigned lo32 = __builtin_amdgcn_readfirstlane((unsigned)code64);
            const unsigned hi32 = __builtin_amdgcn_readfirstlane((unsigned)(code64 >> 32));
            const unsigned long long cw = (((unsigned long long)hi32 << 32) | lo32) >> cshift;
            if ((cw & ((1ull << (4 * P)) - 1ull)) == 0ull) continue;
            const double nu = r[D_NU], s = r[D_S], y = r[D_Y], a = r[D_A];
            const int* kl = reinterpret_cast<const int*>(r + D_KLIM);
            const int klo = kl[0], khi = kl[1];
            const int* kv = reinterpret_cast<const int*>(r + D_KV);
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const unsigned z = (unsigned)(cw >> (4 * p)) & 15u;
                const unsigned zone = z & 7u;
                if (zone == 0u) continue;
                const double x = s * (nuk[p] - nu);
                double v;
                if (PROF == kVVoigt && zone >= 6u) {
                    // beta f_ref beyond R (2-node rule in the reference's variables)
                    const double xr = r[D_SR] * (nuk[p] - nu);
                    const double vw = r[D_W] * gh_wing_re(xr * xr, r[D_AD], A.tab->gh2);
                    if (zone == 7u) {
                        v = vw;
                    } else {
                        const bool inr = kk[p] >= kv[0] && kk[p] <= kv[1];
                        double vc = 0.0;
                        if (inr) vc = a * re_w_zones(x, y, A.tab);
                        v = inr ? vc : vw;
                    }
                } else if (PROF == kVoigt || PROF == kVVoigt) {
                    const double u = x * x;
                    if (zone == 1u) v = gh_wing_re(u, y, A.tab->gh2);
                    else if (zone == 2u) v = gh_wing_re(u, y, A.tab->gh4);
                    else if (zone == 3u) v = gh_wing_re(u, y, A.tab->gh6);
                    else if (zone == 4u) v = gh_wing_re(u, y, A.tab->gh12);
                    else {
                        // slice touches |z| < 8: each lane takes the formula of its own zone
                        const double z2 = u + y * y;
                        if (z2 < 64.0) v = voigt_core_re<40, 14>(x, y, A.tab->w40);
                        else if (z2 < 400.0) v = gh_wing_re(u, y, A.tab->gh12);
                        else if (z2 < 3600.0) v = gh_wing_re(u, y, A.tab->gh6);
                        else if (z2 < 4.84e6) v = gh_wing_re(u, y, A.tab->gh4);
                        else v = gh_wing_re(u, y, A.tab->gh2);
                    }
                    v *= a;
                } else if (PROF == kLorentz) {
                    v = a * rcp64(__builtin_fma(x, x, 1.0));
                } else if (PROF == kGHSampled) {
                    // node pairs: L(D - dj) + L(D + dj) ~ 2 (D^2 + g^2 + dj^2) / ((D^2 + g^2 - dj^2)^2 + 4 dj^2 g^2)
                    const double ad = r[D_AD], g2 = y * y;
                    const double D2 = __builtin_fma(x, x, g2);
                    double accg = 0.0;
                    for (int q = 0; q < A.tab->npair; ++q) {
                        const double dj = ad * A.tab->tpair[q];
                        const double d2 = dj * dj;
                        const double pq = D2 - d2;
                        accg = __builtin_fma(2.0 * A.tab->wpair[q] * (D2 + d2),
                                             rcp64(__builtin_fma(pq, pq, 4.0 * g2 * d2)), accg);
                    }
                    v = a * accg;
                } else if (PROF == kGHBinned) {
                    // atan(y+) - atan(y-) = atan2(dnu g, (D - dj)^2 + g^2 - dnu^2/4)
                    const double ad = r[D_AD];
                    const double hg = G.dnu * y, c = y * y - 0.25 * G.dnu * G.dnu;
                    double accg = 0.0;
                    for (int q = 0; q < A.tab->nconv; ++q) {
                        const double e = x - ad * A.tab->tconv[q];
                        accg = __builtin_fma(A.tab->wconv[q], atan2(hg, __builtin_fma(e, e, c)), accg);
                    }
                    v = a * accg;
                } else if (PROF == kLorentzBinned) {
                    // atan(y+) - atan(y-) = atan2(dnu gamma, (D - dnu/2)(D + dnu/2) + gamma^2)
                    v = a * atan2(G.dnu * y, __builtin_fma(x - 0.5 * G.dnu, x + 0.5 * G.dnu, y * y));
                } else if (PROF == kDopplerBinned) {
                    const double hs = 0.5 * s * G.dnu;
                    v = a * erf_diff64(x - hs, x + hs);
                } else {
                    v = a * exp(-x * x);
                }
                if (z & 8u) v = (kk[p] >= klo && kk[p] <= khi) ? v : 0.0;
                acc[p] += v;
            }
        }
        __syncthreads();
    }
    double* out = A.n_split == 1
                      ? static_cast<double*>(A.sigma) + (int64_t)wi.tp * G.n_points
                      : static_cast<double*>(A.part) + ((int64_t)wi.tp * A.n_split + wi.part) * G.n_points;
#pragma unroll
    for (int p = 0; p < P; ++p)
        if (kk[p] < G.n_points) out[kk[p]] = acc[p];
}

template <int PROF>
void launch_p64(int P, const FwdArgs& a, hipStream_t s) {
    const dim3 grid((unsigned)((int64_t)a.n_tiles * a.n_tp * a.n_split)), block(256);
    switch (P) {
        case 1: hipLaunchKernelGGL((fwd_f64_kernel<PROF, 1>), grid, block, 0, s, a); break;
        case 2: hipLaunchKernelGGL((fwd_f64_kernel<PROF, 2>), grid, block, 0, s, a); break;
        default: hipLaunchKernelGGL((fwd_f64_kernel<PROF, 4>), grid, block, 0, s, a); break;
    }
}

}  // namespace

hipError_t launch_forward_f32(int profile, int waves, int P, const FwdArgs& a, hipStream_t s);

namespace {

// Sum of the n_split partial results of every (T, P) and grid point, in part order.
// FP32: TwoSum of the parts' sums, plus their compensations.
__global__ __launch_bounds__(256) void combine_f32_kernel(const float2* part, float* sigma, int n_split,
                                                          int n_points, int64_t total) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= total) return;
    const int64_t t = i / n_points, k = i - t * n_points;
    const float2* p = part + t * n_split * (int64_t)n_points + k;
    float s = 0.0f, c = 0.0f;
    for (int q = 0; q < n_split; ++q) {
        const float2 v = p[(int64_t)q * n_points];
        const float u = s + v.x;
        const float bp = u - s;
        c += (s - (u - bp)) + (v.x - bp);
        c += v.y;
        s = u;
    }
    sigma[i] = s + c;
}

// The same with the node-sampled sums (far_kernel's shares and ends_kernel's slot): (parts'
// compensated sum, or sigma as the tile kernel wrote it when n_split = 1) + the FP64 sum
// over the slots, rounded once.
__global__ __launch_bounds__(256) void combine_far_kernel(const float2* part, const double* far, float* sigma,
                                                          int n_split, int far_slots, int n_points, int64_t total) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= total) return;
    const int64_t t = i / n_points, k = i - t * n_points;
    double base;
    if (n_split > 1) {
        const float2* p = part + t * n_split * (int64_t)n_points + k;
        float s = 0.0f, c = 0.0f;
        for (int q = 0; q < n_split; ++q) {
            const float2 v = p[(int64_t)q * n_points];
            const float u = s + v.x;
            const float bp = u - s;
            c += (s - (u - bp)) + (v.x - bp);
            c += v.y;
            s = u;
        }
        base = (double)s + (double)c;
    } else {
        base = (double)sigma[i];
    }
    const double* f = far + t * far_slots * (int64_t)n_points + k;
    double fs = 0.0;
    for (int q = 0; q < far_slots; ++q) fs += f[(int64_t)q * n_points];
    sigma[i] = (float)(base + fs);
}

__global__ __launch_bounds__(256) void combine_f64_kernel(const double* part, double* sigma, int n_split,
                                                          int n_points, int64_t total) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= total) return;
    const int64_t t = i / n_points, k = i - t * n_points;
    const double* p = part + t * n_split * (int64_t)n_points + k;
    double s = 0.0;
    for (int q = 0; q < n_split; ++q) s += p[(int64_t)q * n_points];
    sigma[i] = s;
}

}  // namespace

hipError_t launch_combine(int fp64, const FwdArgs& a, hipStream_t s) {
    const bool far = !fp64 && a.far && a.seg;
    if (a.n_split <= 1 && !far) return hipSuccess;
    const int64_t total = (int64_t)a.n_tp * a.G.n_points;
    if (total == 0) return hipSuccess;
    const dim3 grid((unsigned)((total + 255) / 256)), block(256);
    if (far)
        hipLaunchKernelGGL(combine_far_kernel, grid, block, 0, s, static_cast<const float2*>(a.part), a.far,
                           static_cast<float*>(a.sigma), a.n_split, a.far_slots, a.G.n_points, total);
    else if (fp64)
        hipLaunchKernelGGL(combine_f64_kernel, grid, block, 0, s, static_cast<const double*>(a.part),
                           static_cast<double*>(a.sigma), a.n_split, a.G.n_points, total);
    else
        hipLaunchKernelGGL(combine_f32_kernel, grid, block, 0, s, static_cast<const float2*>(a.part),
                           static_cast<float*>(a.sigma), a.n_split, a.G.n_points, total);
    return hipGetLastError();
}

hipError_t launch_forward(int profile, int fp64, int waves, int P, const FwdArgs& a, hipStream_t s) {
    if (a.n_tiles <= 0) return hipSuccess;
    if (profile == kSuperLines) return launch_superlines(fp64, a, s);
    if (!fp64) return launch_forward_f32(profile, waves, P, a, s);
    switch (profile) {
        case kDoppler: launch_p64<kDoppler>(P, a, s); break;
        case kGaussFixed: launch_p64<kGaussFixed>(P, a, s); break;
        case kLorentz: launch_p64<kLorentz>(P, a, s); break;
        case kGHSampled: launch_p64<kGHSampled>(P, a, s); break;
        case kGHBinned: launch_p64<kGHBinned>(P, a, s); break;
        case kVVoigt: launch_p64<kVVoigt>(P, a, s); break;
        case kDopplerBinned: launch_p64<kDopplerBinned>(P, a, s); break;
        case kLorentzBinned: launch_p64<kLorentzBinned>(P, a, s); break;
        default: launch_p64<kVoigt>(P, a, s); break;
    }
    return hipGetLastError();
}

namespace {

// Sec. "Super-lines": per grid point k, the intensities (Eq. 1) of the lines whose nearest
// grid index is k (the sorted lines of key k, in their sorted order) summed in double,
// divided by dnu.  Two passes: every line's intensity (one thread per line, coalesced),
// then per grid point the sum of its contiguous run of lines in sorted order.
__global__ __launch_bounds__(256) void superline_S_kernel(const FwdArgs A) {
    const Geometry G = A.G;
    const int t = blockIdx.y;
    const int l = blockIdx.x * 256 + threadIdx.x;
    const int* off = A.offs ? A.offs + (int64_t)t * A.offs_stride : A.off;
    if (l >= off[G.nkeys]) return;   // the lines of this (T, P) in sorted order
    const int* map = A.map ? A.map + (int64_t)t * A.map_stride : nullptr;
    const TPParam tp = A.tps[t];
    const int gs = line_of(map, l);
    A.line_S[(int64_t)t * A.line_S_stride + l] =
        line_intensity(A.L, gs, A.L.elow[gs], A.L.nu[gs], tp, A.Q[tp.iq]);   // Eq. 1 (or emissivity)
}

__global__ __launch_bounds__(256) void superline_kernel(const FwdArgs A, int fp64) {
    const Geometry G = A.G;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t total = (int64_t)A.n_tp * G.n_points;
    if (i >= total) return;
    const int t = (int)(i / G.n_points);
    const int k = (int)(i - (int64_t)t * G.n_points);
    const int* off = A.offs ? A.offs + (int64_t)t * A.offs_stride : A.off;
    const int l0 = off_at(off, k, G), l1 = off_at(off, (int64_t)k + 1, G);
    const double* S = A.line_S + (int64_t)t * A.line_S_stride;
    double acc = 0.0;
    for (int l = l0; l < l1; ++l) acc += S[l];
    const double v = acc / G.dnu;
    if (fp64) static_cast<double*>(A.sigma)[i] = v;
    else static_cast<float*>(A.sigma)[i] = (float)v;
}

}  // namespace

hipError_t launch_superlines(int fp64, const FwdArgs& a, hipStream_t s) {
    const int64_t total = (int64_t)a.n_tp * a.G.n_points;
    if (total == 0) return hipSuccess;
    if (a.n_lines > 0)
        hipLaunchKernelGGL(superline_S_kernel, dim3((unsigned)((a.n_lines + 255) / 256), (unsigned)a.n_tp), dim3(256),
                           0, s, a);
    hipLaunchKernelGGL(superline_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a, fp64);
    return hipGetLastError();
}

}  // namespace xs
