// FP32 forward tile kernel (the hot loop of the sampling method: sigma_k = sum over
// lines of I f(nu_k - nu_fi) within the cut-off; Sec. "Cross sections" Eq. 6-8,
// Sec. "Standard line profiles and sampling method", Sec. "Off-set").
//
// One workgroup (4 wavefronts) owns a tile of 256*P consecutive grid points; each
// wavefront owns P slices of 64 points (one point per lane per slice) with its sums
// in registers, so no atomics touch the output.  Lines are sorted by their nearest
// grid index kc; the lines overlapping a range of grid points are a contiguous index
// range read from the offsets table.  The workgroup walks its tile's line range in
// batches of 256:
//   1. each thread prepares one line in double precision (intensity Eq. 1 with Q(T)
//      from the device, Doppler width Eq. 16, Lorentz width Eq. 18, offset of the
//      centre from its anchor grid point) into an LDS record of f32 coefficients;
//   2. each wavefront sweeps the batch, reading records by broadcast.
//
// Segmented sweep (grids fine enough that 64P + r_mid < the half window): every
// wavefront splits the sorted lines by kc into five contiguous runs relative to its
// own points [w0, w1]:
//   [w0 - hmax, w1 - hmin)  window ends inside the wave:   wing formula + upper mask
//   [w1 - hmin, w0 - rm)    covers the wave, wings only:   wing formula, no branches
//   [w0 - rm,   w1 + rm]    centre near the wave:          per-slice zone (scalar branch)
// (rm: radius beyond which every point of the wave is in the far zone, from the largest
// Doppler width a line of the centre-near run can have, so it shrinks at low wavenumber)
//   (w1 + rm,  w0 + hmin]   covers the wave, wings only:   wing formula, no branches
//   (w0 + hmin, w1 + hmax]  window starts inside the wave: wing formula + lower mask
// Coarse grids use per-slice codes (skip / zone / mask) for every line instead.
//
// Voigt zones (|z| = |x + iy|): wings |z| >= 40 use the 2-node Gauss-Hermite rational
// (6 FMA + 1 reciprocal per point); 8 <= |z| < 40 the 4-node rule; points with |z| < 8
// take the value the double-precision core pre-pass stored for them.
// x is formed as fma(j, h, xc) from the exact integer offset j = k - kc, so its relative
// error stays ~1e-7 however far the point is from the centre.  Partial sums are
// flushed every 64 lines into a compensated (TwoSum) pair.
#include "xs_forward_common.hpp"

namespace xs {

namespace {

constexpr int kRec = 32;     // record size in 4-byte words (128 B); one line per thread

enum : int {
    R_XC = 0, R_H = 1, R_C0 = 2, R_C1 = 3, R_AMP = 4, R_B = 5, R_SB0 = 6, R_CSC = 7,
    R_JLO = 8, R_JHI = 9, R_KCL = 10, R_KCH = 11, R_RAD = 12, R_SB0I = 13,
    R_CBASE = 14,    // int64 (words 14-15): core value index = cbase + k
    R_M = 16,        // 4-node mid zone: cp1, cd1, A1, B1, cp2, cd2, A2, B2
    R_ANC = 24,      // per-wavefront anchor x at the wave end nearest the centre (<= 8 waves)
    R_CODE = 24      // coded sweep: 4-bit per-slice codes (<= 32 slices), shares the anchor words
};

// The caller's line data one thread needs to prepare a line record (prefetched a
// batch ahead so the global loads overlap the sweep).
struct RawLine {
    double nu, elow, cA;
    float gref, nexp;
    int kc, klo, khi, rc;
    long long coff;
};

template <int PROF>
__device__ __forceinline__ RawLine load_raw(const FwdArgs& A, const int* crc, const long long* coff, int g) {
    RawLine w;
    w.nu = A.L.nu[g];
    w.elow = A.L.elow[g];
    w.cA = A.L.cA[g];
    w.gref = A.L.gref[g];
    w.nexp = A.L.nexp[g];
    w.kc = A.L.kc[g];
    w.klo = A.L.klo[g];
    w.khi = A.L.khi[g];
    if (PROF == kVoigt) { w.rc = crc[g]; w.coff = coff[g]; }
    else { w.rc = -1; w.coff = 0; }
    return w;
}

template <int PROF, int WAVES, int P>
__device__ __forceinline__ void prepare_line(const FwdArgs& A, const TPParam& tp, const Geometry& G,
                                             const RawLine& w, double Q, int t0, bool codes, float* r) {
    constexpr int NS = WAVES * P;
    const double T = tp.T;
    // Eq. 1: I = [g_f A/(8 pi c nu^2)] exp(-c2 E_i/T) (1 - exp(-c2 nu/T)) / Q(T)
    const double S = w.cA * exp(-(kC2 * w.elow) / T) * (-expm1(-(kC2 * w.nu) / T)) / Q;
    const double aD = w.nu * tp.beta;                                              // Eq. 16
    const double gam = (double)w.gref * exp((double)w.nexp * tp.ln_T0_T) * tp.p_over_p0;  // Eq. 18
    const double d = (G.nu_a + (double)w.kc * G.dnu) - w.nu;   // anchor offset nu_kc - nu
    int* ri = reinterpret_cast<int*>(r);
    r[R_SB0] = (float)(t0 - w.kc);
    ri[R_SB0I] = t0 - w.kc;
    r[R_JLO] = (float)(w.klo - w.kc);
    r[R_JHI] = (float)(w.khi - w.kc);
    int kcl = 0, kch = -1, rad = -1;
    double hd = 0.0, xd = 0.0;      // double-precision h and xc (scaled), for anchors
    if (PROF == kVoigt) {
        const double s = kSQRT_LN2 / aD;
        const double y = gam * s;
        const double a = S * kSQRT_LN2_PI / aD;
        // power-of-two scaling keeps x^4 inside the float range for very narrow lines
        const double xmax = s * (G.cutoff + 2.0 * G.dnu) + 1.0;
        int e;
        frexp(xmax, &e);
        e = e > 31 ? e - 31 : 0;
        const double sc = ldexp(1.0, -e), sc2 = sc * sc;
        const double y2 = y * y;
        const double ampf = a * y * kINV_SQRT_PI;
        hd = s * G.dnu * sc;
        xd = s * d * sc;
        r[R_XC] = (float)xd;
        r[R_H] = (float)hd;
        r[R_C0] = (float)((y2 - 0.5) * sc2);
        r[R_C1] = (float)(2.0 * y2 * sc2 * sc2);
        r[R_AMP] = (float)(ampf * sc2);
        r[R_B] = (float)(ampf * sc2 * sc2);
        r[R_CSC] = (float)ldexp(1.0, e);
#pragma unroll
        for (int jp = 0; jp < 2; ++jp) {
            const double t2 = A.tab->gh4.t[jp] * A.tab->gh4.t[jp];
            const double Aj = a * (y / kPI) * 2.0 * A.tab->gh4.w[jp];
            r[R_M + 4 * jp + 0] = (float)(y2 - t2);
            r[R_M + 4 * jp + 1] = (float)(4.0 * t2 * y2);
            r[R_M + 4 * jp + 2] = (float)Aj;
            r[R_M + 4 * jp + 3] = (float)(Aj * 2.0 * t2);
        }
        rad = y2 < kMidR2 ? radius_steps(sqrt(kMidR2 - y2), s * G.dnu, s * d) : -1;
        if (w.rc >= 0) {
            const int64_t lo = (int64_t)w.kc - w.rc, hi = (int64_t)w.kc + w.rc;
            kcl = (int)(lo > w.klo ? lo : w.klo);
            kch = (int)(hi < w.khi ? hi : w.khi);
        }
        *reinterpret_cast<long long*>(r + R_CBASE) = w.coff - (long long)kcl;
    } else if (PROF == kLorentz) {
        const double ig = gam > 0.0 ? 1.0 / gam : 0.0;
        hd = G.dnu * ig;
        xd = d * ig;
        r[R_XC] = (float)xd;
        r[R_H] = (float)hd;
        r[R_AMP] = (float)(S * ig * (1.0 / kPI));
    } else if (PROF == kGHSampled || PROF == kGHBinned) {
        // Gauss-Hermite convolution (Eq. 30-31 as read): nodes shift the Lorentzian by
        // delta_j = alpha_D t_j / sqrt(ln 2); work in wavenumber units D = nu_k - nu
        r[R_XC] = (float)d;
        r[R_H] = (float)G.dnu;
        r[R_M + 0] = (float)(gam * gam);
        r[R_M + 1] = (float)(aD / kSQRT_LN2);
        if (PROF == kGHSampled) {
            r[R_AMP] = (float)(S * gam / (kPI * 1.7724538509055160273));   // S gamma / pi^(3/2)
            r[R_M + 2] = (float)(4.0 * gam * gam);
        } else {
            r[R_AMP] = (float)(S / (kPI * 1.7724538509055160273 * G.dnu));   // S / (pi^(3/2) dnu)
            r[R_M + 3] = (float)(G.dnu * gam);
            r[R_M + 4] = (float)(gam * gam - 0.25 * G.dnu * G.dnu);
        }
    } else {
        // Gaussian (Eq. 15); x scaled by sqrt(1/ln 2) so exp(-x^2) = exp2(-x'^2)
        const double alpha = (PROF == kDoppler) ? aD : A.alpha_fixed;
        const double s = kSQRT_LN2 / alpha;
        const double sl = s * 1.2011224087864498;
        r[R_XC] = (float)(sl * d);
        r[R_H] = (float)(sl * G.dnu);
        r[R_AMP] = (float)(S * kSQRT_LN2_PI / alpha);
        rad = radius_steps(10.5, s * G.dnu, s * d);   // exp(-x^2) underflows beyond
    }
    ri[R_KCL] = kcl;
    ri[R_KCH] = kch;
    ri[R_RAD] = rad;
    if (!codes) {
        // x at the end of each wavefront's range nearest the centre: wing points are then
        // x = anchor + (k - k_anchor) h with both terms of one sign
#pragma unroll
        for (int wv = 0; wv < WAVES; ++wv) {
            const int wa = t0 + 64 * P * wv;
            const int ka = wa > w.kc ? wa : wa + 64 * P - 1;
            r[R_ANC + wv] = (float)__builtin_fma((double)(ka - w.kc), hd, xd);
        }
    } else {
        unsigned cw[(NS + 7) / 8];
#pragma unroll
        for (int q = 0; q < (NS + 7) / 8; ++q) cw[q] = 0;
#pragma unroll
        for (int sl = 0; sl < NS; ++sl) {
            const int kA = t0 + 64 * sl, kB = kA + 63;
            unsigned code = 0;
            if (!(kB < w.klo || kA > w.khi)) {
                const bool full = (kA >= w.klo && kB <= w.khi);
                unsigned zone = 1;
                if (PROF == kVoigt) {
                    if (kA <= kch && kB >= kcl) zone = 3;
                    else if (rad >= 0 && (int64_t)kA <= (int64_t)w.kc + rad && (int64_t)kB >= (int64_t)w.kc - rad) zone = 2;
                } else if (PROF == kLorentz || PROF == kGHSampled) {
                    zone = gam > 0.0 ? 1u : 0u;
                } else if (PROF == kGHBinned) {
                    zone = 1u;
                } else {
                    zone = ((int64_t)kA <= (int64_t)w.kc + rad && (int64_t)kB >= (int64_t)w.kc - rad) ? 1u : 0u;
                }
                code = zone ? (zone | (full ? 0u : 4u)) : 0u;
            }
            cw[sl / 8] |= code << (4 * (sl % 8));
        }
#pragma unroll
        for (int q = 0; q < (NS + 7) / 8; ++q) r[R_CODE + q] = __uint_as_float(cw[q]);
    }
}

// wing formula (2-node rule, scaled variables)
__device__ __forceinline__ float v_far(const float* r, float j) {
    const float x = __builtin_fmaf(j, r[R_H], r[R_XC]);
    const float pp = __builtin_fmaf(x, x, r[R_C0]);
    const float den = __builtin_fmaf(pp, pp, r[R_C1]);
    const float num = __builtin_fmaf(pp, r[R_AMP], r[R_B]);
    return num * __builtin_amdgcn_rcpf(den);
}

// 4-node rule (unscaled x)
__device__ __forceinline__ float v_mid(const float* r, float j) {
    const float x = __builtin_fmaf(j, r[R_H], r[R_XC]) * r[R_CSC];
    const float p1 = __builtin_fmaf(x, x, r[R_M + 0]);
    const float p2 = __builtin_fmaf(x, x, r[R_M + 4]);
    const float d1 = __builtin_fmaf(p1, p1, r[R_M + 1]);
    const float d2 = __builtin_fmaf(p2, p2, r[R_M + 5]);
    const float n1 = __builtin_fmaf(p1, r[R_M + 2], r[R_M + 3]);
    const float n2 = __builtin_fmaf(p2, r[R_M + 6], r[R_M + 7]);
    return __builtin_fmaf(n1, __builtin_amdgcn_rcpf(d1), n2 * __builtin_amdgcn_rcpf(d2));
}

// core slice: stored value inside [kcl, kch], 4-node rule elsewhere
__device__ __forceinline__ float v_core(const FwdArgs& A, const float* r, float j, int k) {
    const int* ri = reinterpret_cast<const int*>(r);
    const float vm = v_mid(r, j);
    const long long cb = *reinterpret_cast<const long long*>(r + R_CBASE);
    const bool in = (k >= ri[R_KCL]) && (k <= ri[R_KCH]);
    float vc = 0.0f;
    if (in) vc = A.core_val[cb + k];
    return in ? vc : vm;
}

__device__ __forceinline__ float v_lor(const float* r, float j) {
    const float x = __builtin_fmaf(j, r[R_H], r[R_XC]);
    return r[R_AMP] * __builtin_amdgcn_rcpf(__builtin_fmaf(x, x, 1.0f));
}

// Gauss-Hermite sum of shifted Lorentzians, node pairs +-t_j:
// L(D - dj) + L(D + dj) = (gamma/pi) 2 (D^2 + g^2 + dj^2) / ((D^2 + g^2 - dj^2)^2 + 4 dj^2 g^2)
__device__ __forceinline__ float v_ghs(const Tables* tab, const float* r, float j) {
    const float D = __builtin_fmaf(j, r[R_H], r[R_XC]);
    const float g2 = r[R_M + 0], ad = r[R_M + 1], g4 = r[R_M + 2];
    const float D2 = __builtin_fmaf(D, D, g2);
    float acc = 0.0f;
#pragma unroll
    for (int q = 0; q < kGHConv / 2; ++q) {
        const float t = tab->tconvf[kGHConv / 2 + q];
        const float dj = ad * t;
        const float d2 = dj * dj;
        const float p = D2 - d2;
        const float den = __builtin_fmaf(p, p, g4 * d2);
        acc = __builtin_fmaf(2.0f * tab->wconvf[kGHConv / 2 + q] * (D2 + d2), __builtin_amdgcn_rcpf(den), acc);
    }
    return r[R_AMP] * acc;
}

// bin-averaged Gauss-Hermite Voigt: atan(y+) - atan(y-) = atan2(dnu g, (D - dj)^2 + g^2 - dnu^2/4)
__device__ __forceinline__ float v_ghb(const Tables* tab, const float* r, float j) {
    const float D = __builtin_fmaf(j, r[R_H], r[R_XC]);
    const float ad = r[R_M + 1], hg = r[R_M + 3], c = r[R_M + 4];
    float acc = 0.0f;
    for (int q = 0; q < kGHConv; ++q) {
        const float e = D - ad * tab->tconvf[q];
        acc = __builtin_fmaf(tab->wconvf[q], atan2f(hg, __builtin_fmaf(e, e, c)), acc);
    }
    return r[R_AMP] * acc;
}

__device__ __forceinline__ float v_gauss(const float* r, float j) {
    const float x = __builtin_fmaf(j, r[R_H], r[R_XC]);
    return r[R_AMP] * __builtin_amdgcn_exp2f(-x * x);
}

template <int PROF, int WAVES, int P, bool SEG>
__global__ __launch_bounds__(64 * WAVES) void fwd_f32_kernel(const FwdArgs A) {
    constexpr int NT = 64 * WAVES;       // threads = lines per LDS batch
    constexpr int W = NT * P;            // grid points per tile
    constexpr int WW = 64 * P;           // grid points per wavefront
    __shared__ float rec[NT * kRec];

    const Geometry G = A.G;
    // the wavefront index is uniform within a wavefront: keep it (and everything derived
    // from it: run bounds, loop counters, LDS record offsets) in scalar registers
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const WorkItem wi = work_item(A);
    const TPParam tp = A.tps[wi.tp];
    const int* crc = PROF == kVoigt ? A.core_rc + (int64_t)wi.tp * A.core_stride : nullptr;
    const long long* coff = PROF == kVoigt ? A.core_off + (int64_t)wi.tp * A.core_stride : nullptr;
    const int t0 = wi.tile * W, t1 = t0 + W - 1;
    const int w0 = t0 + wave * WW, w1 = w0 + WW - 1;

    // lines overlapping the tile; this workgroup takes every n_split-th batch of them
    const int b0 = off_at(A.off, (int64_t)t0 - G.hmax, G);
    const int b5 = off_at(A.off, (int64_t)t1 + G.hmax + 1, G);
    const int bstride = NT * A.n_split;
    const int bfirst = b0 + NT * wi.part;
    int rm = tp.rm;
    if (SEG && tp.rm_scale > 0.0) {
        // the centre-near run holds lines with kc within rm of the wave, i.e. wavenumbers
        // inside [nlo, nhi]; their Doppler widths, hence the radius, are bounded there
        const double nlo = G.nu_a + ((double)w0 - rm - 1) * G.dnu;
        const double nhi = G.nu_a + ((double)w1 + rm + 1) * G.dnu;
        const double rw = ceil(tp.rm_scale * fmax(fabs(nlo), fabs(nhi))) + 2.0;
        if (rw < (double)rm) rm = __builtin_amdgcn_readfirstlane((int)rw);
    }
    int s0 = 0, s1 = 0, s2 = 0, s3 = 0, s4 = 0, s5 = 0;
    if (SEG) {
        s0 = off_at(A.off, (int64_t)w0 - G.hmax, G);
        s1 = off_at(A.off, (int64_t)w1 - G.hmin, G);
        s2 = off_at(A.off, (int64_t)w0 - rm, G);
        s3 = off_at(A.off, (int64_t)w1 + rm + 1, G);
        s4 = off_at(A.off, (int64_t)w0 + G.hmin + 1, G);
        s5 = off_at(A.off, (int64_t)w1 + G.hmax + 1, G);
    }
    const double Q = A.Q[tp.iq];

    float jl[P], jlo_w[P], jhi_w[P], part[P], sum[P], comp[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        jl[p] = (float)(64 * (wave * P + p) + lane);     // k - t0
        jlo_w[p] = (float)(64 * p + lane);              // k - w0
        jhi_w[p] = (float)(64 * p + lane - (WW - 1));   // k - w1
        part[p] = 0.f; sum[p] = 0.f; comp[p] = 0.f;
    }
    const int cword = R_CODE + (wave * P) / 8;
    const int cshift = 4 * ((wave * P) % 8);
    const int anc = R_ANC + wave;

    RawLine nxt;
    if (bfirst + tid < b5) nxt = load_raw<PROF>(A, crc, coff, bfirst + tid);
    for (int bs = bfirst; bs < b5; bs += bstride) {
        const int g = bs + tid;
        if (g < b5) prepare_line<PROF, WAVES, P>(A, tp, G, nxt, Q, t0, !SEG, rec + tid * kRec);
        __syncthreads();
        if (g + bstride < b5) nxt = load_raw<PROF>(A, crc, coff, g + bstride);   // overlaps the sweep below
        const int be = bs + NT < b5 ? bs + NT : b5;
        for (int cs = bs; cs < be; cs += 64) {
            const int ce = cs + 64 < be ? cs + 64 : be;
            if (SEG) {
                if (PROF == kVoigt || PROF == kLorentz) {
                    // ---- run 1: window ends inside the wave (upper mask)
                    const int lo = cs > s0 ? cs : s0, hi = ce < s1 ? ce : s1;
                    for (int l = lo; l < hi; ++l) {
                        const float* r = rec + (l - bs) * kRec;
                        const float sb0 = r[R_SB0], jhi = r[R_JHI];
#pragma unroll
                        for (int p = 0; p < P; ++p) {
                            const float j = jl[p] + sb0;
                            const float v = (PROF == kVoigt) ? v_far(r, j) : v_lor(r, j);
                            part[p] += (j <= jhi) ? v : 0.0f;
                        }
                    }
                    // ---- run 5: window starts inside the wave (lower mask)
                    const int lo5 = cs > s4 ? cs : s4, hi5 = ce < s5 ? ce : s5;
                    for (int l = lo5; l < hi5; ++l) {
                        const float* r = rec + (l - bs) * kRec;
                        const float sb0 = r[R_SB0], jlo = r[R_JLO];
#pragma unroll
                        for (int p = 0; p < P; ++p) {
                            const float j = jl[p] + sb0;
                            const float v = (PROF == kVoigt) ? v_far(r, j) : v_lor(r, j);
                            part[p] += (j >= jlo) ? v : 0.0f;
                        }
                    }
                    // ---- runs 2 and 4: wing formula from the anchor, no branches
#pragma unroll
                    for (int side = 0; side < 2; ++side) {
                        const int a0 = side == 0 ? s1 : s3, a1 = side == 0 ? s2 : s4;
                        const int lo2 = cs > a0 ? cs : a0, hi2 = ce < a1 ? ce : a1;
                        const float* jd = side == 0 ? jlo_w : jhi_w;
#pragma unroll 2
                        for (int l = lo2; l < hi2; ++l) {
                            const float* r = rec + (l - bs) * kRec;
                            const float4 h0 = *reinterpret_cast<const float4*>(r);
                            const float2 h1 = *reinterpret_cast<const float2*>(r + 4);
                            const float xa = r[anc];
                            const float h = h0.y, amp = h1.x;
                            if (PROF == kVoigt) {
                                const float c0 = h0.z, c1 = h0.w, bb = h1.y;
#pragma unroll
                                for (int p = 0; p < P; ++p) {
                                    const float x = __builtin_fmaf(jd[p], h, xa);
                                    const float pp = __builtin_fmaf(x, x, c0);
                                    const float den = __builtin_fmaf(pp, pp, c1);
                                    const float num = __builtin_fmaf(pp, amp, bb);
                                    part[p] = __builtin_fmaf(num, __builtin_amdgcn_rcpf(den), part[p]);
                                }
                            } else {
#pragma unroll
                                for (int p = 0; p < P; ++p) {
                                    const float x = __builtin_fmaf(jd[p], h, xa);
                                    part[p] = __builtin_fmaf(amp, __builtin_amdgcn_rcpf(__builtin_fmaf(x, x, 1.0f)), part[p]);
                                }
                            }
                        }
                    }
                }
                // ---- run 3: centre near the wave
                {
                    const int lo3 = cs > s2 ? cs : s2, hi3 = ce < s3 ? ce : s3;
                    for (int l = lo3; l < hi3; ++l) {
                        const float* r = rec + (l - bs) * kRec;
                        const int* ri = reinterpret_cast<const int*>(r);
                        const float sb0 = r[R_SB0];
                        if (PROF == kLorentz) {
#pragma unroll
                            for (int p = 0; p < P; ++p) part[p] += v_lor(r, jl[p] + sb0);
                            continue;
                        }
                        // scalar copies of the line's integer geometry
                        const int kc = t0 - __builtin_amdgcn_readfirstlane(ri[R_SB0I]);
                        const int rad = __builtin_amdgcn_readfirstlane(ri[R_RAD]);
                        const int kcl = __builtin_amdgcn_readfirstlane(ri[R_KCL]);
                        const int kch = __builtin_amdgcn_readfirstlane(ri[R_KCH]);
                        float vc[P];
                        if (PROF == kVoigt) {
                            // issue the stored core-value loads first
                            const long long cb = *reinterpret_cast<const long long*>(r + R_CBASE);
#pragma unroll
                            for (int p = 0; p < P; ++p) {
                                const int k = w0 + 64 * p + lane;
                                vc[p] = (k >= kcl && k <= kch) ? A.core_val[cb + k] : 0.0f;
                            }
                        }
#pragma unroll
                        for (int p = 0; p < P; ++p) {
                            const int kA = w0 + 64 * p, kB = kA + 63;
                            const float j = jl[p] + sb0;
                            const bool near = rad >= 0 && (int64_t)kA <= (int64_t)kc + rad &&
                                              (int64_t)kB >= (int64_t)kc - rad;
                            if (PROF == kVoigt) {
                                if (kA <= kch && kB >= kcl) {
                                    const int k = kA + lane;
                                    const float vm = v_mid(r, j);
                                    part[p] += (k >= kcl && k <= kch) ? vc[p] : vm;
                                } else if (near) {
                                    part[p] += v_mid(r, j);
                                } else {
                                    part[p] += v_far(r, j);
                                }
                            } else {
                                if (near) part[p] += v_gauss(r, j);
                            }
                        }
                    }
                }
            } else {
                // ---- coded sweep: every line carries per-slice codes
                for (int l = cs; l < ce; ++l) {
                    const float* r = rec + (l - bs) * kRec;
                    const unsigned cw =
                        __builtin_amdgcn_readfirstlane(__float_as_uint(r[cword])) >> cshift;
                    if ((cw & ((1u << (4 * P)) - 1u)) == 0u) continue;
                    const float sb0 = r[R_SB0], jlo = r[R_JLO], jhi = r[R_JHI];
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        const unsigned z = (cw >> (4 * p)) & 15u;
                        const unsigned zone = z & 3u;
                        if (zone == 0u) continue;
                        const float j = jl[p] + sb0;
                        float v;
                        if (PROF == kVoigt) {
                            if (zone == 1u) v = v_far(r, j);
                            else if (zone == 2u) v = v_mid(r, j);
                            else v = v_core(A, r, j, w0 + 64 * p + lane);
                        } else if (PROF == kLorentz) {
                            v = v_lor(r, j);
                        } else if (PROF == kGHSampled) {
                            v = v_ghs(A.tab, r, j);
                        } else if (PROF == kGHBinned) {
                            v = v_ghb(A.tab, r, j);
                        } else {
                            v = v_gauss(r, j);
                        }
                        if (z & 4u) v = (j >= jlo && j <= jhi) ? v : 0.0f;
                        part[p] += v;
                    }
                }
            }
            // compensated flush of the 64-line partial sums (TwoSum)
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const float t = sum[p] + part[p];
                const float bp = t - sum[p];
                const float e = (sum[p] - (t - bp)) + (part[p] - bp);
                comp[p] += e;
                sum[p] = t;
                part[p] = 0.f;
            }
        }
        __syncthreads();
    }

    if (A.n_split == 1) {
        float* out = static_cast<float*>(A.sigma) + (int64_t)wi.tp * G.n_points;
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int k = w0 + 64 * p + lane;
            if (k < G.n_points) out[k] = sum[p] + comp[p];
        }
    } else {
        float2* out = static_cast<float2*>(A.part) + ((int64_t)wi.tp * A.n_split + wi.part) * G.n_points;
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int k = w0 + 64 * p + lane;
            if (k < G.n_points) out[k] = make_float2(sum[p], comp[p]);
        }
    }
}

template <int PROF, int WAVES, int P>
void launch_one(const FwdArgs& a, hipStream_t s) {
    const dim3 grid((unsigned)((int64_t)a.n_tiles * a.n_tp * a.n_split)), block(64 * WAVES);
    if (PROF <= kVoigt && a.seg) hipLaunchKernelGGL((fwd_f32_kernel<PROF, WAVES, P, PROF <= kVoigt>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((fwd_f32_kernel<PROF, WAVES, P, false>), grid, block, 0, s, a);
}

template <int PROF>
void launch_p(int waves, int P, const FwdArgs& a, hipStream_t s) {
    if (waves == 4) {
        switch (P) {
            case 1: launch_one<PROF, 4, 1>(a, s); break;
            case 2: launch_one<PROF, 4, 2>(a, s); break;
            default: launch_one<PROF, 4, 4>(a, s); break;
        }
    } else {
        switch (P) {
            case 1: launch_one<PROF, 8, 1>(a, s); break;
            case 2: launch_one<PROF, 8, 2>(a, s); break;
            default: launch_one<PROF, 8, 4>(a, s); break;
        }
    }
}

}  // namespace

hipError_t launch_forward_f32(int profile, int waves, int P, const FwdArgs& a, hipStream_t s) {
    if (a.n_tiles <= 0) return hipSuccess;
    switch (profile) {
        case kDoppler: launch_p<kDoppler>(waves, P, a, s); break;
        case kGaussFixed: launch_p<kGaussFixed>(waves, P, a, s); break;
        case kLorentz: launch_p<kLorentz>(waves, P, a, s); break;
        case kGHSampled: launch_p<kGHSampled>(waves, P, a, s); break;
        case kGHBinned: launch_p<kGHBinned>(waves, P, a, s); break;
        default: launch_p<kVoigt>(waves, P, a, s); break;
    }
    return hipGetLastError();
}

}  // namespace xs
