// FP32 forward path: sigma_k = sum over lines of I f(nu_k - nu_fi) within the cut-off
// (the sampling method; Sec. "Cross sections" Eq. 6-8, Sec. "Standard line profiles and
// sampling method", Sec. "Off-set").
//
// record_kernel, once per (line, T, P): the double-precision line setup (intensity Eq. 1
// with Q(T) from the device, Doppler width Eq. 16, Lorentz width Eq. 18, offset of the
// centre from its nearest grid point) reduced to single-precision coefficients:
//   hot record (8 words) -- what the wing loops read for every line;
//   cold record (16 words) -- zone radii, core-value range and offset, 4-node
//     coefficients, the Gauss-Hermite profile parameters: read for lines whose centre is
//     near the tile;
//   scale (double) -- x per cm^-1 of offset, for the per-tile anchors.
//
// fwd_f32_kernel: a workgroup (WAVES wavefronts) owns a tile of 64*WAVES*P consecutive
// grid points; each wavefront owns P slices of 64 points (one point per lane per slice)
// with its sums in registers, so no atomics touch the output.  Lines are sorted by their
// nearest grid index kc; the lines overlapping a tile are a contiguous range of the sorted
// list, and workgroup q of the n_split sharing a tile takes its LDS batches q, q+n_split,..
// Per batch of 64*WAVES lines: the hot records are copied to LDS (coalesced), each thread
// adds its line's tile fields (grid offset, per-wavefront anchors or per-slice codes) and,
// for lines centred near the tile, the cold record; the wavefronts then sweep the batch
// reading records by broadcast.
//
// Segmented sweep (grids fine enough that 64P + r_mid < the half window): every
// wavefront splits the sorted lines by kc into five contiguous runs relative to its
// own points [w0, w1]:
//   [w0 - hmax, w1 - hmin)  window ends inside the wave:   wing formula + upper mask
//   [w1 - hmin, w0 - rm)    covers the wave, wings only:   wing formula, no branches
//   [w0 - rm,   w1 + rm]    centre near the wave:          per-slice zone (scalar branch)
//   (w1 + rm,  w0 + hmin]   covers the wave, wings only:   wing formula, no branches
//   (w0 + hmin, w1 + hmax]  window starts inside the wave: wing formula + lower mask
// (rm: radius beyond which every point of the wave is in the far zone, from the largest
// Doppler width a line of the centre-near run can have, so it shrinks at low wavenumber)
// Coarse grids use per-slice codes (skip / zone / mask) for every line instead.
// FP32 Voigt: the lines centred more than R = max(far reach, |z| < 8 radius) from the wave
// are node-sampled by the far-wing kernels (xs_far.hip) and left out here, the centre-near
// run shrinking to [w0 - min(rm, R), w1 + min(rm, R)]; when every window-end line lies
// beyond both radii the first and last runs go to those kernels too, and the tile stages
// only the lines within R of it.  The centre-near run then takes per-slice rule codes
// computed once per line at staging (2-node, 4-node, or stored core values).
//
// Vectorized Voigt (Sec. "Vectorized Voigt approximation"): within R of the centre the
// Voigt zones below; beyond R the reference profile times beta, which for the reference's
// Doppler width (that of a line at 1 cm^-1; the host requires sqrt(ln2) R / alpha_ref >=
// 2e4) is the Lorentzian to a relative 3/(2 x_ref^2) <= 4e-9:
//     beta I' (gamma/pi) / (D^2 + gamma^2) = B / (x^2 + Y),  x the line's scaled offset,
// two FMA and a reciprocal per point.  Four more hot words carry Y, B and the index
// bounds of the R region; the segmented sweep splits each wing run in three (outside R,
// crossing R: per-lane select, inside R), and the centre-near run selects per lane.
//
// Voigt zones (|z| = |x + iy|): wings |z| >= 40 use the 2-node Gauss-Hermite rational
// (6 FMA + 1 reciprocal per point); 8 <= |z| < 40 the 4-node rule; points with |z| < 8
// take the value the double-precision core pre-pass stored for them.
// x is formed as fma(j, h, xc) from the exact integer offset j = k - kc, or in the wing
// runs as fma(k - k_anchor, h, x_anchor) from an anchor at the wavefront end nearest the
// centre (computed in double), so its relative error stays ~1e-7 however far the point is
// from the centre.  Partial sums are flushed every 64 lines into a compensated (TwoSum) pair.
#include "xs_far.hpp"
#include "xs_records.hpp"

namespace xs {

namespace {

// ------------------------------------------------------------------ record kernel
template <int PROF>
__global__ __launch_bounds__(256) void record_kernel(const RecArgs A) {
    using L = HotOf<PROF>;
    // ci: position of the record (the compacted index under an intensity threshold)
    const int ci = blockIdx.x * 256 + threadIdx.x;
    if (ci >= A.n_lines || (A.map && (unsigned long long)ci >= *A.count)) return;
    const int g = line_of(A.map, ci);
    const TPParam tp = *A.tp;
    const Geometry G = A.G;
    const double Q = A.Q[tp.iq];
    const double nu = A.L.nu[g];
    const int kc = A.L.kc[g], klo = A.L.klo[g], khi = A.L.khi[g];
    const double S = line_intensity(A.L, g, A.L.elow[g], nu, tp, Q);                      // Eq. 1
    const double aD = nu * tp.beta;                                                               // Eq. 16
    const double gam = (double)A.L.gref[g] * exp((double)A.L.nexp[g] * tp.ln_T0_T) * tp.p_over_p0;  // Eq. 18
    const double d = (G.nu_a + (double)kc * G.dnu) - nu;   // centre offset nu_kc - nu
    constexpr int NH = hot_words(PROF);
    float h[NH];
    int c[kCold];
    float* cf = reinterpret_cast<float*>(c);
#pragma unroll
    for (int i = 0; i < NH; ++i) h[i] = 0.0f;
#pragma unroll
    for (int i = 0; i < kCold; ++i) c[i] = 0;
    h[L::JLO] = (float)(klo - kc);
    h[L::JHI] = (float)(khi - kc);
    c[C_KC] = kc;
    c[C_RAD] = -1;
    c[C_KCH] = -1;
    double scale;
    if (is_voigt(PROF)) {
        const double2 vv = (PROF == kVVoigt && A.vv) ? A.vv[g] : make_double2(1.0, 1.0);
        const double s = kSQRT_LN2 / aD;
        const double y = gam * s;
        const double a = S * vv.y * kSQRT_LN2_PI / aD;
        // power-of-two scaling keeps x^4 inside the float range for very narrow lines
        const double xmax = s * (G.cutoff + 2.0 * G.dnu) + 1.0;
        int e;
        frexp(xmax, &e);
        e = e > 31 ? e - 31 : 0;
        const double sc = ldexp(1.0, -e), sc2 = sc * sc;
        const double y2 = y * y;
        const double ampf = a * y * kINV_SQRT_PI;
        scale = s * sc;
        h[L::XC] = (float)(scale * d);
        h[L::H] = (float)(scale * G.dnu);
        h[L::C0] = (float)((y2 - 0.5) * sc2);
        h[L::C1] = (float)(2.0 * y2 * sc2 * sc2);
        h[L::AMP] = (float)(ampf * sc2);
        h[L::B] = (float)(ampf * sc2 * sc2);
        if (PROF == kVVoigt) {
            // wing: beta I' (gamma/pi) / (D^2 + gamma^2) = B / (x^2 + Y), x = scale D
            h[L::VY] = (float)(y2 * sc2);
            h[L::VB] = (float)(vv.x * S * vv.y * (gam / kPI) * scale * scale);
            const double kvl = ceil((nu - G.vv_radius - G.nu_a) / G.dnu);
            const double kvh = floor((nu + G.vv_radius - G.nu_a) / G.dnu);
            const double lim = 16777216.0;   // keep the float offsets exact
            h[L::JVLO] = (float)fmax(kvl - (double)kc, -lim);
            h[L::JVHI] = (float)fmin(kvh - (double)kc, lim);
        }
        cf[C_CSC] = (float)ldexp(1.0, e);
        // 4-node rule (unscaled x): node pair j = a, b has p_j = x^2 + y^2 - t_j^2,
        // d_j = p_j^2 + 4 t_j^2 y^2 and n_j = amp w_j (p_j + 2 t_j^2), amp = 2 a y / pi
        // (Voigt: rebuilt by the kernels from C1, AMP and the x scale, see mid_from_hot)
        if (PROF == kVVoigt) {
            const double amp = a * (y / kPI) * 2.0;
            const double t2a = A.tab->gh4.t[0] * A.tab->gh4.t[0], t2b = A.tab->gh4.t[1] * A.tab->gh4.t[1];
            const double ma = amp * A.tab->gh4.w[0], mb = amp * A.tab->gh4.w[1];
            cf[C_M + 0] = (float)(y2 - t2a);
            cf[C_M + 1] = (float)(4.0 * t2a * y2);
            cf[C_M + 2] = (float)ma;
            cf[C_M + 3] = (float)(ma * 2.0 * t2a);
            cf[C_M + 4] = (float)(y2 - t2b);
            cf[C_M + 5] = (float)(4.0 * t2b * y2);
            cf[C_M + 6] = (float)mb;
            cf[C_M + 7] = (float)(mb * 2.0 * t2b);
        }
        c[C_RAD] = y2 < kMidR2 ? radius_steps(sqrt(kMidR2 - y2), s * G.dnu, s * d) : -1;
        const int rc = A.core_rc[g];
        int kcl = 0, kch = -1;
        if (rc >= 0) {
            const int64_t lo = (int64_t)kc - rc, hi = (int64_t)kc + rc;
            kcl = (int)(lo > klo ? lo : klo);
            kch = (int)(hi < khi ? hi : khi);
        }
        c[C_KCL] = kcl;
        c[C_KCH] = kch;
        const long long cb = A.core_off[g] - (long long)kcl;
        c[C_CBASE] = (int)(unsigned)(cb & 0xffffffffll);
        c[C_CBASE + 1] = (int)(cb >> 32);
    } else if (PROF == kLorentz) {
        const double ig = gam > 0.0 ? 1.0 / gam : 0.0;
        scale = ig;
        h[L::XC] = (float)(d * ig);
        h[L::H] = (float)(G.dnu * ig);
        h[L::AMP] = (float)(S * ig * (1.0 / kPI));
        c[C_FLAG] = gam > 0.0 ? 1 : 0;
    } else if (PROF == kGHSampled || PROF == kGHBinned) {
        // Gauss-Hermite convolution (Eq. 30-31 as read): nodes shift the Lorentzian by
        // delta_j = alpha_D t_j / sqrt(ln 2); work in wavenumber units D = nu_k - nu
        scale = 1.0;
        h[L::XC] = (float)d;
        h[L::H] = (float)G.dnu;
        cf[C_M + 0] = (float)(gam * gam);
        cf[C_M + 1] = (float)(aD / kSQRT_LN2);
        if (PROF == kGHSampled) {
            h[L::AMP] = (float)(S * gam / (kPI * 1.7724538509055160273));   // S gamma / pi^(3/2)
            cf[C_M + 2] = (float)(4.0 * gam * gam);
        } else {
            h[L::AMP] = (float)(S / (kPI * 1.7724538509055160273 * G.dnu));   // S / (pi^(3/2) dnu)
            cf[C_M + 3] = (float)(G.dnu * gam);
            cf[C_M + 4] = (float)(gam * gam - 0.25 * G.dnu * G.dnu);
        }
        c[C_FLAG] = gam > 0.0 ? 1 : 0;
    } else if (PROF == kLorentzBinned) {
        // bin average of Eq. 17: S/(pi dnu) atan2(dnu gamma, D^2 + gamma^2 - dnu^2/4)
        scale = 1.0;
        h[L::XC] = (float)d;
        h[L::H] = (float)G.dnu;
        h[L::AMP] = (float)(S / (kPI * G.dnu));
        cf[C_M + 0] = (float)(G.dnu * gam);
        cf[C_M + 1] = (float)(gam * gam - 0.25 * G.dnu * G.dnu);
        // the three bins nearest the centre are evaluated in double (D^2 - dnu^2/4 cancels
        // there): centre offset d and gamma
        const long long bd = __double_as_longlong(d), bg = __double_as_longlong(gam);
        c[C_M + 2] = (int)(unsigned)(bd & 0xffffffffll);
        c[C_M + 3] = (int)(bd >> 32);
        c[C_M + 4] = (int)(unsigned)(bg & 0xffffffffll);
        c[C_M + 5] = (int)(bg >> 32);
    } else if (PROF == kDopplerBinned) {
        // bin average of Eq. 15 (Doppler HWHM): S/(2 dnu) [erf(x+) - erf(x-)], evaluated in
        // double from the centre offset d and s = sqrt(ln2)/alpha_D (cold words)
        const double s = kSQRT_LN2 / aD;
        scale = 1.0;
        h[L::XC] = (float)d;
        h[L::H] = (float)G.dnu;
        h[L::AMP] = (float)(S / (2.0 * G.dnu));
        const long long bd = __double_as_longlong(d), bs = __double_as_longlong(s);
        c[C_M + 0] = (int)(unsigned)(bd & 0xffffffffll);
        c[C_M + 1] = (int)(bd >> 32);
        c[C_M + 2] = (int)(unsigned)(bs & 0xffffffffll);
        c[C_M + 3] = (int)(bs >> 32);
        c[C_RAD] = radius_steps(10.5 + 0.5 * s * G.dnu, s * G.dnu, s * d);   // both edges beyond x = 10.5
    } else {
        // Gaussian (Eq. 15); x scaled by sqrt(1/ln 2) so exp(-x^2) = exp2(-x'^2)
        const double alpha = (PROF == kDoppler) ? aD : A.alpha_fixed;
        const double s = kSQRT_LN2 / alpha;
        scale = s * 1.2011224087864498;
        h[L::XC] = (float)(scale * d);
        h[L::H] = (float)(scale * G.dnu);
        h[L::AMP] = (float)(S * kSQRT_LN2_PI / alpha);
        c[C_RAD] = radius_steps(10.5, s * G.dnu, s * d);   // exp(-x^2) underflows beyond
    }
    float4* ho = reinterpret_cast<float4*>(A.hot + (int64_t)ci * NH);
#pragma unroll
    for (int q = 0; q < NH / 4; ++q) ho[q] = make_float4(h[4 * q], h[4 * q + 1], h[4 * q + 2], h[4 * q + 3]);
    // cold words 0-7 and 8-15 in their two planes (the second not needed for Voigt)
    int4* co = reinterpret_cast<int4*>(A.cold + (int64_t)ci * 8);
    co[0] = make_int4(c[0], c[1], c[2], c[3]);
    co[1] = make_int4(c[4], c[5], c[6], c[7]);
    if (PROF != kVoigt) {
        int4* cb = reinterpret_cast<int4*>(A.cold_b + (int64_t)ci * 8);
        cb[0] = make_int4(c[8], c[9], c[10], c[11]);
        cb[1] = make_int4(c[12], c[13], c[14], c[15]);
    }
    A.xscale[ci] = scale;
}

// ------------------------------------------------------------------ tile kernel
// LDS image of one batch: line records of RS words (the 8 hot words, then for the
// segmented sweep one anchor per wavefront, so a wing-loop line is read from one base
// address), the grid offset, slice codes (coded sweep) and the cold fields (one array
// per field, indexed by the line's place in the batch).
template <int NT, int RS, int NTF, int NM, int NKR = NT, int NCK = NT>
struct Lds {
    float4 rec[NT * RS / 4];
    float sb0[NT];          // t0 - kc
    float tf[NTF];          // slice-code words (coded sweep: NCW per line, stride NT; Voigt
                            // segmented sweep: 2-bit rule codes)
    float csc[NCK];         // x scale and core range (in the record's spare words when it
    int kcl[NCK], kch[NCK]; // has three, see CK_IN_REC)
    int kc[NKR], rad[NKR];  // centre and mid radius (not staged where rule codes replace them)
    long long cb[NT];
    alignas(16) float m[NM * NT];   // cold profile words (stride NT; Voigt segmented
                                    // sweep: the line's eight words together)
};
// segmented sweep: no slice codes (keeps the Vectorized Voigt image at 32 KiB, five
// workgroups per CU)
template <int NT, int RS, int NM, int NKR, int NCK>
struct Lds<NT, RS, 0, NM, NKR, NCK> {
    float4 rec[NT * RS / 4];
    float sb0[NT];
    float csc[NCK];
    int kcl[NCK], kch[NCK];
    int kc[NKR], rad[NKR];
    long long cb[NT];
    alignas(16) float m[NM * NT];
};

// wing formula (2-node rule, scaled variables)
template <int PROF>
__device__ __forceinline__ float v_far(const float* r, float j) {
    using L = HotOf<PROF>;
    const float x = __builtin_fmaf(j, r[L::H], r[L::XC]);
    const float pp = __builtin_fmaf(x, x, r[L::C0]);
    const float den = __builtin_fmaf(pp, pp, r[L::C1]);
    const float num = __builtin_fmaf(pp, r[L::AMP], r[L::B]);
    return num * __builtin_amdgcn_rcpf(den);
}

// 4-node rule coefficients of one line, from y^2 and the amplitude (node pairs t_j, w_j):
// p_j = x^2 + y^2 - t_j^2, d_j = p_j^2 + 4 t_j^2 y^2, n_j = amp w_j (p_j + 2 t_j^2)
struct Mid {
    float m0, m1, m2, m3, m4, m5, m6, m7;
};

// the line's coefficients from the LDS copy of its cold words (stride NT)
template <int NT>
__device__ __forceinline__ Mid mid_coef(const float* m) {
    Mid c;
    c.m0 = m[0]; c.m1 = m[NT]; c.m2 = m[2 * NT]; c.m3 = m[3 * NT];
    c.m4 = m[4 * NT]; c.m5 = m[5 * NT]; c.m6 = m[6 * NT]; c.m7 = m[7 * NT];
    return c;
}

// the same from the line's eight consecutive words (two LDS reads)
__device__ __forceinline__ Mid mid_coef8(const float* m) {
    const float4 a = *reinterpret_cast<const float4*>(m), b = *reinterpret_cast<const float4*>(m + 4);
    Mid c;
    c.m0 = a.x; c.m1 = a.y; c.m2 = a.z; c.m3 = a.w;
    c.m4 = b.x; c.m5 = b.y; c.m6 = b.z; c.m7 = b.w;
    return c;
}

// 4-node rule at unscaled x, added to acc
__device__ __forceinline__ float mid_rule(const Mid& c, float x, float acc) {
    const float p1 = __builtin_fmaf(x, x, c.m0);
    const float p2 = __builtin_fmaf(x, x, c.m4);
    const float d1 = __builtin_fmaf(p1, p1, c.m1);
    const float d2 = __builtin_fmaf(p2, p2, c.m5);
    const float n1 = __builtin_fmaf(p1, c.m2, c.m3);
    const float n2 = __builtin_fmaf(p2, c.m6, c.m7);
    return __builtin_fmaf(n1, __builtin_amdgcn_rcpf(d1), __builtin_fmaf(n2, __builtin_amdgcn_rcpf(d2), acc));
}

// 4-node rule (unscaled x)
template <int PROF>
__device__ __forceinline__ float v_mid(const float* r, const Mid& c, float csc, float j) {
    using L = HotOf<PROF>;
    const float x = __builtin_fmaf(j, r[L::H], r[L::XC]) * csc;
    const float p1 = __builtin_fmaf(x, x, c.m0);
    const float p2 = __builtin_fmaf(x, x, c.m4);
    const float d1 = __builtin_fmaf(p1, p1, c.m1);
    const float d2 = __builtin_fmaf(p2, p2, c.m5);
    const float n1 = __builtin_fmaf(p1, c.m2, c.m3);
    const float n2 = __builtin_fmaf(p2, c.m6, c.m7);
    return __builtin_fmaf(n1, __builtin_amdgcn_rcpf(d1), n2 * __builtin_amdgcn_rcpf(d2));
}

using LD = HotOf<kVoigt>;   // layout of the other profiles

__device__ __forceinline__ float v_lor(const float* r, float j) {
    const float x = __builtin_fmaf(j, r[LD::H], r[LD::XC]);
    return r[LD::AMP] * __builtin_amdgcn_rcpf(__builtin_fmaf(x, x, 1.0f));
}

// Gauss-Hermite sum of shifted Lorentzians, node pairs +-t_j:
// L(D - dj) + L(D + dj) = (gamma/pi) 2 (D^2 + g^2 + dj^2) / ((D^2 + g^2 - dj^2)^2 + 4 dj^2 g^2)
template <int NT>
__device__ __forceinline__ float v_ghs(const Tables* tab, const float* r, const float* m, float j) {
    const float D = __builtin_fmaf(j, r[LD::H], r[LD::XC]);
    const float g2 = m[0], ad = m[NT], g4 = m[2 * NT];
    const float D2 = __builtin_fmaf(D, D, g2);
    float acc = 0.0f;
    const int np = tab->npair;
    for (int q = 0; q < np; ++q) {
        const float dj = ad * tab->tpairf[q];
        const float d2 = dj * dj;
        const float p = D2 - d2;
        const float den = __builtin_fmaf(p, p, g4 * d2);
        acc = __builtin_fmaf(2.0f * tab->wpairf[q] * (D2 + d2), __builtin_amdgcn_rcpf(den), acc);
    }
    return r[LD::AMP] * acc;
}

// bin-averaged Gauss-Hermite Voigt: atan(y+) - atan(y-) = atan2(dnu g, (D - dj)^2 + g^2 - dnu^2/4)
template <int NT>
__device__ __forceinline__ float v_ghb(const Tables* tab, const float* r, const float* m, float j) {
    const float D = __builtin_fmaf(j, r[LD::H], r[LD::XC]);
    const float ad = m[NT], hg = m[3 * NT], c = m[4 * NT];
    float acc = 0.0f;
    const int nn = tab->nconv;
    for (int q = 0; q < nn; ++q) {
        const float e = D - ad * tab->tconvf[q];
        acc = __builtin_fmaf(tab->wconvf[q], atan2f(hg, __builtin_fmaf(e, e, c)), acc);
    }
    return r[LD::AMP] * acc;
}

__device__ __forceinline__ float v_gauss(const float* r, float j) {
    const float x = __builtin_fmaf(j, r[LD::H], r[LD::XC]);
    return r[LD::AMP] * __builtin_amdgcn_exp2f(-x * x);
}

// Vectorized Voigt wing beyond R: B / (x^2 + Y)
__device__ __forceinline__ float v_vvw(const float* r, float j) {
    using L = HotOf<kVVoigt>;
    static_assert(L::H == 0 && L::VY == 1 && L::VB == 2 && L::XC == 3, "wing words");
    const float4 q = *reinterpret_cast<const float4*>(r);   // h, Y, B, xc
    const float x = __builtin_fmaf(j, q.x, q.w);
    return q.z * __builtin_amdgcn_rcpf(__builtin_fmaf(x, x, q.y));
}

// Branch-free wing loop over sorted lines [lo, hi) of the batch starting at bs:
// x = anchor + (k - k_anchor) h, with jd[p] = k - k_anchor of this lane's points.  The
// anchor of this wavefront is word IA of the line record or, with IA < 0, rebuilt per
// line as (k_anchor - kc) h + xc, k_anchor - kc = (t0 - kc) + koff (two operations per
// line instead of WAVES record words).  KIND: 0 the Voigt 2-node rule, 1 the Lorentzian,
// 2 the Vectorized Voigt wing beyond R.
template <int PROF, int KIND, int P, int RS, int IA>
__device__ __forceinline__ void wing_run(const float* rec, const float* sb0, float koff, int bs, int lo, int hi,
                                         const float (&jd)[P], float (&part)[P]) {
    using L = HotOf<PROF>;
#pragma unroll 2
    for (int l = lo; l < hi; ++l) {
        const float* r = rec + (l - bs) * RS;
        float xa;
        if constexpr (IA >= 0) xa = r[IA];
        else xa = __builtin_fmaf(sb0[l - bs] + koff, r[L::H], r[L::XC]);
        if constexpr (KIND == 0) {
            // h, C0, C1, AMP, B: one float4 and one word in either layout
            float h, c0, c1, amp, bb;
            if constexpr (PROF == kVVoigt) {
                const float4 q = *reinterpret_cast<const float4*>(r + L::C0);
                h = r[L::H]; c0 = q.x; c1 = q.y; amp = q.z; bb = q.w;
                static_assert(L::C1 == L::C0 + 1 && L::AMP == L::C0 + 2 && L::B == L::C0 + 3, "layout");
            } else {
                const float4 q = *reinterpret_cast<const float4*>(r);
                h = q.x; c0 = q.y; c1 = q.z; amp = q.w; bb = r[L::B];
                static_assert(L::H == 0 && L::C0 == 1 && L::C1 == 2 && L::AMP == 3, "layout");
            }
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const float x = __builtin_fmaf(jd[p], h, xa);
                const float pp = __builtin_fmaf(x, x, c0);
                const float den = __builtin_fmaf(pp, pp, c1);
                const float num = __builtin_fmaf(pp, amp, bb);
                part[p] = __builtin_fmaf(num, __builtin_amdgcn_rcpf(den), part[p]);
            }
        } else if constexpr (KIND == 3) {
            // Voigt far wing, |x| >= kFarX: one pole, amp / (x^2 + y^2 - 1/2) in the scaled
            // variables (C0 = (y^2 - 1/2) sc^2, AMP = a y sc^2 / sqrt(pi)); against
            // Re w(z) = (y/sqrt(pi)) |z|^-2 (1 + (3x^2 - y^2)/(2|z|^4) + ...) its relative
            // error is (x^2 - y^2)/|z|^4 + O(|z|^-4), at most 1/kFarX^2
            const float4 q = *reinterpret_cast<const float4*>(r);
            static_assert(L::H == 0 && L::C0 == 1 && L::AMP == 3, "layout");
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const float x = __builtin_fmaf(jd[p], q.x, xa);
                part[p] = __builtin_fmaf(q.w, __builtin_amdgcn_rcpf(__builtin_fmaf(x, x, q.y)), part[p]);
            }
        } else if constexpr (KIND == 1) {
            const float4 q = *reinterpret_cast<const float4*>(r);
            const float h = q.x, amp = q.w;
            static_assert(L::H == 0 && L::AMP == 3, "layout");
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const float x = __builtin_fmaf(jd[p], h, xa);
                part[p] = __builtin_fmaf(amp, __builtin_amdgcn_rcpf(__builtin_fmaf(x, x, 1.0f)), part[p]);
            }
        } else {
            const float4 q = *reinterpret_cast<const float4*>(r);   // h, Y, B, xc
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const float x = __builtin_fmaf(jd[p], q.x, xa);
                part[p] = __builtin_fmaf(q.z, __builtin_amdgcn_rcpf(__builtin_fmaf(x, x, q.y)), part[p]);
            }
        }
    }
}

// Wing-only runs of wavefront WV (its anchor word is a compile-time offset): for the
// Voigt and Lorentz profiles one run on each side, [lo2, hi2) and [lo4, hi4); for the
// Vectorized Voigt the runs outside R ([lo2, ha) left, [hd, hi4) right) take the
// reference wing and the runs inside R ([hb, hi2) left, [lo4, hc) right) the 2-node rule.
// Wing-only runs of one wavefront.  Lorentz: [lo2, hi2) left of the wave and [lo4, hi4)
// right of it; Voigt: the same runs, each split where the lines' far-wing radius kFarX
// crosses the wave (one pole beyond it, the 2-node rule inside); Vectorized Voigt: [lo2, ha) beyond R and [hb, hi2) inside R on
// the left, [lo4, hc) inside R and [hd, hi4) beyond R on the right.  IA: anchor word of
// this wavefront, or -1 to rebuild anchors from (t0 - kc) + kl (left, kl = w0 - t0) or
// + kr (right, kr = w1 - t0).
template <int PROF, int P, int RS, int IA>
__device__ __forceinline__ void wing_runs(const float* rec, const float* sb0, float kl, float kr, int bs, int lo2,
                                          int hi2, int lo4, int hi4, int ha, int hb, int hc, int hd,
                                          const float (&jlo_w)[P], const float (&jhi_w)[P], float (&part)[P]) {
    if constexpr (PROF == kVVoigt) {
        wing_run<PROF, 2, P, RS, IA>(rec, sb0, kl, bs, lo2, ha, jlo_w, part);
        wing_run<PROF, 0, P, RS, IA>(rec, sb0, kl, bs, hb, hi2, jlo_w, part);
        wing_run<PROF, 0, P, RS, IA>(rec, sb0, kr, bs, lo4, hc, jhi_w, part);
        wing_run<PROF, 2, P, RS, IA>(rec, sb0, kr, bs, hd, hi4, jhi_w, part);
    } else if constexpr (PROF == kVoigt) {
        // [lo2, ha) and [hd, hi4): every point of the wave at |x| >= kFarX (one pole);
        // [hb, hi2) and [lo4, hc): the 2-node rule
        wing_run<PROF, 3, P, RS, IA>(rec, sb0, kl, bs, lo2, ha, jlo_w, part);
        wing_run<PROF, 0, P, RS, IA>(rec, sb0, kl, bs, hb, hi2, jlo_w, part);
        wing_run<PROF, 0, P, RS, IA>(rec, sb0, kr, bs, lo4, hc, jhi_w, part);
        wing_run<PROF, 3, P, RS, IA>(rec, sb0, kr, bs, hd, hi4, jhi_w, part);
    } else {
        wing_run<PROF, 1, P, RS, IA>(rec, sb0, kl, bs, lo2, hi2, jlo_w, part);
        wing_run<PROF, 1, P, RS, IA>(rec, sb0, kr, bs, lo4, hi4, jhi_w, part);
    }
}

// A batch's global data of one thread: NQ float4 chunks of the hot records (chunks tid,
// NT + tid, ... of the batch; chunk c is quarter c % NQ of line c / NQ) and its own line's
// offset data.  Loaded when the batch is staged: holding the next batch's data in registers
// through the sweep (a prefetch) made the compiler spill them, which waits for the loads
// at once and cost more than it hid.
template <int NQ>
struct BatchLoad {
    float4 h[NQ];
    int kc;
    double nu, scale;
};

template <int NT, int NQ>
__device__ __forceinline__ BatchLoad<NQ> load_batch(const FwdArgs& A, const int* map, const float4* ghot,
                                                   const double* gscale, int bs, int b5, int tid) {
    BatchLoad<NQ> f;
    const int64_t cend = NQ * (int64_t)b5;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int64_t c = NQ * (int64_t)bs + q * NT + tid;
        f.h[q] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (c < cend) f.h[q] = ghot[c];
    }
    f.kc = 0;
    f.nu = 0.0;
    f.scale = 0.0;
    const int g = bs + tid;
    if (g < b5) {
        const int gs = line_of(map, g);
        f.kc = A.L.kc[gs];
        f.nu = A.L.nu[gs];
        f.scale = gscale[g];
    }
    return f;
}

template <int PROF, int WAVES, int P, bool SEG>
__global__ __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(WAVES == 1 ? 6 : 1))) void fwd_f32_kernel(const FwdArgs A) {
    constexpr int NT = 64 * WAVES;       // threads = lines per LDS batch
    constexpr int W = NT * P;            // grid points per tile
    constexpr int WW = 64 * P;           // grid points per wavefront
    constexpr int NS = WAVES * P;        // slices per tile
    constexpr int NCW = (NS + 7) / 8;    // code words (4 bits per slice)
    using L = HotOf<PROF>;
    constexpr int RH = hot_words(PROF);   // hot record words
    constexpr int NQ = RH / 4;            // float4 chunks per hot record
    // per-wavefront anchor words in the LDS record (segmented sweep), or anchors rebuilt
    // per line (a smaller LDS image, more resident workgroups)
    constexpr bool ANCH = SEG && anchors_in_lds(PROF);
    // LDS record words, a multiple of 4 (records are copied and read as float4)
    constexpr int RS = ANCH ? (RH + WAVES + 3) / 4 * 4 : RH;
    static_assert(RS % 4 == 0, "record stride");
    // segmented Voigt sweep: 2-bit rule code per slice (0 the 2-node rule, 1 the 4-node
    // rule, 2 stored core values inside the 4-node rule: only for a non-empty core range, so
    // the values a code-2 slice loads at indices clamped into the range exist) of the lines
    // centred near the tile
    constexpr int NZW = (2 * NS + 31) / 32;
    constexpr bool ZC = SEG && PROF == kVoigt;
    constexpr int NTF = SEG ? (ZC ? NZW * NT : 0) : NCW * NT;
    // cold profile words in LDS
    constexpr int NM = is_voigt(PROF) ? 8 : (PROF == kGHSampled || PROF == kGHBinned) ? 5
                       : PROF == kDopplerBinned ? 4 : PROF == kLorentzBinned ? 6 : 2;
    // Voigt segmented sweep whose LDS record has three spare words after the anchors: the
    // x scale and core range go there (a smaller image, more resident workgroups)
    constexpr bool CK_IN_REC = ZC && RS - RH - WAVES >= 3;
    constexpr int CKW = RH + WAVES;   // first spare word
    __shared__ Lds<NT, RS, NTF, NM, ZC ? 1 : NT, CK_IN_REC ? 1 : NT> S;

    const Geometry G = A.G;
    // the wavefront index is uniform within a wavefront: keep it (and everything derived
    // from it: run bounds, loop counters, LDS offsets) in scalar registers
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const WorkItem wi = work_item(A);
    const TPParam tp = A.tps[wi.tp];
    const int64_t row = (int64_t)wi.tp * A.rec_stride;
    const float4* ghot = reinterpret_cast<const float4*>(A.hot + row * RH);
    // cold records: words 0-7 of the row's lines, then words 8-15 (second plane)
    const int4* gcold = reinterpret_cast<const int4*>(A.cold + row * kCold);
    const int4* gcoldb = reinterpret_cast<const int4*>(A.cold + row * kCold + A.rec_stride * 8);
    const MidNodes mnodes = mid_nodes(A.tab);
    const double* gscale = A.xscale + row;
    // intensity threshold: this (T, P)'s kept lines and offsets table
    const int* map = A.map ? A.map + (int64_t)wi.tp * A.map_stride : nullptr;
    const int* off = A.offs ? A.offs + (int64_t)wi.tp * A.offs_stride : A.off;
    const int t0 = wi.tile * W, t1 = t0 + W - 1;
    const int w0 = t0 + wave * WW, w1 = w0 + WW - 1;

    // lines overlapping the tile; this workgroup takes every n_split-th batch of them.  With
    // the window ends node-sampled too (far_ends), only lines centred within the far reach
    // (or the centre-near radius) of the tile remain here.
    const bool ends_far = SEG && PROF == kVoigt && A.far && A.far_ends;
    const int64_t rnear = wave_far_r(tp, G, t0, t1, far_reach(WW));
    const int b0 = off_at(off, (int64_t)t0 - (ends_far ? rnear : G.hmax), G);
    const int b5 = off_at(off, (int64_t)t1 + (ends_far ? rnear : G.hmax) + 1, G);
    const int bstride = NT * A.n_split;
    const int bfirst = b0 + NT * wi.part;
    const int rm_tile = tp.rm;
    // the centre-near run holds lines with kc within rm of the wave
    const int rm = SEG ? wave_rm(tp, G, w0, w1) : tp.rm;
    int s0 = 0, s1 = 0, s2 = 0, s3 = 0, s4 = 0, s5 = 0;
    int ha = 0, hb = 0, hc = 0, hd = 0;
    int hcl = 0, hcr = 0;   // node-sampled lines (far_kernel): [s1, hcl) left, [hcr, s4) right
    if (SEG) {
        s0 = off_at(off, (int64_t)w0 - G.hmax, G);
        s1 = off_at(off, (int64_t)w1 - G.hmin, G);
        s2 = off_at(off, (int64_t)w0 - rm, G);
        s3 = off_at(off, (int64_t)w1 + rm + 1, G);
        s4 = off_at(off, (int64_t)w0 + G.hmin + 1, G);
        s5 = off_at(off, (int64_t)w1 + G.hmax + 1, G);
        if (PROF == kVoigt) { ha = hb = s1; hc = hd = s4; }   // no one-pole lines unless bounded
        if (PROF == kVoigt && tp.rm_scale > 0.0) {
            // wing-only runs split at the far-wing radius: every point of the wave lies at
            // |x| >= kFarX from a line with |kc - k| > rf for all k of the wave, where
            // rf >= kFarX alpha_D / (sqrt(ln2) dnu) + 1/2 over the wavenumbers of the lines
            // the runs can hold (rm_scale is that radius per cm^-1 at the 2-node bound 40)
            const double nlo = G.nu_a + ((double)w0 - G.hmax - 1) * G.dnu;
            const double nhi = G.nu_a + ((double)w1 + G.hmax + 1) * G.dnu;
            const double rfd = ceil(tp.rm_scale * (kFarX / 40.0) * fmax(fabs(nlo), fabs(nhi))) + 2.0;
            const int64_t rf = rfd < 1.0e9 ? (int64_t)rfd : 1000000000;
            const int64_t l0 = (int64_t)w1 - G.hmin, l1 = (int64_t)w0 - rm;
            const int64_t r0 = (int64_t)w1 + rm + 1, r1 = (int64_t)w0 + G.hmin + 1;
            auto cl = [](int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo : (v > hi ? hi : v); };
            ha = hb = off_at(off, cl((int64_t)w0 - rf, l0, l1), G);
            hc = hd = off_at(off, cl((int64_t)w1 + rf + 1, r0, r1), G);
        }
        if (PROF == kVVoigt) {
            // wing-only runs split where R can cross the wave: left lines with kc < w0 - rvmax
            // see only points beyond R, those with kc >= w1 - rvmin only points inside R
            // (bounds clamped into the runs, so the pieces stay ordered)
            const int64_t l0 = (int64_t)w1 - G.hmin, l1 = (int64_t)w0 - rm;
            const int64_t r0 = (int64_t)w1 + rm + 1, r1 = (int64_t)w0 + G.hmin + 1;
            auto cl = [](int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo : (v > hi ? hi : v); };
            ha = off_at(off, cl((int64_t)w0 - G.rvmax, l0, l1), G);
            hb = off_at(off, cl((int64_t)w1 - G.rvmin, l0, l1), G);
            hc = off_at(off, cl((int64_t)w0 + G.rvmin + 1, r0, r1), G);
            hd = off_at(off, cl((int64_t)w1 + G.rvmax + 1, r0, r1), G);
        }
        hcl = s1;
        hcr = s4;
        if (PROF == kVoigt && A.far) {
            const FarRange fr = far_range(off, G, w0, w1, rm, wave_far_r(tp, G, w0, w1, far_reach(WW)));
            hcl = fr.hcl;
            hcr = fr.hcr;
            // lines of the centre-near run beyond R are node-sampled too
            s2 = s2 > hcl ? s2 : hcl;
            s3 = s3 < hcr ? s3 : hcr;
        }
        if (ends_far) {   // runs 1 and 5 belong to the far kernel
            s0 = s1;
            s5 = s4;
        }
    }

    float jl[P], jlo_w[P], jhi_w[P], part[P], sum[P], comp[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        jl[p] = (float)(64 * (wave * P + p) + lane);     // k - t0
        jlo_w[p] = (float)(64 * p + lane);              // k - w0
        jhi_w[p] = (float)(64 * p + lane - (WW - 1));   // k - w1
        part[p] = 0.f; sum[p] = 0.f; comp[p] = 0.f;
    }
    const int cword = (wave * P) / 8;
    const int cshift = 4 * ((wave * P) % 8);
    const int zword = (2 * wave * P) / 32;    // this wavefront's rule codes (2P bits)
    const int zshift = (2 * wave * P) % 32;

    for (int bs = bfirst; bs < b5; bs += bstride) {
        const BatchLoad<NQ> bl = load_batch<NT, NQ>(A, map, ghot, gscale, bs, b5, tid);
        const int g = bs + tid;
        // ---- batch set-up: hot records (coalesced loads; chunk c is quarter c % NQ of
        // line c / NQ), then this thread's line
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int c = q * NT + tid;
            if (NQ * (int64_t)bs + c < NQ * (int64_t)b5) S.rec[(c / NQ) * (RS / 4) + (c % NQ)] = bl.h[q];
        }
        if (g < b5) {
            const int kc = bl.kc;
            S.sb0[tid] = (float)(t0 - kc);
            if constexpr (ANCH) {
                // x at the end of each wavefront's range nearest the centre: wing points are
                // then x = anchor + (k - k_anchor) h with both terms of one sign
                const double d = (G.nu_a + (double)kc * G.dnu) - bl.nu;
                const double hd = bl.scale * G.dnu, xd = bl.scale * d;
#pragma unroll
                for (int wv = 0; wv < WAVES; ++wv) {
                    const int wa = t0 + WW * wv;
                    const int ka = wa > kc ? wa : wa + WW - 1;
                    reinterpret_cast<float*>(S.rec)[tid * RS + RH + wv] =
                        (float)__builtin_fma((double)(ka - kc), hd, xd);
                }
            }
            // cold fields for lines whose centre can be near the tile (every line for
            // the coded sweep)
            const bool near = !SEG || (PROF != kLorentz && (int64_t)kc >= (int64_t)t0 - rm_tile &&
                                       (int64_t)kc <= (int64_t)t1 + rm_tile);
            if (near) {
                const int4* cg = gcold + (int64_t)g * 2;
                const int4 q0 = cg[0], q1 = cg[1];
                int4 q2, q3;
                if constexpr (PROF == kVoigt) {
                    // the 4-node coefficients from the hot words C1, AMP and the x scale
                    const float2 ca = *reinterpret_cast<const float2*>(A.hot + (row + g) * RH + L::C1);
                    static_assert(L::AMP == L::C1 + 1, "layout");
                    float mm[8];
                    mid_from_hot(ca.x, ca.y, __int_as_float(q0.x), mnodes, mm);
                    q2 = make_int4(__float_as_int(mm[0]), __float_as_int(mm[1]), __float_as_int(mm[2]),
                                   __float_as_int(mm[3]));
                    q3 = make_int4(__float_as_int(mm[4]), __float_as_int(mm[5]), __float_as_int(mm[6]),
                                   __float_as_int(mm[7]));
                } else {
                    const int4* cb = gcoldb + (int64_t)g * 2;
                    q2 = cb[0];
                    q3 = cb[1];
                }
                if constexpr (CK_IN_REC) {
                    float* rw = reinterpret_cast<float*>(S.rec) + tid * RS + CKW;
                    rw[0] = __int_as_float(q0.x);
                    rw[1] = __int_as_float(q0.w);
                    rw[2] = __int_as_float(q1.x);
                } else {
                    S.csc[tid] = __int_as_float(q0.x);
                    S.kcl[tid] = q0.w;
                    S.kch[tid] = q1.x;
                }
                if constexpr (!ZC) {
                    S.kc[tid] = q0.y;
                    S.rad[tid] = q0.z;
                }
                S.cb[tid] = (long long)(((unsigned long long)(unsigned)q1.w << 32) | (unsigned)q1.z);
                if constexpr (ZC) {
                    static_assert(NM == 8, "Voigt cold words");
                    float4* m4 = reinterpret_cast<float4*>(S.m) + 2 * tid;
                    m4[0] = make_float4(__int_as_float(q2.x), __int_as_float(q2.y), __int_as_float(q2.z),
                                        __int_as_float(q2.w));
                    m4[1] = make_float4(__int_as_float(q3.x), __int_as_float(q3.y), __int_as_float(q3.z),
                                        __int_as_float(q3.w));
                } else {
                    S.m[0 * NT + tid] = __int_as_float(q2.x);
                    S.m[1 * NT + tid] = __int_as_float(q2.y);
                    if constexpr (NM > 2) S.m[2 * NT + tid] = __int_as_float(q2.z);
                    if constexpr (NM > 3) S.m[3 * NT + tid] = __int_as_float(q2.w);
                    if constexpr (NM > 4) S.m[4 * NT + tid] = __int_as_float(q3.x);
                    if constexpr (NM > 5) S.m[5 * NT + tid] = __int_as_float(q3.y);
                    if constexpr (NM > 6) S.m[6 * NT + tid] = __int_as_float(q3.z);
                    if constexpr (NM > 7) S.m[7 * NT + tid] = __int_as_float(q3.w);
                }
                if constexpr (ZC) {
                    const int rad = q0.z, kcl = q0.w, kch = q1.x;
                    unsigned zw[NZW];
#pragma unroll
                    for (int q = 0; q < NZW; ++q) zw[q] = 0;
#pragma unroll
                    for (int sl = 0; sl < NS; ++sl) {
                        const int kA = t0 + 64 * sl, kB = kA + 63;
                        const unsigned z = (kcl <= kch && kA <= kch && kB >= kcl) ? 2u
                                           : (rad >= 0 && kA - kc <= rad && kc - kB <= rad) ? 1u : 0u;
                        zw[(2 * sl) / 32] |= z << ((2 * sl) % 32);
                    }
#pragma unroll
                    for (int q = 0; q < NZW; ++q) S.tf[q * NT + tid] = __uint_as_float(zw[q]);
                }
                if constexpr (!SEG) {
                    // 4-bit code per slice: zone (0 skip, 1 far, 2 mid, 3 core) | 4 (mask)
                    // | 8 (Vectorized Voigt: points beyond R)
                    const int gs = line_of(map, g);
                    const int klo = A.L.klo[gs], khi = A.L.khi[gs];
                    const int rad = q0.z, kcl = q0.w, kch = q1.x, flag = q1.y;
                    unsigned cw[NCW];
#pragma unroll
                    for (int q = 0; q < NCW; ++q) cw[q] = 0;
#pragma unroll
                    for (int sl = 0; sl < NS; ++sl) {
                        const int kA = t0 + 64 * sl, kB = kA + 63;
                        unsigned code = 0;
                        if (!(kB < klo || kA > khi)) {
                            const bool full = (kA >= klo && kB <= khi);
                            unsigned zone = 1, vvb = 0;
                            if (is_voigt(PROF)) {
                                if (kA <= kch && kB >= kcl) zone = 3;
                                else if (rad >= 0 && (int64_t)kA <= (int64_t)kc + rad &&
                                         (int64_t)kB >= (int64_t)kc - rad) zone = 2;
                                if (PROF == kVVoigt) {
                                    // 8: the slice may hold points beyond R (per-lane select);
                                    // zone 0 with 8: every point is beyond R
                                    const bool inside = (int64_t)kA >= (int64_t)kc - G.rvmin &&
                                                        (int64_t)kB <= (int64_t)kc + G.rvmin;
                                    const bool outside = (int64_t)kB < (int64_t)kc - G.rvmax ||
                                                         (int64_t)kA > (int64_t)kc + G.rvmax;
                                    if (!inside) vvb = 8u;
                                    if (outside) zone = 0u;
                                }
                            } else if (PROF == kLorentz || PROF == kGHSampled) {
                                zone = flag ? 1u : 0u;
                            } else if (PROF == kGHBinned || PROF == kLorentzBinned) {
                                zone = 1u;
                            } else {
                                zone = ((int64_t)kA <= (int64_t)kc + rad && (int64_t)kB >= (int64_t)kc - rad) ? 1u : 0u;
                            }
                            code = (zone | vvb) ? (zone | vvb | (full ? 0u : 4u)) : 0u;
                        }
                        cw[sl / 8] |= code << (4 * (sl % 8));
                    }
#pragma unroll
                    for (int q = 0; q < NCW; ++q) S.tf[q * NT + tid] = __uint_as_float(cw[q]);
                }
            }
        }
        __syncthreads();
        const float* rec = reinterpret_cast<const float*>(S.rec);
        const int be = bs + NT < b5 ? bs + NT : b5;
        for (int cs = bs; cs < be; cs += 64) {
            const int ce = cs + 64 < be ? cs + 64 : be;
            if constexpr (SEG) {
                if (is_voigt(PROF) || PROF == kLorentz) {
                    // ---- run 1: window ends inside the wave (upper mask)
                    const int lo = cs > s0 ? cs : s0, hi = ce < s1 ? ce : s1;
                    for (int l = lo; l < hi; ++l) {
                        const float* r = rec + (l - bs) * RS;
                        const float sb0 = S.sb0[l - bs], jhi = r[L::JHI];
#pragma unroll
                        for (int p = 0; p < P; ++p) {
                            const float j = jl[p] + sb0;
                            const float v = (PROF == kVoigt) ? v_far<PROF>(r, j) : (PROF == kVVoigt) ? v_vvw(r, j) : v_lor(r, j);
                            part[p] += (j <= jhi) ? v : 0.0f;
                        }
                    }
                    // ---- run 5: window starts inside the wave (lower mask)
                    const int lo5 = cs > s4 ? cs : s4, hi5 = ce < s5 ? ce : s5;
                    for (int l = lo5; l < hi5; ++l) {
                        const float* r = rec + (l - bs) * RS;
                        const float sb0 = S.sb0[l - bs], jlo = r[L::JLO];
#pragma unroll
                        for (int p = 0; p < P; ++p) {
                            const float j = jl[p] + sb0;
                            const float v = (PROF == kVoigt) ? v_far<PROF>(r, j) : (PROF == kVVoigt) ? v_vvw(r, j) : v_lor(r, j);
                            part[p] += (j >= jlo) ? v : 0.0f;
                        }
                    }
                    // ---- Vectorized Voigt: wing-only lines whose R boundary may fall on the
                    // wave (per-lane select between the 2-node rule and the reference wing)
                    if (PROF == kVVoigt) {
                        const int la = cs > ha ? cs : ha, lb = ce < hb ? ce : hb;
                        const int lc = cs > hc ? cs : hc, ld = ce < hd ? ce : hd;
                        for (int l = la; l < lb; ++l) {
                            const float* r = rec + (l - bs) * RS;
                            const float sb0 = S.sb0[l - bs], jvh = r[L::JVHI];
#pragma unroll
                            for (int p = 0; p < P; ++p) {
                                const float j = jl[p] + sb0;
                                part[p] += (j <= jvh) ? v_far<PROF>(r, j) : v_vvw(r, j);
                            }
                        }
                        for (int l = lc; l < ld; ++l) {
                            const float* r = rec + (l - bs) * RS;
                            const float sb0 = S.sb0[l - bs], jvl = r[L::JVLO];
#pragma unroll
                            for (int p = 0; p < P; ++p) {
                                const float j = jl[p] + sb0;
                                part[p] += (j >= jvl) ? v_far<PROF>(r, j) : v_vvw(r, j);
                            }
                        }
                    }
                    // ---- wing-only runs from the anchor, no branches (without the
                    // node-sampled lines)
                    {
                        const int lo2 = cs > hcl ? cs : hcl, hi2 = ce < s2 ? ce : s2;
                        const int lo4 = cs > s3 ? cs : s3, hi4 = ce < hcr ? ce : hcr;
                        // pieces: [lo2, xa) and [xd, hi4) beyond R (Vectorized Voigt) or beyond
                        // the far-wing radius (Voigt), [xb, hi2) and [lo4, xc) inside
                        const int xa = ce < ha ? ce : ha, xb0 = cs > hb ? cs : hb;
                        const int xc0 = ce < hc ? ce : hc, xd = cs > hd ? cs : hd;
                        const int xb = xb0 > lo2 ? xb0 : lo2, xc = xc0 < hi4 ? xc0 : hi4;
                        const float kl = (float)(wave * WW), kr = (float)(wave * WW + WW - 1);
                        if constexpr (!ANCH) {
                            wing_runs<PROF, P, RS, -1>(rec, S.sb0, kl, kr, bs, lo2, hi2, lo4, hi4, xa, xb, xc, xd, jlo_w,
                                                       jhi_w, part);
                        } else {
                            switch (wave) {
                                case 0: wing_runs<PROF, P, RS, RH + 0>(rec, S.sb0, kl, kr, bs, lo2, hi2, lo4, hi4, xa, xb, xc, xd, jlo_w, jhi_w, part); break;
                                case 1: wing_runs<PROF, P, RS, RH + (WAVES > 1 ? 1 : 0)>(rec, S.sb0, kl, kr, bs, lo2, hi2, lo4, hi4, xa, xb, xc, xd, jlo_w, jhi_w, part); break;
                                case 2: wing_runs<PROF, P, RS, RH + (WAVES > 2 ? 2 : 0)>(rec, S.sb0, kl, kr, bs, lo2, hi2, lo4, hi4, xa, xb, xc, xd, jlo_w, jhi_w, part); break;
                                case 3: wing_runs<PROF, P, RS, RH + (WAVES > 3 ? 3 : 0)>(rec, S.sb0, kl, kr, bs, lo2, hi2, lo4, hi4, xa, xb, xc, xd, jlo_w, jhi_w, part); break;
                                case 4: wing_runs<PROF, P, RS, RH + (WAVES > 4 ? 4 : 0)>(rec, S.sb0, kl, kr, bs, lo2, hi2, lo4, hi4, xa, xb, xc, xd, jlo_w, jhi_w, part); break;
                                case 5: wing_runs<PROF, P, RS, RH + (WAVES > 5 ? 5 : 0)>(rec, S.sb0, kl, kr, bs, lo2, hi2, lo4, hi4, xa, xb, xc, xd, jlo_w, jhi_w, part); break;
                                case 6: wing_runs<PROF, P, RS, RH + (WAVES > 6 ? 6 : 0)>(rec, S.sb0, kl, kr, bs, lo2, hi2, lo4, hi4, xa, xb, xc, xd, jlo_w, jhi_w, part); break;
                                default: wing_runs<PROF, P, RS, RH + (WAVES > 7 ? 7 : 0)>(rec, S.sb0, kl, kr, bs, lo2, hi2, lo4, hi4, xa, xb, xc, xd, jlo_w, jhi_w, part); break;
                            }
                        }
                    }
                }
                // ---- run 3: centre near the wave
                {
                    const int lo3 = cs > s2 ? cs : s2, hi3 = ce < s3 ? ce : s3;
                    if constexpr (PROF == kVoigt) {
                        // record words in registers for every slice, two lines at a time (one
                        // wait for both lines' LDS words), in passes of four lines whose
                        // core-value requests are issued first; each slice's rule adds
                        // straight into its sum
                        static_assert(L::H == 0 && L::C0 == 1 && L::C1 == 2 && L::AMP == 3 && L::B == 4 &&
                                      L::XC == 5, "layout");
                        constexpr unsigned zmask = P >= 16 ? 0xffffffffu : ((1u << (2 * P)) - 1u);
                        // a line's first slice with stored core values (P: none) and its values
                        // there (lanes clamped into the core range): requested for all lines of
                        // a pass before any is evaluated, so the requests overlap; a further
                        // core slice (cores wider than one slice) loads its own
                        auto core_first = [&](int i, unsigned zc, int& pc) {
                            const unsigned cm = (zc >> 1) & 0x55555555u;   // bit 2p: z = 2
                            pc = cm ? (int)(__builtin_ctz(cm) >> 1) : P;
                            float v = 0.0f;
                            if (cm) {
                                const float* rr = rec + i * RS;
                                const int kcl = CK_IN_REC ? __float_as_int(rr[CKW + 1]) : S.kcl[CK_IN_REC ? 0 : i];
                                const int kch = CK_IN_REC ? __float_as_int(rr[CKW + 2]) : S.kch[CK_IN_REC ? 0 : i];
                                const int k = w0 + 64 * pc + lane;
                                v = A.core_val[S.cb[i] + (k < kcl ? kcl : (k > kch ? kch : k))];
                            }
                            return v;
                        };
                        auto line3 = [&](int i, const float4 q, const float2 q2, float sb0, unsigned zc, float cpre,
                                         int pc) {
                            if (zc == 0u) {
                                // the mid zone (|z| < 40, which holds the core) misses the wave
#pragma unroll
                                for (int p = 0; p < P; ++p) {
                                    const float x = __builtin_fmaf(jl[p] + sb0, q.x, q2.y);
                                    const float pp = __builtin_fmaf(x, x, q.y);
                                    const float den = __builtin_fmaf(pp, pp, q.z);
                                    part[p] = __builtin_fmaf(__builtin_fmaf(pp, q.w, q2.x), __builtin_amdgcn_rcpf(den), part[p]);
                                }
                                return;
                            }
                            const float* rr = rec + i * RS;
                            const int kcl = CK_IN_REC ? __float_as_int(rr[CKW + 1]) : S.kcl[CK_IN_REC ? 0 : i];
                            const int kch = CK_IN_REC ? __float_as_int(rr[CKW + 2]) : S.kch[CK_IN_REC ? 0 : i];
                            const float csc = CK_IN_REC ? rr[CKW] : S.csc[CK_IN_REC ? 0 : i];
                            const Mid mc = mid_coef8(S.m + 8 * i);
#pragma unroll
                            for (int p = 0; p < P; ++p) {
                                const int kA = w0 + 64 * p;
                                const unsigned z = (zc >> (2 * p)) & 3u;
                                const float x = __builtin_fmaf(jl[p] + sb0, q.x, q2.y);
                                if (z == 0u) {
                                    const float pp = __builtin_fmaf(x, x, q.y);
                                    const float den = __builtin_fmaf(pp, pp, q.z);
                                    part[p] = __builtin_fmaf(__builtin_fmaf(pp, q.w, q2.x), __builtin_amdgcn_rcpf(den), part[p]);
                                } else if (z == 1u) {
                                    part[p] = mid_rule(mc, x * csc, part[p]);
                                } else {
                                    const int k = kA + lane;
                                    const bool in = (k >= kcl && k <= kch);
                                    float vcv;
                                    if (p == pc) {
                                        vcv = cpre;
                                    } else {
                                        const int kk = k < kcl ? kcl : (k > kch ? kch : k);
                                        vcv = A.core_val[S.cb[i] + kk];
                                    }
                                    const float vm = mid_rule(mc, x * csc, 0.0f);
                                    part[p] += in ? vcv : vm;
                                }
                            }
                        };
                        auto zcode = [&](int i) {
                            return (__builtin_amdgcn_readfirstlane(__float_as_uint(S.tf[zword * NT + i])) >> zshift) & zmask;
                        };
                        int l = lo3;
                        // four lines per pass: the four lines' core requests first, then the
                        // lines two at a time
                        for (; l + 3 < hi3; l += 4) {
                            const int i = l - bs;
                            const unsigned z0 = zcode(i), z1 = zcode(i + 1), z2 = zcode(i + 2), z3 = zcode(i + 3);
                            int p0, p1, p2, p3;
                            const float c0 = core_first(i, z0, p0), c1 = core_first(i + 1, z1, p1);
                            const float c2 = core_first(i + 2, z2, p2), c3 = core_first(i + 3, z3, p3);
#pragma unroll
                            for (int h = 0; h < 2; ++h) {
                                const int ih = i + 2 * h;
                                const float* r = rec + ih * RS;
                                const float4 qa = *reinterpret_cast<const float4*>(r);
                                const float2 qa2 = *reinterpret_cast<const float2*>(r + L::B);
                                const float4 qb = *reinterpret_cast<const float4*>(r + RS);
                                const float2 qb2 = *reinterpret_cast<const float2*>(r + RS + L::B);
                                const float sa = S.sb0[ih], sb = S.sb0[ih + 1];
                                line3(ih, qa, qa2, sa, h ? z2 : z0, h ? c2 : c0, h ? p2 : p0);
                                line3(ih + 1, qb, qb2, sb, h ? z3 : z1, h ? c3 : c1, h ? p3 : p1);
                            }
                        }
                        for (; l + 1 < hi3; l += 2) {
                            const int i = l - bs;
                            const float* r = rec + i * RS;
                            const float4 qa = *reinterpret_cast<const float4*>(r);
                            const float2 qa2 = *reinterpret_cast<const float2*>(r + L::B);
                            const float4 qb = *reinterpret_cast<const float4*>(r + RS);
                            const float2 qb2 = *reinterpret_cast<const float2*>(r + RS + L::B);
                            const float sa = S.sb0[i], sb = S.sb0[i + 1];
                            const unsigned za = zcode(i), zb = zcode(i + 1);
                            int pa, pb;
                            const float ca = core_first(i, za, pa), cb = core_first(i + 1, zb, pb);
                            line3(i, qa, qa2, sa, za, ca, pa);
                            line3(i + 1, qb, qb2, sb, zb, cb, pb);
                        }
                        if (l < hi3) {
                            const int i = l - bs;
                            const float* r = rec + i * RS;
                            const unsigned z1 = zcode(i);
                            int p1;
                            const float c1 = core_first(i, z1, p1);
                            line3(i, *reinterpret_cast<const float4*>(r), *reinterpret_cast<const float2*>(r + L::B),
                                  S.sb0[i], z1, c1, p1);
                        }
                    } else
                    for (int l = lo3; l < hi3; ++l) {
                        const int i = l - bs;
                        const float* r = rec + i * RS;
                        const float sb0 = S.sb0[i];
                        if (PROF == kLorentz) {
#pragma unroll
                            for (int p = 0; p < P; ++p) part[p] += v_lor(r, jl[p] + sb0);
                            continue;
                        }
                        // scalar copies of the line's integer geometry; distances from the
                        // centre to grid points stay inside int (grid plus halo < 2^31)
                        const int kc = __builtin_amdgcn_readfirstlane(S.kc[i]);
                        const int rad = __builtin_amdgcn_readfirstlane(S.rad[i]);
                        if (PROF == kVoigt && !(rad >= 0 && w0 - kc <= rad && kc - w1 <= rad)) {
                            // the line's mid zone (|z| < 40, which holds its core) misses the wave:
                            // every point takes the far rule, as the per-slice tests below would
#pragma unroll
                            for (int p = 0; p < P; ++p) part[p] += v_far<PROF>(r, jl[p] + sb0);
                            continue;
                        }
                        const int kcl = __builtin_amdgcn_readfirstlane(S.kcl[i]);
                        const int kch = __builtin_amdgcn_readfirstlane(S.kch[i]);
                        const float csc = S.csc[i];
                        const Mid mc = mid_coef<NT>(S.m + i);
#pragma unroll
                        for (int p = 0; p < P; ++p) {
                            const int kA = w0 + 64 * p, kB = kA + 63;
                            const float j = jl[p] + sb0;
                            const bool nearz = rad >= 0 && kA - kc <= rad && kc - kB <= rad;
                            if (is_voigt(PROF)) {
                                float v;
                                if (kA <= kch && kB >= kcl) {
                                    // stored core values: loaded and consumed inside this branch
                                    // (a load left in flight past it would make the next wing
                                    // loop wait for every outstanding load, the prefetch too)
                                    const int k = kA + lane;
                                    const bool in = (k >= kcl && k <= kch);
                                    float vcv = 0.0f;
                                    if (in) vcv = A.core_val[S.cb[i] + k];
                                    const float vm = v_mid<PROF>(r, mc, csc, j);
                                    v = in ? vcv : vm;
                                } else if (nearz) {
                                    v = v_mid<PROF>(r, mc, csc, j);
                                } else {
                                    v = v_far<PROF>(r, j);
                                }
                                if (PROF == kVVoigt) {
                                    const bool inr = (j >= r[L::JVLO]) && (j <= r[L::JVHI]);
                                    const float w = v_vvw(r, j);
                                    v = inr ? v : w;
                                }
                                part[p] += v;
                            } else {
                                if (nearz) part[p] += v_gauss(r, j);
                            }
                        }
                    }
                }
            } else {
                // ---- coded sweep: every line carries per-slice codes
                for (int l = cs; l < ce; ++l) {
                    const int i = l - bs;
                    const float* r = rec + i * RS;
                    const unsigned cw =
                        __builtin_amdgcn_readfirstlane(__float_as_uint(S.tf[cword * NT + i])) >> cshift;
                    if ((cw & (P >= 8 ? 0xffffffffu : ((1u << (4 * P)) - 1u))) == 0u) continue;
                    const float sb0 = S.sb0[i], jlo = r[L::JLO], jhi = r[L::JHI];
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        const unsigned z = (cw >> (4 * p)) & 15u;
                        const unsigned zone = z & 3u;
                        if (z == 0u) continue;
                        const float j = jl[p] + sb0;
                        float v = 0.0f;
                        if (is_voigt(PROF)) {
                            if (zone == 1u) {
                                v = v_far<PROF>(r, j);
                            } else if (zone != 0u) {
                                const float vm = v_mid<PROF>(r, mid_coef<NT>(S.m + i), S.csc[i], j);
                                if (zone == 2u) {
                                    v = vm;
                                } else {
                                    // core slice: stored value inside [kcl, kch], 4-node rule elsewhere
                                    const int k = w0 + 64 * p + lane;
                                    const int kcl = S.kcl[i], kch = S.kch[i];
                                    const bool in = (k >= kcl) && (k <= kch);
                                    float vcore = 0.0f;
                                    if (in) vcore = A.core_val[S.cb[i] + k];
                                    v = in ? vcore : vm;
                                }
                            }
                            if (PROF == kVVoigt && (z & 8u)) {
                                const bool inr = (j >= r[L::JVLO]) && (j <= r[L::JVHI]);
                                const float w = v_vvw(r, j);
                                v = inr ? v : w;
                            }
                        } else if (PROF == kLorentz) {
                            v = v_lor(r, j);
                        } else if (PROF == kGHSampled) {
                            v = v_ghs<NT>(A.tab, r, S.m + i, j);
                        } else if (PROF == kGHBinned) {
                            v = v_ghb<NT>(A.tab, r, S.m + i, j);
                        } else if (PROF == kLorentzBinned) {
                            if (fabsf(j) > 1.0f) {
                                const float D = __builtin_fmaf(j, r[LD::H], r[LD::XC]);
                                v = r[LD::AMP] * atan2f(S.m[i], __builtin_fmaf(D, D, S.m[NT + i]));
                            } else {
                                // bins next to the centre: (D - dnu/2)(D + dnu/2) + gamma^2 in double
                                const double dd =
                                    __hiloint2double(__float_as_int(S.m[3 * NT + i]), __float_as_int(S.m[2 * NT + i]));
                                const double gg =
                                    __hiloint2double(__float_as_int(S.m[5 * NT + i]), __float_as_int(S.m[4 * NT + i]));
                                const double lo = __builtin_fma((double)j - 0.5, G.dnu, dd);
                                const double hi = __builtin_fma((double)j + 0.5, G.dnu, dd);
                                v = r[LD::AMP] * (float)atan2(G.dnu * gg, __builtin_fma(lo, hi, gg * gg));
                            }
                        } else if (PROF == kDopplerBinned) {
                            const double dd = __hiloint2double(__float_as_int(S.m[NT + i]), __float_as_int(S.m[i]));
                            const double ss =
                                __hiloint2double(__float_as_int(S.m[3 * NT + i]), __float_as_int(S.m[2 * NT + i]));
                            const double D = __builtin_fma((double)j, G.dnu, dd);
                            v = r[LD::AMP] * (float)erf_diff64(ss * (D - 0.5 * G.dnu), ss * (D + 0.5 * G.dnu));
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
    constexpr bool CAN_SEG = PROF <= kVoigt || PROF == kVVoigt;
    if (CAN_SEG && a.seg) hipLaunchKernelGGL((fwd_f32_kernel<PROF, WAVES, P, CAN_SEG>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((fwd_f32_kernel<PROF, WAVES, P, false>), grid, block, 0, s, a);
}

template <int PROF>
void launch_p(int waves, int P, const FwdArgs& a, hipStream_t s) {
    if (waves == 1) {
        switch (P) {
            case 1: launch_one<PROF, 1, 1>(a, s); break;
            case 2: launch_one<PROF, 1, 2>(a, s); break;
            case 8: launch_one<PROF, 1, 8>(a, s); break;
            default: launch_one<PROF, 1, 4>(a, s); break;
        }
    } else if (waves == 2) {
        switch (P) {
            case 1: launch_one<PROF, 2, 1>(a, s); break;
            case 2: launch_one<PROF, 2, 2>(a, s); break;
            case 8: launch_one<PROF, 2, 8>(a, s); break;
            default: launch_one<PROF, 2, 4>(a, s); break;
        }
    } else if (waves == 4) {
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

hipError_t launch_records(int profile, const RecArgs& a, hipStream_t s) {
    if (a.n_lines <= 0) return hipSuccess;
    const dim3 grid((unsigned)((a.n_lines + 255) / 256)), block(256);
    switch (profile) {
        case kDoppler: hipLaunchKernelGGL(record_kernel<kDoppler>, grid, block, 0, s, a); break;
        case kGaussFixed: hipLaunchKernelGGL(record_kernel<kGaussFixed>, grid, block, 0, s, a); break;
        case kLorentz: hipLaunchKernelGGL(record_kernel<kLorentz>, grid, block, 0, s, a); break;
        case kGHSampled: hipLaunchKernelGGL(record_kernel<kGHSampled>, grid, block, 0, s, a); break;
        case kGHBinned: hipLaunchKernelGGL(record_kernel<kGHBinned>, grid, block, 0, s, a); break;
        case kVVoigt: hipLaunchKernelGGL(record_kernel<kVVoigt>, grid, block, 0, s, a); break;
        case kDopplerBinned: hipLaunchKernelGGL(record_kernel<kDopplerBinned>, grid, block, 0, s, a); break;
        case kLorentzBinned: hipLaunchKernelGGL(record_kernel<kLorentzBinned>, grid, block, 0, s, a); break;
        default: hipLaunchKernelGGL(record_kernel<kVoigt>, grid, block, 0, s, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_forward_f32(int profile, int waves, int P, const FwdArgs& a, hipStream_t s) {
    if (a.n_tiles <= 0) return hipSuccess;
    switch (profile) {
        case kDoppler: launch_p<kDoppler>(waves, P, a, s); break;
        case kGaussFixed: launch_p<kGaussFixed>(waves, P, a, s); break;
        case kLorentz: launch_p<kLorentz>(waves, P, a, s); break;
        case kGHSampled: launch_p<kGHSampled>(waves, P, a, s); break;
        case kGHBinned: launch_p<kGHBinned>(waves, P, a, s); break;
        case kVVoigt: launch_p<kVVoigt>(waves, P, a, s); break;
        case kDopplerBinned: launch_p<kDopplerBinned>(waves, P, a, s); break;
        case kLorentzBinned: launch_p<kLorentzBinned>(waves, P, a, s); break;
        default: launch_p<kVoigt>(waves, P, a, s); break;
    }
    return hipGetLastError();
}

}  // namespace xs
