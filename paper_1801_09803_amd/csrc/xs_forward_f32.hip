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
//
// Voigt zones (|z| = |x + iy|): wings |z| >= 40 use the 2-node Gauss-Hermite rational
// (6 FMA + 1 reciprocal per point); 8 <= |z| < 40 the 4-node rule; points with |z| < 8
// take the value the double-precision core pre-pass stored for them.
// x is formed as fma(j, h, xc) from the exact integer offset j = k - kc, or in the wing
// runs as fma(k - k_anchor, h, x_anchor) from an anchor at the wavefront end nearest the
// centre (computed in double), so its relative error stays ~1e-7 however far the point is
// from the centre.  Partial sums are flushed every 64 lines into a compensated (TwoSum) pair.
#include "xs_forward_common.hpp"

namespace xs {

namespace {

// hot record words
enum : int { H_H = 0, H_C0 = 1, H_C1 = 2, H_AMP = 3, H_B = 4, H_XC = 5, H_JLO = 6, H_JHI = 7 };
// cold record words (ints unless noted; C_CBASE is int64, C_M 8 floats)
enum : int { C_CSC = 0, C_KC = 1, C_RAD = 2, C_KCL = 3, C_KCH = 4, C_FLAG = 5, C_CBASE = 6, C_M = 8 };
constexpr int kHot = 8;
constexpr int kCold = 16;

// ------------------------------------------------------------------ record kernel
template <int PROF>
__global__ __launch_bounds__(256) void record_kernel(const RecArgs A) {
    const int g = blockIdx.x * 256 + threadIdx.x;
    if (g >= A.n_lines) return;
    const TPParam tp = *A.tp;
    const Geometry G = A.G;
    const double Q = A.Q[tp.iq];
    const double nu = A.L.nu[g];
    const int kc = A.L.kc[g], klo = A.L.klo[g], khi = A.L.khi[g];
    // Eq. 1: I = [g_f A/(8 pi c nu^2)] exp(-c2 E_i/T) (1 - exp(-c2 nu/T)) / Q(T)
    const double S = A.L.cA[g] * exp(-(kC2 * A.L.elow[g]) / tp.T) * (-expm1(-(kC2 * nu) / tp.T)) / Q;
    const double aD = nu * tp.beta;                                                               // Eq. 16
    const double gam = (double)A.L.gref[g] * exp((double)A.L.nexp[g] * tp.ln_T0_T) * tp.p_over_p0;  // Eq. 18
    const double d = (G.nu_a + (double)kc * G.dnu) - nu;   // centre offset nu_kc - nu
    float h[kHot];
    int c[kCold];
    float* cf = reinterpret_cast<float*>(c);
#pragma unroll
    for (int i = 0; i < kHot; ++i) h[i] = 0.0f;
#pragma unroll
    for (int i = 0; i < kCold; ++i) c[i] = 0;
    h[H_JLO] = (float)(klo - kc);
    h[H_JHI] = (float)(khi - kc);
    c[C_KC] = kc;
    c[C_RAD] = -1;
    c[C_KCH] = -1;
    double scale;
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
        scale = s * sc;
        h[H_XC] = (float)(scale * d);
        h[H_H] = (float)(scale * G.dnu);
        h[H_C0] = (float)((y2 - 0.5) * sc2);
        h[H_C1] = (float)(2.0 * y2 * sc2 * sc2);
        h[H_AMP] = (float)(ampf * sc2);
        h[H_B] = (float)(ampf * sc2 * sc2);
        cf[C_CSC] = (float)ldexp(1.0, e);
#pragma unroll
        for (int jp = 0; jp < 2; ++jp) {
            const double t2 = A.tab->gh4.t[jp] * A.tab->gh4.t[jp];
            const double Aj = a * (y / kPI) * 2.0 * A.tab->gh4.w[jp];
            cf[C_M + 4 * jp + 0] = (float)(y2 - t2);
            cf[C_M + 4 * jp + 1] = (float)(4.0 * t2 * y2);
            cf[C_M + 4 * jp + 2] = (float)Aj;
            cf[C_M + 4 * jp + 3] = (float)(Aj * 2.0 * t2);
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
        h[H_XC] = (float)(d * ig);
        h[H_H] = (float)(G.dnu * ig);
        h[H_AMP] = (float)(S * ig * (1.0 / kPI));
        c[C_FLAG] = gam > 0.0 ? 1 : 0;
    } else if (PROF == kGHSampled || PROF == kGHBinned) {
        // Gauss-Hermite convolution (Eq. 30-31 as read): nodes shift the Lorentzian by
        // delta_j = alpha_D t_j / sqrt(ln 2); work in wavenumber units D = nu_k - nu
        scale = 1.0;
        h[H_XC] = (float)d;
        h[H_H] = (float)G.dnu;
        cf[C_M + 0] = (float)(gam * gam);
        cf[C_M + 1] = (float)(aD / kSQRT_LN2);
        if (PROF == kGHSampled) {
            h[H_AMP] = (float)(S * gam / (kPI * 1.7724538509055160273));   // S gamma / pi^(3/2)
            cf[C_M + 2] = (float)(4.0 * gam * gam);
        } else {
            h[H_AMP] = (float)(S / (kPI * 1.7724538509055160273 * G.dnu));   // S / (pi^(3/2) dnu)
            cf[C_M + 3] = (float)(G.dnu * gam);
            cf[C_M + 4] = (float)(gam * gam - 0.25 * G.dnu * G.dnu);
        }
        c[C_FLAG] = gam > 0.0 ? 1 : 0;
    } else {
        // Gaussian (Eq. 15); x scaled by sqrt(1/ln 2) so exp(-x^2) = exp2(-x'^2)
        const double alpha = (PROF == kDoppler) ? aD : A.alpha_fixed;
        const double s = kSQRT_LN2 / alpha;
        scale = s * 1.2011224087864498;
        h[H_XC] = (float)(scale * d);
        h[H_H] = (float)(scale * G.dnu);
        h[H_AMP] = (float)(S * kSQRT_LN2_PI / alpha);
        c[C_RAD] = radius_steps(10.5, s * G.dnu, s * d);   // exp(-x^2) underflows beyond
    }
    float4* ho = reinterpret_cast<float4*>(A.hot + (int64_t)g * kHot);
    ho[0] = make_float4(h[0], h[1], h[2], h[3]);
    ho[1] = make_float4(h[4], h[5], h[6], h[7]);
    int4* co = reinterpret_cast<int4*>(A.cold + (int64_t)g * kCold);
#pragma unroll
    for (int q = 0; q < 4; ++q) co[q] = make_int4(c[4 * q], c[4 * q + 1], c[4 * q + 2], c[4 * q + 3]);
    A.xscale[g] = scale;
}

// ------------------------------------------------------------------ tile kernel
// LDS image of one batch: line records of RS words (the 8 hot words, then for the
// segmented sweep one anchor per wavefront, so a wing-loop line is read from one base
// address), the grid offset, slice codes (coded sweep) and the cold fields (one array
// per field, indexed by the line's place in the batch).
template <int NT, int RS, int NTF>
struct Lds {
    float4 rec[NT * RS / 4];
    float sb0[NT];          // t0 - kc
    float tf[NTF * NT];     // slice-code words (coded sweep)
    float csc[NT];
    int kc[NT], rad[NT], kcl[NT], kch[NT];
    long long cb[NT];
    float m[8 * NT];
};

// wing formula (2-node rule, scaled variables)
__device__ __forceinline__ float v_far(const float* r, float j) {
    const float x = __builtin_fmaf(j, r[H_H], r[H_XC]);
    const float pp = __builtin_fmaf(x, x, r[H_C0]);
    const float den = __builtin_fmaf(pp, pp, r[H_C1]);
    const float num = __builtin_fmaf(pp, r[H_AMP], r[H_B]);
    return num * __builtin_amdgcn_rcpf(den);
}

// 4-node rule (unscaled x); m points at the line's first coefficient, stride NT
template <int NT>
__device__ __forceinline__ float v_mid(const float* r, const float* m, float csc, float j) {
    const float x = __builtin_fmaf(j, r[H_H], r[H_XC]) * csc;
    const float p1 = __builtin_fmaf(x, x, m[0 * NT]);
    const float p2 = __builtin_fmaf(x, x, m[4 * NT]);
    const float d1 = __builtin_fmaf(p1, p1, m[1 * NT]);
    const float d2 = __builtin_fmaf(p2, p2, m[5 * NT]);
    const float n1 = __builtin_fmaf(p1, m[2 * NT], m[3 * NT]);
    const float n2 = __builtin_fmaf(p2, m[6 * NT], m[7 * NT]);
    return __builtin_fmaf(n1, __builtin_amdgcn_rcpf(d1), n2 * __builtin_amdgcn_rcpf(d2));
}

__device__ __forceinline__ float v_lor(const float* r, float j) {
    const float x = __builtin_fmaf(j, r[H_H], r[H_XC]);
    return r[H_AMP] * __builtin_amdgcn_rcpf(__builtin_fmaf(x, x, 1.0f));
}

// Gauss-Hermite sum of shifted Lorentzians, node pairs +-t_j:
// L(D - dj) + L(D + dj) = (gamma/pi) 2 (D^2 + g^2 + dj^2) / ((D^2 + g^2 - dj^2)^2 + 4 dj^2 g^2)
template <int NT>
__device__ __forceinline__ float v_ghs(const Tables* tab, const float* r, const float* m, float j) {
    const float D = __builtin_fmaf(j, r[H_H], r[H_XC]);
    const float g2 = m[0], ad = m[NT], g4 = m[2 * NT];
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
    return r[H_AMP] * acc;
}

// bin-averaged Gauss-Hermite Voigt: atan(y+) - atan(y-) = atan2(dnu g, (D - dj)^2 + g^2 - dnu^2/4)
template <int NT>
__device__ __forceinline__ float v_ghb(const Tables* tab, const float* r, const float* m, float j) {
    const float D = __builtin_fmaf(j, r[H_H], r[H_XC]);
    const float ad = m[NT], hg = m[3 * NT], c = m[4 * NT];
    float acc = 0.0f;
    for (int q = 0; q < kGHConv; ++q) {
        const float e = D - ad * tab->tconvf[q];
        acc = __builtin_fmaf(tab->wconvf[q], atan2f(hg, __builtin_fmaf(e, e, c)), acc);
    }
    return r[H_AMP] * acc;
}

__device__ __forceinline__ float v_gauss(const float* r, float j) {
    const float x = __builtin_fmaf(j, r[H_H], r[H_XC]);
    return r[H_AMP] * __builtin_amdgcn_exp2f(-x * x);
}

// Branch-free wing loop over sorted lines [lo, hi) of the batch starting at bs:
// x = anchor + (k - k_anchor) h, with jd[p] = k - k_anchor of this lane's points; the
// anchor of this wavefront is word ia of the line record.
template <int PROF, int P, int RS, int IA>
__device__ __forceinline__ void wing_run(const float* rec, int bs, int lo, int hi, const float (&jd)[P],
                                         float (&part)[P]) {
#pragma unroll 2
    for (int l = lo; l < hi; ++l) {
        const float* r = rec + (l - bs) * RS;
        const float4 h0 = *reinterpret_cast<const float4*>(r);
        const float xa = r[IA];
        const float h = h0.x;
        if (PROF == kVoigt) {
            const float c0 = h0.y, c1 = h0.z, amp = h0.w, bb = r[H_B];
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const float x = __builtin_fmaf(jd[p], h, xa);
                const float pp = __builtin_fmaf(x, x, c0);
                const float den = __builtin_fmaf(pp, pp, c1);
                const float num = __builtin_fmaf(pp, amp, bb);
                part[p] = __builtin_fmaf(num, __builtin_amdgcn_rcpf(den), part[p]);
            }
        } else {
            const float amp = h0.w;
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const float x = __builtin_fmaf(jd[p], h, xa);
                part[p] = __builtin_fmaf(amp, __builtin_amdgcn_rcpf(__builtin_fmaf(x, x, 1.0f)), part[p]);
            }
        }
    }
}

// Both wing-only runs of wavefront WV (its anchor word is a compile-time offset).
template <int PROF, int P, int RS, int WV>
__device__ __forceinline__ void wing_runs(const float* rec, int bs, int lo2, int hi2, int lo4, int hi4,
                                          const float (&jlo_w)[P], const float (&jhi_w)[P], float (&part)[P]) {
    wing_run<PROF, P, RS, kHot + WV>(rec, bs, lo2, hi2, jlo_w, part);
    wing_run<PROF, P, RS, kHot + WV>(rec, bs, lo4, hi4, jhi_w, part);
}

// The next batch's global data of one thread: two float4 of the hot records (chunks
// tid and NT + tid of the batch) and its own line's offset data.
struct Prefetch {
    float4 h0, h1;
    int kc;
    double nu, scale;
};

template <int NT>
__device__ __forceinline__ Prefetch load_batch(const FwdArgs& A, const float4* ghot, const double* gscale, int bs,
                                               int b5, int tid) {
    Prefetch f;
    f.h0 = make_float4(0.f, 0.f, 0.f, 0.f);
    f.h1 = f.h0;
    f.kc = 0;
    f.nu = 0.0;
    f.scale = 0.0;
    const int64_t c0 = 2 * (int64_t)bs + tid, c1 = c0 + NT, cend = 2 * (int64_t)b5;
    if (c0 < cend) f.h0 = ghot[c0];
    if (c1 < cend) f.h1 = ghot[c1];
    const int g = bs + tid;
    if (g < b5) {
        f.kc = A.L.kc[g];
        f.nu = A.L.nu[g];
        f.scale = gscale[g];
    }
    return f;
}

template <int PROF, int WAVES, int P, bool SEG>
__global__ __launch_bounds__(64 * WAVES) void fwd_f32_kernel(const FwdArgs A) {
    constexpr int NT = 64 * WAVES;       // threads = lines per LDS batch
    constexpr int W = NT * P;            // grid points per tile
    constexpr int WW = 64 * P;           // grid points per wavefront
    constexpr int NS = WAVES * P;        // slices per tile
    constexpr int NCW = (NS + 7) / 8;    // code words (4 bits per slice)
    constexpr int RS = SEG ? kHot + WAVES : kHot;   // LDS record words
    constexpr int NTF = SEG ? 1 : NCW;
    __shared__ Lds<NT, RS, NTF> S;

    const Geometry G = A.G;
    // the wavefront index is uniform within a wavefront: keep it (and everything derived
    // from it: run bounds, loop counters, LDS offsets) in scalar registers
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const WorkItem wi = work_item(A);
    const TPParam tp = A.tps[wi.tp];
    const int64_t row = (int64_t)wi.tp * A.rec_stride;
    const float4* ghot = reinterpret_cast<const float4*>(A.hot + row * kHot);
    const int4* gcold = reinterpret_cast<const int4*>(A.cold + row * kCold);
    const double* gscale = A.xscale + row;
    const int t0 = wi.tile * W, t1 = t0 + W - 1;
    const int w0 = t0 + wave * WW, w1 = w0 + WW - 1;

    // lines overlapping the tile; this workgroup takes every n_split-th batch of them
    const int b0 = off_at(A.off, (int64_t)t0 - G.hmax, G);
    const int b5 = off_at(A.off, (int64_t)t1 + G.hmax + 1, G);
    const int bstride = NT * A.n_split;
    const int bfirst = b0 + NT * wi.part;
    const int rm_tile = tp.rm;
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

    Prefetch nxt = load_batch<NT>(A, ghot, gscale, bfirst, b5, tid);
    for (int bs = bfirst; bs < b5; bs += bstride) {
        const int g = bs + tid;
        // ---- batch set-up: hot records (coalesced loads; chunk c is half c%2 of line
        // c/2), then this thread's line
        if (2 * (int64_t)bs + tid < 2 * (int64_t)b5) S.rec[(tid >> 1) * (RS / 4) + (tid & 1)] = nxt.h0;
        if (2 * (int64_t)bs + NT + tid < 2 * (int64_t)b5)
            S.rec[(NT / 2 + (tid >> 1)) * (RS / 4) + (tid & 1)] = nxt.h1;
        if (g < b5) {
            const int kc = nxt.kc;
            S.sb0[tid] = (float)(t0 - kc);
            if (SEG) {
                // x at the end of each wavefront's range nearest the centre: wing points are
                // then x = anchor + (k - k_anchor) h with both terms of one sign
                const double d = (G.nu_a + (double)kc * G.dnu) - nxt.nu;
                const double hd = nxt.scale * G.dnu, xd = nxt.scale * d;
#pragma unroll
                for (int wv = 0; wv < WAVES; ++wv) {
                    const int wa = t0 + WW * wv;
                    const int ka = wa > kc ? wa : wa + WW - 1;
                    reinterpret_cast<float*>(S.rec)[tid * RS + kHot + wv] =
                        (float)__builtin_fma((double)(ka - kc), hd, xd);
                }
            }
            // cold fields for lines whose centre can be near the tile (every line for
            // the coded sweep)
            const bool near = !SEG || (PROF != kLorentz && (int64_t)kc >= (int64_t)t0 - rm_tile &&
                                       (int64_t)kc <= (int64_t)t1 + rm_tile);
            if (near) {
                const int4* cg = gcold + (int64_t)g * (kCold / 4);
                const int4 q0 = cg[0], q1 = cg[1], q2 = cg[2], q3 = cg[3];
                S.csc[tid] = __int_as_float(q0.x);
                S.kc[tid] = q0.y;
                S.rad[tid] = q0.z;
                S.kcl[tid] = q0.w;
                S.kch[tid] = q1.x;
                S.cb[tid] = (long long)(((unsigned long long)(unsigned)q1.w << 32) | (unsigned)q1.z);
                S.m[0 * NT + tid] = __int_as_float(q2.x);
                S.m[1 * NT + tid] = __int_as_float(q2.y);
                S.m[2 * NT + tid] = __int_as_float(q2.z);
                S.m[3 * NT + tid] = __int_as_float(q2.w);
                S.m[4 * NT + tid] = __int_as_float(q3.x);
                S.m[5 * NT + tid] = __int_as_float(q3.y);
                S.m[6 * NT + tid] = __int_as_float(q3.z);
                S.m[7 * NT + tid] = __int_as_float(q3.w);
                if (!SEG) {
                    // 4-bit code per slice: zone (0 skip, 1 far, 2 mid, 3 core) | 4 (mask)
                    const int klo = A.L.klo[g], khi = A.L.khi[g];
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
                            unsigned zone = 1;
                            if (PROF == kVoigt) {
                                if (kA <= kch && kB >= kcl) zone = 3;
                                else if (rad >= 0 && (int64_t)kA <= (int64_t)kc + rad &&
                                         (int64_t)kB >= (int64_t)kc - rad) zone = 2;
                            } else if (PROF == kLorentz || PROF == kGHSampled) {
                                zone = flag ? 1u : 0u;
                            } else if (PROF == kGHBinned) {
                                zone = 1u;
                            } else {
                                zone = ((int64_t)kA <= (int64_t)kc + rad && (int64_t)kB >= (int64_t)kc - rad) ? 1u : 0u;
                            }
                            code = zone ? (zone | (full ? 0u : 4u)) : 0u;
                        }
                        cw[sl / 8] |= code << (4 * (sl % 8));
                    }
#pragma unroll
                    for (int q = 0; q < NCW; ++q) S.tf[q * NT + tid] = __uint_as_float(cw[q]);
                }
            }
        }
        __syncthreads();
        if (bs + bstride < b5) nxt = load_batch<NT>(A, ghot, gscale, bs + bstride, b5, tid);   // overlaps the sweep
        const float* rec = reinterpret_cast<const float*>(S.rec);
        const int be = bs + NT < b5 ? bs + NT : b5;
        for (int cs = bs; cs < be; cs += 64) {
            const int ce = cs + 64 < be ? cs + 64 : be;
            if (SEG) {
                if (PROF == kVoigt || PROF == kLorentz) {
                    // ---- run 1: window ends inside the wave (upper mask)
                    const int lo = cs > s0 ? cs : s0, hi = ce < s1 ? ce : s1;
                    for (int l = lo; l < hi; ++l) {
                        const float* r = rec + (l - bs) * RS;
                        const float sb0 = S.sb0[l - bs], jhi = r[H_JHI];
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
                        const float* r = rec + (l - bs) * RS;
                        const float sb0 = S.sb0[l - bs], jlo = r[H_JLO];
#pragma unroll
                        for (int p = 0; p < P; ++p) {
                            const float j = jl[p] + sb0;
                            const float v = (PROF == kVoigt) ? v_far(r, j) : v_lor(r, j);
                            part[p] += (j >= jlo) ? v : 0.0f;
                        }
                    }
                    // ---- runs 2 and 4: wing formula from the anchor, no branches
                    {
                        const int lo2 = cs > s1 ? cs : s1, hi2 = ce < s2 ? ce : s2;
                        const int lo4 = cs > s3 ? cs : s3, hi4 = ce < s4 ? ce : s4;
                        switch (wave) {
                            case 0: wing_runs<PROF, P, RS, 0>(rec, bs, lo2, hi2, lo4, hi4, jlo_w, jhi_w, part); break;
                            case 1: wing_runs<PROF, P, RS, 1>(rec, bs, lo2, hi2, lo4, hi4, jlo_w, jhi_w, part); break;
                            case 2: wing_runs<PROF, P, RS, 2>(rec, bs, lo2, hi2, lo4, hi4, jlo_w, jhi_w, part); break;
                            case 3: wing_runs<PROF, P, RS, 3>(rec, bs, lo2, hi2, lo4, hi4, jlo_w, jhi_w, part); break;
                            case 4: wing_runs<PROF, P, RS, (WAVES > 4 ? 4 : 0)>(rec, bs, lo2, hi2, lo4, hi4, jlo_w, jhi_w, part); break;
                            case 5: wing_runs<PROF, P, RS, (WAVES > 5 ? 5 : 0)>(rec, bs, lo2, hi2, lo4, hi4, jlo_w, jhi_w, part); break;
                            case 6: wing_runs<PROF, P, RS, (WAVES > 6 ? 6 : 0)>(rec, bs, lo2, hi2, lo4, hi4, jlo_w, jhi_w, part); break;
                            default: wing_runs<PROF, P, RS, (WAVES > 7 ? 7 : 0)>(rec, bs, lo2, hi2, lo4, hi4, jlo_w, jhi_w, part); break;
                        }
                    }
                }
                // ---- run 3: centre near the wave
                {
                    const int lo3 = cs > s2 ? cs : s2, hi3 = ce < s3 ? ce : s3;
                    for (int l = lo3; l < hi3; ++l) {
                        const int i = l - bs;
                        const float* r = rec + i * RS;
                        const float sb0 = S.sb0[i];
                        if (PROF == kLorentz) {
#pragma unroll
                            for (int p = 0; p < P; ++p) part[p] += v_lor(r, jl[p] + sb0);
                            continue;
                        }
                        // scalar copies of the line's integer geometry
                        const int kc = __builtin_amdgcn_readfirstlane(S.kc[i]);
                        const int rad = __builtin_amdgcn_readfirstlane(S.rad[i]);
                        const int kcl = __builtin_amdgcn_readfirstlane(S.kcl[i]);
                        const int kch = __builtin_amdgcn_readfirstlane(S.kch[i]);
                        const float csc = S.csc[i];
#pragma unroll
                        for (int p = 0; p < P; ++p) {
                            const int kA = w0 + 64 * p, kB = kA + 63;
                            const float j = jl[p] + sb0;
                            const bool nearz = rad >= 0 && (int64_t)kA <= (int64_t)kc + rad &&
                                               (int64_t)kB >= (int64_t)kc - rad;
                            if (PROF == kVoigt) {
                                if (kA <= kch && kB >= kcl) {
                                    // stored core values: loaded and consumed inside this branch
                                    // (a load left in flight past it would make the next wing
                                    // loop wait for every outstanding load, the prefetch too)
                                    const int k = kA + lane;
                                    const bool in = (k >= kcl && k <= kch);
                                    float vcv = 0.0f;
                                    if (in) vcv = A.core_val[S.cb[i] + k];
                                    const float vm = v_mid<NT>(r, S.m + i, csc, j);
                                    part[p] += in ? vcv : vm;
                                } else if (nearz) {
                                    part[p] += v_mid<NT>(r, S.m + i, csc, j);
                                } else {
                                    part[p] += v_far(r, j);
                                }
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
                    if ((cw & ((1u << (4 * P)) - 1u)) == 0u) continue;
                    const float sb0 = S.sb0[i], jlo = r[H_JLO], jhi = r[H_JHI];
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        const unsigned z = (cw >> (4 * p)) & 15u;
                        const unsigned zone = z & 3u;
                        if (zone == 0u) continue;
                        const float j = jl[p] + sb0;
                        float v;
                        if (PROF == kVoigt) {
                            if (zone == 1u) {
                                v = v_far(r, j);
                            } else {
                                const float vm = v_mid<NT>(r, S.m + i, S.csc[i], j);
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
                        } else if (PROF == kLorentz) {
                            v = v_lor(r, j);
                        } else if (PROF == kGHSampled) {
                            v = v_ghs<NT>(A.tab, r, S.m + i, j);
                        } else if (PROF == kGHBinned) {
                            v = v_ghb<NT>(A.tab, r, S.m + i, j);
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

hipError_t launch_records(int profile, const RecArgs& a, hipStream_t s) {
    if (a.n_lines <= 0) return hipSuccess;
    const dim3 grid((unsigned)((a.n_lines + 255) / 256)), block(256);
    switch (profile) {
        case kDoppler: hipLaunchKernelGGL(record_kernel<kDoppler>, grid, block, 0, s, a); break;
        case kGaussFixed: hipLaunchKernelGGL(record_kernel<kGaussFixed>, grid, block, 0, s, a); break;
        case kLorentz: hipLaunchKernelGGL(record_kernel<kLorentz>, grid, block, 0, s, a); break;
        case kGHSampled: hipLaunchKernelGGL(record_kernel<kGHSampled>, grid, block, 0, s, a); break;
        case kGHBinned: hipLaunchKernelGGL(record_kernel<kGHBinned>, grid, block, 0, s, a); break;
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
        default: launch_p<kVoigt>(waves, P, a, s); break;
    }
    return hipGetLastError();
}

}  // namespace xs
