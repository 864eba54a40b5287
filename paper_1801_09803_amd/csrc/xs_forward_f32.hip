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

constexpr int kRec = 32;     // record size in 4-byte words (128 B)
constexpr int kBatch = 256;  // lines per LDS batch

enum : int {
    R_XC = 0, R_H = 1, R_C0 = 2, R_C1 = 3, R_AMP = 4, R_B = 5, R_SB0 = 6, R_CSC = 7,
    R_CODE0 = 8, R_CODE1 = 9, R_JLO = 10, R_JHI = 11,
    R_M = 12,        // 4-node mid zone: cp1, cd1, A1, B1, cp2, cd2, A2, B2
    R_KCL = 20, R_KCH = 21, R_RAD = 22, R_SB0I = 23,
    R_CBASE = 24     // int64 (words 24-25): core value index = cbase + k
};

template <int PROF>
__device__ __forceinline__ void prepare_line(const FwdArgs& A, const Geometry& G, int g, double Q,
                                             int t0, int NS, bool codes, float* r) {
    const LineSetup ls = line_setup(A.L, A.tp, g, Q);
    const double d = (G.nu_a + (double)ls.kc * G.dnu) - ls.nu;   // anchor offset nu_kc - nu
    int* ri = reinterpret_cast<int*>(r);
    r[R_SB0] = (float)(t0 - ls.kc);
    ri[R_SB0I] = t0 - ls.kc;
    r[R_JLO] = (float)(ls.klo - ls.kc);
    r[R_JHI] = (float)(ls.khi - ls.kc);
    int kcl = 0, kch = -1, rad = -1;
    double s = 1.0, y = 0.0;
    if (PROF == kVoigt) {
        s = kSQRT_LN2 / ls.aD;
        y = ls.gam * s;
        const double a = ls.S * kSQRT_LN2_PI / ls.aD;
        // power-of-two scaling keeps x^4 inside the float range for very narrow lines
        const double xmax = s * (G.cutoff + 2.0 * G.dnu) + 1.0;
        int e;
        frexp(xmax, &e);
        e = e > 31 ? e - 31 : 0;
        const double sc = ldexp(1.0, -e), sc2 = sc * sc;
        const double y2 = y * y;
        const double ampf = a * y * kINV_SQRT_PI;
        r[R_XC] = (float)(s * d * sc);
        r[R_H] = (float)(s * G.dnu * sc);
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
        const int rc = A.core_rc[g];
        if (rc >= 0) {
            const int64_t lo = (int64_t)ls.kc - rc, hi = (int64_t)ls.kc + rc;
            kcl = (int)(lo > ls.klo ? lo : ls.klo);
            kch = (int)(hi < ls.khi ? hi : ls.khi);
        }
        *reinterpret_cast<long long*>(r + R_CBASE) = A.core_off[g] - (long long)kcl;
    } else if (PROF == kLorentz) {
        const double ig = ls.gam > 0.0 ? 1.0 / ls.gam : 0.0;
        s = ig;
        r[R_XC] = (float)(d * ig);
        r[R_H] = (float)(G.dnu * ig);
        r[R_AMP] = (float)(ls.S * ig * (1.0 / kPI));
    } else {
        // Gaussian (Eq. 15); x scaled by sqrt(1/ln 2) so exp(-x^2) = exp2(-x'^2)
        const double alpha = (PROF == kDoppler) ? ls.aD : A.alpha_fixed;
        s = kSQRT_LN2 / alpha;
        const double sl = s * 1.2011224087864498;
        r[R_XC] = (float)(sl * d);
        r[R_H] = (float)(sl * G.dnu);
        r[R_AMP] = (float)(ls.S * kSQRT_LN2_PI / alpha);
        rad = radius_steps(10.5, s * G.dnu, s * d);   // exp(-x^2) underflows beyond
    }
    ri[R_KCL] = kcl;
    ri[R_KCH] = kch;
    ri[R_RAD] = rad;
    if (codes) {
        unsigned c0 = 0, c1 = 0;
        for (int sl = 0; sl < NS; ++sl) {
            const int kA = t0 + 64 * sl, kB = kA + 63;
            unsigned code = 0;
            if (!(kB < ls.klo || kA > ls.khi)) {
                const bool full = (kA >= ls.klo && kB <= ls.khi);
                unsigned zone = 1;
                if (PROF == kVoigt) {
                    if (kA <= kch && kB >= kcl) zone = 3;
                    else if (rad >= 0 && (int64_t)kA <= (int64_t)ls.kc + rad && (int64_t)kB >= (int64_t)ls.kc - rad) zone = 2;
                } else if (PROF == kLorentz) {
                    zone = ls.gam > 0.0 ? 1u : 0u;
                } else {
                    zone = ((int64_t)kA <= (int64_t)ls.kc + rad && (int64_t)kB >= (int64_t)ls.kc - rad) ? 1u : 0u;
                }
                code = zone ? (zone | (full ? 0u : 4u)) : 0u;
            }
            if (sl < 8) c0 |= code << (4 * sl); else c1 |= code << (4 * (sl - 8));
        }
        r[R_CODE0] = __uint_as_float(c0);
        r[R_CODE1] = __uint_as_float(c1);
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

__device__ __forceinline__ float v_gauss(const float* r, float j) {
    const float x = __builtin_fmaf(j, r[R_H], r[R_XC]);
    return r[R_AMP] * __builtin_amdgcn_exp2f(-x * x);
}

template <int PROF, int P, bool SEG>
__global__ __launch_bounds__(256) void fwd_f32_kernel(const FwdArgs A) {
    constexpr int W = 256 * P;
    constexpr int WW = 64 * P;
    constexpr int NS = 4 * P;
    __shared__ float rec[kBatch * kRec];

    const Geometry G = A.G;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int tile = tile_of_block(blockIdx.x, A.n_tiles, A.xcd_contiguous);
    const int t0 = tile * W, t1 = t0 + W - 1;
    const int w0 = t0 + wave * WW, w1 = w0 + WW - 1;

    const int b0 = off_at(A.off, (int64_t)t0 - G.hmax, G);
    const int b5 = off_at(A.off, (int64_t)t1 + G.hmax + 1, G);
    const int rm = A.tp.rm;
    // per-wavefront runs (line indices), SEG mode
    int s0 = 0, s1 = 0, s2 = 0, s3 = 0, s4 = 0, s5 = 0;
    if (SEG) {
        s0 = off_at(A.off, (int64_t)w0 - G.hmax, G);
        s1 = off_at(A.off, (int64_t)w1 - G.hmin, G);
        s2 = off_at(A.off, (int64_t)w0 - rm, G);
        s3 = off_at(A.off, (int64_t)w1 + rm + 1, G);
        s4 = off_at(A.off, (int64_t)w0 + G.hmin + 1, G);
        s5 = off_at(A.off, (int64_t)w1 + G.hmax + 1, G);
    }
    const double Q = A.Q[A.tp.iq];

    float jl[P], part[P], sum[P], comp[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        jl[p] = (float)(64 * (wave * P + p) + lane);
        part[p] = 0.f; sum[p] = 0.f; comp[p] = 0.f;
    }
    const int cword = R_CODE0 + (wave * P) / 8;
    const int cshift = 4 * ((wave * P) % 8);

    for (int bs = b0; bs < b5; bs += kBatch) {
        const int g = bs + tid;
        if (g < b5) prepare_line<PROF>(A, G, g, Q, t0, NS, !SEG, rec + tid * kRec);
        __syncthreads();
        const int be = bs + kBatch < b5 ? bs + kBatch : b5;
        for (int cs = bs; cs < be; cs += 64) {
            const int ce = cs + 64 < be ? cs + 64 : be;
            if (SEG) {
                // ---- run 1: window ends inside the wave (upper mask)
                if (PROF == kVoigt || PROF == kLorentz) {
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
                    // ---- runs 2 and 4 (and 3 for Lorentz): wing formula, no branches
                    for (int seg = 0; seg < 2; ++seg) {
                        const int a0 = seg == 0 ? s1 : s3, a1 = seg == 0 ? s2 : s4;
                        const int lo2 = cs > a0 ? cs : a0, hi2 = ce < a1 ? ce : a1;
#pragma unroll 2
                        for (int l = lo2; l < hi2; ++l) {
                            const float* r = rec + (l - bs) * kRec;
                            const float4 h0 = *reinterpret_cast<const float4*>(r);
                            const float4 h1 = *reinterpret_cast<const float4*>(r + 4);
                            const float xc = h0.x, h = h0.y, amp = h1.x, sb0 = h1.z;
                            if (PROF == kVoigt) {
                                const float c0 = h0.z, c1 = h0.w, bb = h1.y;
#pragma unroll
                                for (int p = 0; p < P; ++p) {
                                    const float x = __builtin_fmaf(jl[p] + sb0, h, xc);
                                    const float pp = __builtin_fmaf(x, x, c0);
                                    const float den = __builtin_fmaf(pp, pp, c1);
                                    const float num = __builtin_fmaf(pp, amp, bb);
                                    part[p] = __builtin_fmaf(num, __builtin_amdgcn_rcpf(den), part[p]);
                                }
                            } else {
#pragma unroll
                                for (int p = 0; p < P; ++p) {
                                    const float x = __builtin_fmaf(jl[p] + sb0, h, xc);
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
#pragma unroll
                        for (int p = 0; p < P; ++p) {
                            const int kA = w0 + 64 * p, kB = kA + 63;
                            const float j = jl[p] + sb0;
                            const bool near = rad >= 0 && (int64_t)kA <= (int64_t)kc + rad &&
                                              (int64_t)kB >= (int64_t)kc - rad;
                            if (PROF == kVoigt) {
                                if (kA <= kch && kB >= kcl) part[p] += v_core(A, r, j, kA + lane);
                                else if (near) part[p] += v_mid(r, j);
                                else part[p] += v_far(r, j);
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

    float* out = static_cast<float*>(A.sigma);
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int k = w0 + 64 * p + lane;
        if (k < G.n_points) out[k] = sum[p] + comp[p];
    }
}

template <int PROF, int P>
void launch_one(const FwdArgs& a, hipStream_t s) {
    const dim3 grid(a.n_tiles), block(256);
    if (a.seg) hipLaunchKernelGGL((fwd_f32_kernel<PROF, P, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((fwd_f32_kernel<PROF, P, false>), grid, block, 0, s, a);
}

template <int PROF>
void launch_p(int P, const FwdArgs& a, hipStream_t s) {
    switch (P) {
        case 1: launch_one<PROF, 1>(a, s); break;
        case 2: launch_one<PROF, 2>(a, s); break;
        default: launch_one<PROF, 4>(a, s); break;
    }
}

}  // namespace

hipError_t launch_forward_f32(int profile, int P, const FwdArgs& a, hipStream_t s) {
    if (a.n_tiles <= 0) return hipSuccess;
    switch (profile) {
        case kDoppler: launch_p<kDoppler>(P, a, s); break;
        case kGaussFixed: launch_p<kGaussFixed>(P, a, s); break;
        case kLorentz: launch_p<kLorentz>(P, a, s); break;
        default: launch_p<kVoigt>(P, a, s); break;
    }
    return hipGetLastError();
}

}  // namespace xs
