// Node-sampled Voigt far wing of the FP32 segmented sweep (Sec. "Standard line profiles and
// sampling method", Sec. "Voigt profile"): far_kernel sums, per wavefront of the tile
// kernel, the wing values of the lines centred beyond its node-sampling radius at 16 nodes
// and interpolates them to its points; ends_kernel does the same for the lines whose
// cut-off window ends inside the wavefront, with the points of the end's block evaluated
// one by one.  Their sums go to far slots that launch_combine adds to the tile kernel's.
#include "xs_far.hpp"
#include "xs_records.hpp"

namespace xs {

namespace {

// Node-sampled Voigt far wing: one wavefront per (wavefront tile wv, (T, P), share q).  The
// lines [s1, hcl) and [hcr, s4) (windows covering the wavefront, centres at least R away)
// go in chunks q, q + far_share, ... of 64, one line per lane (the next chunk's line data
// loaded while the current one is summed), first those beyond the |z| < 40 radius (2-node
// rule, hot record only), then those inside it (4-node rule, its coefficients rebuilt from
// the hot record and the x scale), with FP64 sums per lane and node; the share's node totals go to
// far_nodes[tp][wave][node][share], for far_finish_kernel to add up and interpolate.

// wave-wide sum of v (every lane ends with the total)
__device__ __forceinline__ double wave_total(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// the LDS words one lane wrote become visible to the other lanes of its wavefront
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 2-node value of a line (hot record h4 = {H, C0, C1, AMP}, h2 = {B, XC}) at x, amplitudes scaled by up
__device__ __forceinline__ float far_value(const float4& h4, const float2& h2, float x, float up) {
    const float pp = __builtin_fmaf(x, x, h4.y);
    const float den = __builtin_fmaf(pp, pp, h4.z);
    const float num = __builtin_fmaf(pp, h4.w * up, h2.x * up);
    return num * __builtin_amdgcn_rcpf(den);
}

// 4-node value at unscaled x from the coefficients m0..m7 (amplitudes m2, m3, m6, m7
// already scaled)
__device__ __forceinline__ float far_value4(const float4& ma, const float4& mb, float x) {
    const float p1 = __builtin_fmaf(x, x, ma.x);
    const float p2 = __builtin_fmaf(x, x, mb.x);
    const float d1 = __builtin_fmaf(p1, p1, ma.y);
    const float d2 = __builtin_fmaf(p2, p2, mb.y);
    const float n1 = __builtin_fmaf(p1, ma.z, ma.w);
    const float n2 = __builtin_fmaf(p2, mb.z, mb.w);
    return __builtin_fmaf(n1, __builtin_amdgcn_rcpf(d1), n2 * __builtin_amdgcn_rcpf(d2));
}

template <int P>
__global__ __launch_bounds__(256) void far_kernel(const FwdArgs A, int n_waves) {
    constexpr int WW = 64 * P;
    using L = HotOf<kVoigt>;
    static_assert(L::H == 0 && L::C0 == 1 && L::C1 == 2 && L::AMP == 3 && L::XC == L::B + 1, "layout");
    static_assert(C_CSC == 0 && C_M == 8 && kCold == 16, "cold layout");
    const int lane = threadIdx.x & 63, wl = threadIdx.x >> 6;
    const int64_t total = (int64_t)n_waves * A.n_tp * A.far_share;
    const int64_t gw = (int64_t)blockIdx.x * 4 + wl;
    if (gw >= total) return;   // whole wavefronts; no block barrier
    const int q = (int)(gw % A.far_share);
    const int64_t rest = gw / A.far_share;
    const int it = (int)(rest % A.n_tp);
    const int wv = (int)(rest / A.n_tp);
    const Geometry G = A.G;
    const TPParam tp = A.tps[it];
    const int w0 = wv * WW, w1 = w0 + WW - 1;
    const int* map = A.map ? A.map + (int64_t)it * A.map_stride : nullptr;
    const int* off = A.offs ? A.offs + (int64_t)it * A.offs_stride : A.off;
    const float* hot = A.hot + (int64_t)it * A.rec_stride * kHot;
    const int* cold = A.cold + (int64_t)it * A.rec_stride * kCold;   // words 0-7 plane of the row
    const MidNodes mnodes = mid_nodes(A.tab);
    const FarRange fr = far_range(off, G, w0, w1, wave_rm(tp, G, w0, w1), wave_far_r(tp, G, w0, w1, far_reach(WW)));
    // per lane and node: FP32 sums of up to four lines, added to FP64 sums; amplitudes
    // scaled by 2^32 (exact) keep tiny values out of the single-precision subnormal range
    constexpr float kUp = 4294967296.0f;
    double acc[kFarN];
    float a32[kFarN];
#pragma unroll
    for (int m = 0; m < kFarN; ++m) {
        acc[m] = 0.0;
        a32[m] = 0.0f;
    }
    int nacc = 0;
    auto flush = [&]() {
        if (++nacc == 4) {
            nacc = 0;
#pragma unroll
            for (int m = 0; m < kFarN; ++m) {
                acc[m] += (double)a32[m];
                a32[m] = 0.0f;
            }
        }
    };
    {
        // 2-node lines: [s1, ml) then [mr, s4)
        const int nl = fr.ml - fr.s1, nv = nl + (fr.s4 - fr.mr);
        // line data of entry v of the sequence: H, C0, C1, AMP; B, XC; kc
        float4 h4 = make_float4(0.f, 0.f, 0.f, 0.f);
        float2 h2 = make_float2(0.f, 0.f);
        int kc = 0;
        auto fetch = [&](int v) {
            if (v < nv) {
                const int l = v < nl ? fr.s1 + v : fr.mr + (v - nl);
                h4 = *reinterpret_cast<const float4*>(hot + (int64_t)l * kHot);
                h2 = *reinterpret_cast<const float2*>(hot + (int64_t)l * kHot + L::B);
                kc = A.L.kc[line_of(map, l)];
            }
        };
        // this share's chunks of 64 lines: q, q + far_share, ...
        const int step = 64 * A.far_share;
        fetch(64 * q + lane);
        for (int c = 64 * q; c < nv; c += step) {
            const bool in = c + lane < nv;
            const float4 a4 = h4;
            const float2 a2 = h2;
            const int akc = kc;
            fetch(c + step + lane);
            if (in) {
                const float x0 = __builtin_fmaf((float)(w0 - akc), a4.x, a2.y);   // x at w0
#pragma unroll
                for (int m = 0; m < kFarN; ++m)
                    a32[m] += far_value(a4, a2, __builtin_fmaf(node_pos<WW>(m), a4.x, x0), kUp);
            }
            flush();
        }
    }
    {
        // 4-node lines (inside the |z| < 40 radius): [ml, hcl) then [hcr, mr)
        const int nl = fr.hcl - fr.ml, nv = nl + (fr.mr - fr.hcr);
        for (int c = 64 * q; c < nv; c += 64 * A.far_share) {
            const int v = c + lane;
            if (v < nv) {
                const int l = v < nl ? fr.ml + v : fr.hcr + (v - nl);
                const float2 hx = *reinterpret_cast<const float2*>(hot + (int64_t)l * kHot + L::B);   // B, XC
                const float4 h4 = *reinterpret_cast<const float4*>(hot + (int64_t)l * kHot);     // H, C0, C1, AMP
                const float hh = h4.x;
                const float csc = __int_as_float(cold[(int64_t)l * 8 + C_CSC]);   // first cold plane
                float mm[8];
                mid_from_hot(h4.z, h4.w, csc, mnodes, mm);
                const float4 ma = make_float4(mm[0], mm[1], mm[2] * kUp, mm[3] * kUp);
                const float4 mb = make_float4(mm[4], mm[5], mm[6] * kUp, mm[7] * kUp);
                const int akc = A.L.kc[line_of(map, l)];
                const float x0 = __builtin_fmaf((float)(w0 - akc), hh, hx.y);   // scaled x at w0
#pragma unroll
                for (int m = 0; m < kFarN; ++m)
                    a32[m] += far_value4(ma, mb, __builtin_fmaf(node_pos<WW>(m), hh, x0) * csc);
            }
            flush();
        }
    }
    // this share's node totals: node m from lane m
    double mine = 0.0;
#pragma unroll
    for (int m = 0; m < kFarN; ++m) {
        const double t = wave_total((acc[m] + (double)a32[m]) * (1.0 / 4294967296.0));
        mine = lane == m ? t : mine;
    }
    if (lane < kFarN) A.far_nodes[(((int64_t)it * n_waves + wv) * kFarN + lane) * A.far_share + q] = mine;
}

// The far kernel's node totals of each wavefront, summed over its shares in share order,
// interpolated to the wavefront's points into far slot 0.  One wavefront per (wavefront
// tile, (T, P)).
template <int P>
__global__ __launch_bounds__(256) void far_finish_kernel(const FwdArgs A, int n_waves) {
    constexpr int WW = 64 * P;
    __shared__ double tl[4][kFarN];
    const int lane = threadIdx.x & 63, wl = threadIdx.x >> 6;
    const int64_t gw = (int64_t)blockIdx.x * 4 + wl;
    if (gw >= (int64_t)n_waves * A.n_tp) return;   // whole wavefronts; no block barrier
    const int it = (int)(gw % A.n_tp);
    const int wv = (int)(gw / A.n_tp);
    const int w0 = wv * WW;
    if (lane < kFarN) {
        const double* nd = A.far_nodes + (((int64_t)it * n_waves + wv) * kFarN + lane) * A.far_share;
        double v = 0.0;
        for (int q = 0; q < A.far_share; ++q) v += nd[q];
        tl[wl][lane] = v;
    }
    wave_lds_sync();
    double* out = A.far + (int64_t)it * A.far_slots * A.G.n_points;
#pragma unroll 1
    for (int p = 0; p < P; ++p) {
        const int o = 64 * p + lane;
        double w[kFarN];
        far_weights<WW>(o, w);
        double v = 0.0;
#pragma unroll
        for (int m = 0; m < kFarN; ++m) v = __builtin_fma(w[m], tl[wl][m], v);
        const int k = w0 + o;
        if (k < A.G.n_points) out[k] = v;
    }
}

// Window ends of the FP32 Voigt sweep (A.far_ends): the lines [s0, s1) whose cut-off window
// ends inside a wavefront and [s4, s5) whose window starts inside it, all at least the far
// reach (and the |z| < 40 radius) from every point of it.  One workgroup of four
// wavefronts per (wavefront tile, (T, P)); its result goes to far slot 1.
//
// The wavefront is cut into NB blocks of BW points.  A left line whose window ends in block
// b (its last point w0 + m, m clamped to the wavefront) covers blocks 0..b-1 whole: its
// values at the kFarN nodes go to bucket b of the left side, and block c sees the sum of
// the left buckets above it (a suffix sum).  Its points in block b itself (up to w0 + m)
// are evaluated one by one.  Right lines mirror this (windows starting at w0 + m: prefix
// sums, points from w0 + m).  A window clipped at the grid's last point counts as ending
// there: the left bucket holding that point takes every left line up to s1 as candidate
// (a window clipped at the first point starts in bucket 0 of the first wavefront, whose
// candidates already reach down to s4).
//
// Each wavefront of the workgroup walks the buckets of one side in turn, every other one
// (side = wavefront & 1, buckets (wavefront >> 1) + 2i); the lanes take consecutive
// candidate lines of a bucket (sorted by centre: a window end lies hmin..hmax steps from
// it, so a bucket's candidates are a contiguous run), each keeping the node and point sums
// of its lines (FP32 over four lines, then FP64), and the wavefront adds them up at the
// bucket's end.  Each point o then takes the interpolation of its block's node values
// (suffix + prefix) over all nodes plus its block's point sums of both sides.  Fixed order
// throughout: the result does not depend on the run.
template <int P>
struct EndsShape {
    static constexpr int WW = 64 * P;
    static constexpr int BW = P == 1 ? 4 : 8;      // points per block
    static constexpr int NB = WW / BW;             // blocks per wavefront (32 or 16)
};

// wave-wide sum of a float (every lane ends with the total)
__device__ __forceinline__ float wave_total_f(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int P>
__global__ __launch_bounds__(256) void ends_kernel(const FwdArgs A, int n_waves) {
    using ES = EndsShape<P>;
    constexpr int WW = ES::WW, BW = ES::BW, NB = ES::NB;
    using L = HotOf<kVoigt>;
    static_assert(L::H == 0 && L::C0 == 1 && L::C1 == 2 && L::AMP == 3 && L::XC == L::B + 1, "layout");
    static_assert(NB % 2 == 0, "buckets split over two wavefronts per side");
    __shared__ float eb[2][NB][kFarN];   // node sums per (side, block), scaled by 2^32
    __shared__ float ep[2][WW];          // point sums per side, scaled by 2^32
    const int lane = threadIdx.x & 63, wl = threadIdx.x >> 6;
    const int64_t gb = blockIdx.x;
    if (gb >= (int64_t)n_waves * A.n_tp) return;   // the whole workgroup
    const int it = (int)(gb % A.n_tp);
    const int wv = (int)(gb / A.n_tp);
    const Geometry G = A.G;
    const int w0 = wv * WW, w1 = w0 + WW - 1;
    const int* map = A.map ? A.map + (int64_t)it * A.map_stride : nullptr;
    const int* off = A.offs ? A.offs + (int64_t)it * A.offs_stride : A.off;
    const float* hot = A.hot + (int64_t)it * A.rec_stride * kHot;
    const int s0 = off_at(off, (int64_t)w0 - G.hmax, G), s1 = off_at(off, (int64_t)w1 - G.hmin, G);
    const int s4 = off_at(off, (int64_t)w0 + G.hmin + 1, G), s5 = off_at(off, (int64_t)w1 + G.hmax + 1, G);
    constexpr float kUp = 4294967296.0f;
    for (int o = threadIdx.x; o < 2 * WW; o += 256) (&ep[0][0])[o] = 0.0f;
    __syncthreads();
    const int side = wl & 1;
    for (int b = wl >> 1; b < NB; b += 2) {
        // candidate lines of bucket b (uniform)
        const int64_t e0 = (int64_t)w0 + b * BW, e1 = e0 + BW - 1;
        int r0, r1;
        if (side == 0) {
            const bool last = e0 <= (int64_t)G.n_points - 1 && (int64_t)G.n_points - 1 <= e1;
            r0 = off_at(off, e0 - G.hmax, G);
            r1 = last ? s1 : off_at(off, e1 - G.hmin + 1, G);
            r0 = r0 > s0 ? r0 : s0;
            r1 = r1 < s1 ? r1 : s1;
        } else {
            r0 = off_at(off, e0 + G.hmin, G);
            r1 = off_at(off, e1 + G.hmax + 1, G);
            r0 = r0 > s4 ? r0 : s4;
            r1 = r1 < s5 ? r1 : s5;
        }
        float n32[kFarN], p32[BW];
        double n64[kFarN], p64[BW];
#pragma unroll
        for (int m = 0; m < kFarN; ++m) { n32[m] = 0.0f; n64[m] = 0.0; }
#pragma unroll
        for (int j = 0; j < BW; ++j) { p32[j] = 0.0f; p64[j] = 0.0; }
        int nacc = 0;
        // line data of the lane's next line (loaded while the current one is summed):
        // H, C0, C1, AMP; B, XC; kc; window end relative to w0 (-1: none here)
        float4 h4 = make_float4(0.f, 0.f, 0.f, 0.f);
        float2 h2 = make_float2(0.f, 0.f);
        int hkc = 0, hm = -1;
        auto fetch = [&](int l) {
            hm = -1;
            if (l < r1) {
                const int g = line_of(map, l);
                h4 = *reinterpret_cast<const float4*>(hot + (int64_t)l * kHot);
                h2 = *reinterpret_cast<const float2*>(hot + (int64_t)l * kHot + L::B);
                hkc = A.L.kc[g];
                if (side == 0) {
                    const int e = A.L.khi[g] - w0;
                    hm = e < 0 ? -1 : (e > WW - 1 ? WW - 1 : e);
                } else {
                    const int e = A.L.klo[g] - w0;
                    hm = e > WW - 1 ? -1 : (e < 0 ? 0 : e);
                }
            }
        };
        fetch(r0 + lane);
        for (int c = r0; c < r1; c += 64) {
            {
                const float4 a4 = h4;
                const float2 a2 = h2;
                const int akc = hkc, m = hm;
                fetch(c + 64 + lane);
                if (m >= 0 && m / BW == b) {
                    const float x0 = __builtin_fmaf((float)(w0 - akc), a4.x, a2.y);   // x at w0
#pragma unroll
                    for (int mm = 0; mm < kFarN; ++mm)
                        n32[mm] += far_value(a4, a2, __builtin_fmaf(node_pos<WW>(mm), a4.x, x0), kUp);
                    const int j0 = m - b * BW;   // the window's end within the block
#pragma unroll
                    for (int j = 0; j < BW; ++j) {
                        const bool cover = side == 0 ? (j <= j0) : (j >= j0);
                        const float v = far_value(a4, a2, __builtin_fmaf((float)(b * BW + j), a4.x, x0), kUp);
                        p32[j] += cover ? v : 0.0f;
                    }
                }
            }
            if (++nacc == 4) {
                nacc = 0;
#pragma unroll
                for (int mm = 0; mm < kFarN; ++mm) { n64[mm] += (double)n32[mm]; n32[mm] = 0.0f; }
#pragma unroll
                for (int j = 0; j < BW; ++j) { p64[j] += (double)p32[j]; p32[j] = 0.0f; }
            }
        }
        // the bucket's totals (single-precision tree over the lanes' sums)
        float* bucket = eb[side][b];
        if (r1 > r0) {
#pragma unroll
            for (int mm = 0; mm < kFarN; ++mm) {
                const float t = wave_total_f((float)(n64[mm] + (double)n32[mm]));
                if (lane == 0) bucket[mm] = t;
            }
#pragma unroll
            for (int j = 0; j < BW; ++j) {
                const float t = wave_total_f((float)(p64[j] + (double)p32[j]));
                if (lane == j) ep[side][b * BW + j] = t;
            }
        } else if (lane < kFarN) {
            bucket[lane] = 0.0f;
        }
    }
    __syncthreads();
    // left buckets become suffix sums (the lines covering the blocks below them), right
    // buckets prefix sums; one node per lane of wavefront 0 (left) and 1 (right)
    if (wl < 2 && lane < kFarN) {
        double run = 0.0;
        if (wl == 0) {
            for (int c = NB - 1; c >= 0; --c) {
                const double v = (double)eb[0][c][lane];
                eb[0][c][lane] = (float)run;
                run += v;
            }
        } else {
            for (int c = 0; c < NB; ++c) {
                const double v = (double)eb[1][c][lane];
                eb[1][c][lane] = (float)run;
                run += v;
            }
        }
    }
    __syncthreads();
    double* out = A.far + ((int64_t)it * A.far_slots + 1) * G.n_points;
    constexpr double kDown = 1.0 / 4294967296.0;
    for (int o = threadIdx.x; o < WW; o += 256) {
        const int blk = o / BW;
        double w[kFarN];
        far_weights<WW>(o, w);
        double v = 0.0;
#pragma unroll
        for (int m = 0; m < kFarN; ++m)
            v = __builtin_fma(w[m], (double)eb[0][blk][m] + (double)eb[1][blk][m], v);
        const int k = w0 + o;
        if (k < G.n_points) out[k] = (v + ((double)ep[0][o] + (double)ep[1][o])) * kDown;
    }
}

}  // namespace

hipError_t launch_far(int waves, int P, const FwdArgs& a, hipStream_t s) {
    if (a.n_tiles <= 0 || !a.far || !a.seg) return hipSuccess;
    const int n_waves = a.n_tiles * waves;
    const int64_t total = (int64_t)n_waves * a.n_tp * a.far_share;
    const dim3 grid((unsigned)((total + 3) / 4)), block(256);
    switch (P) {
        case 1: hipLaunchKernelGGL(far_kernel<1>, grid, block, 0, s, a, n_waves); break;
        case 2: hipLaunchKernelGGL(far_kernel<2>, grid, block, 0, s, a, n_waves); break;
        case 8: hipLaunchKernelGGL(far_kernel<8>, grid, block, 0, s, a, n_waves); break;
        default: hipLaunchKernelGGL(far_kernel<4>, grid, block, 0, s, a, n_waves); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t fin = (int64_t)n_waves * a.n_tp;
    const dim3 grid_f((unsigned)((fin + 3) / 4));
    switch (P) {
        case 1: hipLaunchKernelGGL(far_finish_kernel<1>, grid_f, block, 0, s, a, n_waves); break;
        case 2: hipLaunchKernelGGL(far_finish_kernel<2>, grid_f, block, 0, s, a, n_waves); break;
        case 8: hipLaunchKernelGGL(far_finish_kernel<8>, grid_f, block, 0, s, a, n_waves); break;
        default: hipLaunchKernelGGL(far_finish_kernel<4>, grid_f, block, 0, s, a, n_waves); break;
    }
    e = hipGetLastError();
    if (e != hipSuccess || !a.far_ends) return e;
    const int64_t ends = (int64_t)n_waves * a.n_tp;   // one workgroup each
    const dim3 grid_e((unsigned)ends);
    switch (P) {
        case 1: hipLaunchKernelGGL(ends_kernel<1>, grid_e, block, 0, s, a, n_waves); break;
        case 2: hipLaunchKernelGGL(ends_kernel<2>, grid_e, block, 0, s, a, n_waves); break;
        case 8: hipLaunchKernelGGL(ends_kernel<8>, grid_e, block, 0, s, a, n_waves); break;
        default: hipLaunchKernelGGL(ends_kernel<4>, grid_e, block, 0, s, a, n_waves); break;
    }
    return hipGetLastError();
}

}  // namespace xs
