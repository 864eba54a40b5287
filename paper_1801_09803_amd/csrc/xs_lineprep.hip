// Partition function (Eq. 2) and line preparation for the tile kernels:
// per-line wavenumber nu = E_up - E_low, the T-independent factor of Eq. 1, the
// cut-off window on the grid (Sec. "Off-set"), and a stable sort of the kept lines
// by their nearest grid index, so that the lines overlapping any grid tile form a
// contiguous index range found through an offsets table.
#include "xs_internal.hpp"
#include "xs_lineprep.hpp"
#include "xs_reduce.hpp"

namespace xs {

// Q(T) and dQ/dT partial sums: block b of temperature blockIdx.y sums states
// b, b + nb, ... (per thread: i = b*256 + t + k*nb*256).  With vibrational energies Ev
// (non-LTE, Sec. "Treating non-local thermodynamic equilibrium") the Boltzmann factor is
// exp(-c2 Ev/T_vib) exp(-c2 (E - Ev)/T), T the rotational temperature, and the
// derivative is taken with respect to T.
__global__ __launch_bounds__(256) void q_partial_kernel(const double* __restrict__ E,
                                                        const int* __restrict__ g,
                                                        const double* __restrict__ Ev, int64_t n,
                                                        const double* __restrict__ T,
                                                        const double* __restrict__ Tv, int nb,
                                                        double* __restrict__ part) {
    __shared__ double lds[4];
    const double t = T[blockIdx.y];
    const double tv = Ev ? Tv[blockIdx.y] : t;
    double q = 0.0, dq = 0.0;
    const int64_t stride = (int64_t)nb * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
        const double e = E[i];
        const double ev = Ev ? Ev[i] : 0.0;
        const double er = e - ev;
        const double bz = (double)g[i] * (Ev ? exp(-(kC2 * ev) / tv - (kC2 * er) / t) : exp(-(kC2 * e) / t));
        q += bz;
        dq += bz * ((kC2 * er) / (t * t));
    }
    const double sq = block_sum256(q, lds);
    const double sdq = block_sum256(dq, lds);
    if (threadIdx.x == 0) {
        part[(2 * (int64_t)blockIdx.y) * nb + blockIdx.x] = sq;
        part[(2 * (int64_t)blockIdx.y + 1) * nb + blockIdx.x] = sdq;
    }
}

__global__ __launch_bounds__(256) void q_final_kernel(const double* __restrict__ part, int nb,
                                                      double* __restrict__ Q, double* __restrict__ dQ) {
    __shared__ double lds[4];
    const double* pq = part + (2 * (int64_t)blockIdx.x) * nb;
    const double* pd = pq + nb;
    double q = 0.0, d = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) { q += pq[i]; d += pd[i]; }
    const double sq = block_sum256(q, lds);
    const double sd = block_sum256(d, lds);
    if (threadIdx.x == 0) {
        if (Q) Q[blockIdx.x] = sq;
        if (dQ) dQ[blockIdx.x] = sd;
    }
}

hipError_t launch_partition(const double* E, const int* g, const double* Ev, int64_t n, const double* T_dev,
                            const double* Tv_dev, int nT, double* part, int nb, double* Q, double* dQ,
                            hipStream_t s) {
    hipLaunchKernelGGL(q_partial_kernel, dim3(nb, nT), dim3(256), 0, s, E, g, Ev, n, T_dev, Tv_dev, nb, part);
    hipLaunchKernelGGL(q_final_kernel, dim3(nT), dim3(256), 0, s, part, nb, Q, dQ);
    return hipGetLastError();
}

// ------------------------------------------------------------------ line prep
__global__ __launch_bounds__(256) void prep_kernel(PrepArgs a) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= a.n) return;
    const int up = a.upper[i] - a.index_base;
    const int lo = a.lower[i] - a.index_base;
    uint32_t key = (uint32_t)a.geo.nkeys;     // dropped unless proven otherwise
    if (up < 0 || up >= a.n_states || lo < 0 || lo >= a.n_states) {
        atomicOr(a.flag, kFlagIndex);
    } else {
        const double Eu = a.E[up], El = a.E[lo];
        const double nu = Eu - El;
        if (!(nu > 0.0)) {
            atomicOr(a.flag, kFlagNu);
        } else {
            const Geometry G = a.geo;
            const double flo = ceil(((nu - G.cutoff) - G.nu_a) / G.dnu);
            const double fhi = floor(((nu + G.cutoff) - G.nu_a) / G.dnu);
            if (fhi >= 0.0 && flo <= (double)(G.n_points - 1)) {
                const int klo = (int)fmax(flo, 0.0);
                const int khi = (int)fmin(fhi, (double)(G.n_points - 1));
                const double fkc = floor((nu - G.nu_a) / G.dnu + 0.5);
                const int kc = (int)fmin(fmax(fkc, -2.0e9), 2.0e9);
                const int64_t k = (int64_t)kc + G.hmax;
                if (k < 0 || k >= G.nkeys) {
                    atomicOr(a.flag, kFlagKey);
                } else {
                    key = (uint32_t)k;
                    float gr, ne;
                    if (a.broad == 1) { gr = a.gref_line[i]; ne = a.nexp_line[i]; }
                    else if (a.broad == 2) {
                        int j = a.J[lo];
                        j = j < 0 ? 0 : (j >= a.n_j ? a.n_j - 1 : j);
                        gr = a.gref_tab[j]; ne = a.nexp_tab[j];
                    } else { gr = a.gamma_const; ne = a.n_const; }
                    const double Aein = a.a_is_log ? exp((double)a.A[i]) : (double)a.A[i];
                    PrepRec r;
                    r.nu = nu;
                    r.elow = El;
                    r.cA = (double)a.g[up] * Aein / (8.0 * kPI * kC_CGS * nu * nu);
                    r.gref = gr;
                    r.nexp = ne;
                    r.kc = kc;
                    r.klo = klo;
                    r.khi = khi;
                    r.pad = 0;
                    a.p_rec[i] = r;
                }
            }
        }
    }
    a.keys[i] = key;
    a.vals[i] = (uint32_t)i;
}

// ------------------------------------------------- LSD radix sort, 4-bit digits
// Blocks of 256 threads x 16 consecutive items ("blocked" layout).  Ranks within a
// block follow item order, so each pass is stable and the sort is deterministic.
constexpr int kItems = 16;
constexpr int kTile = 256 * kItems;

__global__ __launch_bounds__(256) void radix_hist_kernel(const uint32_t* __restrict__ keys, int64_t n,
                                                         int shift, int nblk, uint32_t* __restrict__ hist) {
    __shared__ uint32_t cnt[16];
    if (threadIdx.x < 16) cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t i = base + k;
        if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 15u], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 16) hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = cnt[threadIdx.x];
}

// Exclusive scan of a 256-thread block's values (fixed order); returns the prefix and
// writes the block total to *total.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* lds, uint32_t* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t incl = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
    }
    __syncthreads();
    if (lane == 63) lds[wave] = incl;
    __syncthreads();
    uint32_t wbase = 0;
    for (int w = 0; w < wave; ++w) wbase += lds[w];
    *total = lds[0] + lds[1] + lds[2] + lds[3];
    return wbase + incl - v;
}

// One pass of the LSD sort for one block of kTile items: ranks by digit in item order
// (stable), the block's items staged in LDS in that order, then written out by
// consecutive local positions, so each digit's run of the block lands as one contiguous,
// coalesced range at its global offset.
__global__ __launch_bounds__(256) void radix_scatter_kernel(const uint32_t* __restrict__ kin,
                                                            const uint32_t* __restrict__ vin, int64_t n,
                                                            int shift, int nblk,
                                                            const uint32_t* __restrict__ goff,
                                                            uint32_t* __restrict__ kout,
                                                            uint32_t* __restrict__ vout) {
    __shared__ uint32_t cnt[16 * 256];   // [digit][thread]
    __shared__ uint32_t dbase[16];
    __shared__ uint32_t gbase[16];
    __shared__ uint32_t wsum[4];
    __shared__ uint32_t sk[kTile], sv[kTile];
    const int t = threadIdx.x;
    const int64_t b0 = (int64_t)blockIdx.x * kTile;
    const int64_t base = b0 + (int64_t)t * kItems;
    const int valid = (int)(n - b0 < kTile ? n - b0 : kTile);
    uint32_t key[kItems], val[kItems], rank[kItems];
#pragma unroll
    for (int d = 0; d < 16; ++d) cnt[d * 256 + t] = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t i = base + k;
        key[k] = i < n ? kin[i] : 0xffffffffu;
        val[k] = i < n ? vin[i] : 0u;
    }
    // own counts (LDS column of this thread; no other thread touches it)
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        if (base + k < n) {
            const uint32_t d = (key[k] >> shift) & 15u;
            rank[k] = cnt[d * 256 + t];
            cnt[d * 256 + t] = rank[k] + 1;
        }
    }
    __syncthreads();
    // flat exclusive scan of cnt in digit-major order: thread t owns entries 16t..16t+15
    uint32_t loc[16];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) { loc[k] = s; s += cnt[16 * t + k]; }
    uint32_t total;
    const uint32_t pre = block_exclusive_scan(s, wsum, &total);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) cnt[16 * t + k] = pre + loc[k];
    __syncthreads();
    if (t < 16) {
        dbase[t] = cnt[t * 256];
        gbase[t] = goff[(int64_t)t * nblk + blockIdx.x];
    }
    // stage in block order: local position = start of (digit, thread) + rank
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        if (base + k < n) {
            const uint32_t d = (key[k] >> shift) & 15u;
            const uint32_t lp = cnt[d * 256 + t] + rank[k];
            sk[lp] = key[k];
            sv[lp] = val[k];
        }
    }
    __syncthreads();
    for (int j = t; j < valid; j += 256) {
        const uint32_t kk = sk[j];
        const uint32_t d = (kk >> shift) & 15u;
        const uint32_t pos = gbase[d] + ((uint32_t)j - dbase[d]);
        if ((int64_t)pos < n) {   // always true for a consistent histogram
            kout[pos] = kk;
            vout[pos] = sv[j];
        }
    }
}

// Exclusive scan of m uint32 values (m <= 4096 * 4096): tile sums, one-block scan of
// the tile sums, then per-tile rescans with their base.
__global__ __launch_bounds__(256) void scan_tile_sums_kernel(const uint32_t* __restrict__ x, int64_t m,
                                                             uint32_t* __restrict__ tsum) {
    __shared__ uint32_t wsum[4];
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * 16;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) if (base + k < m) s += x[base + k];
    uint32_t total;
    block_exclusive_scan(s, wsum, &total);
    if (threadIdx.x == 0) tsum[blockIdx.x] = total;
}

__global__ __launch_bounds__(256) void scan_small_kernel(uint32_t* __restrict__ tsum, int64_t nt) {
    __shared__ uint32_t wsum[4];
    const int64_t base = (int64_t)threadIdx.x * 16;
    uint32_t v[16];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) { v[k] = (base + k < nt) ? tsum[base + k] : 0u; s += v[k]; }
    uint32_t total;
    uint32_t pre = block_exclusive_scan(s, wsum, &total);
#pragma unroll
    for (int k = 0; k < 16; ++k) { if (base + k < nt) tsum[base + k] = pre; pre += v[k]; }
}

__global__ __launch_bounds__(256) void scan_apply_kernel(const uint32_t* __restrict__ x, int64_t m,
                                                         const uint32_t* __restrict__ tsum,
                                                         uint32_t* __restrict__ y) {
    __shared__ uint32_t wsum[4];
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * 16;
    uint32_t v[16];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) { v[k] = (base + k < m) ? x[base + k] : 0u; s += v[k]; }
    uint32_t total;
    uint32_t pre = block_exclusive_scan(s, wsum, &total) + tsum[blockIdx.x];
#pragma unroll
    for (int k = 0; k < 16; ++k) { if (base + k < m) y[base + k] = pre; pre += v[k]; }
}

hipError_t launch_exclusive_scan(const uint32_t* x, int64_t m, uint32_t* y, uint32_t* tsum, hipStream_t s) {
    const int64_t nt = (m + kTile - 1) / kTile;
    if (nt > kTile) return hipErrorInvalidValue;
    hipLaunchKernelGGL(scan_tile_sums_kernel, dim3((unsigned)nt), dim3(256), 0, s, x, m, tsum);
    hipLaunchKernelGGL(scan_small_kernel, dim3(1), dim3(256), 0, s, tsum, nt);
    hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)nt), dim3(256), 0, s, x, m, tsum, y);
    return hipGetLastError();
}

int radix_passes(uint32_t max_key) {
    int bits = 0;
    while (bits < 32 && (max_key >> bits) != 0) ++bits;
    return (bits + 3) / 4;
}

int64_t radix_hist_len(int64_t n) { return 16 * ((n + kTile - 1) / kTile); }

// Sorts (keys, vals) by key; ping-pongs through (k2, v2).  Returns in *out_k / *out_v
// the buffers that hold the result.
hipError_t launch_radix_sort(uint32_t* k1, uint32_t* v1, uint32_t* k2, uint32_t* v2, int64_t n,
                             uint32_t max_key, uint32_t* hist, uint32_t* hoff, uint32_t* tsum,
                             uint32_t** out_k, uint32_t** out_v, hipStream_t s) {
    const int nblk = (int)((n + kTile - 1) / kTile);
    const int passes = radix_passes(max_key);
    uint32_t *ka = k1, *va = v1, *kb = k2, *vb = v2;
    for (int p = 0; p < passes && n > 0; ++p) {
        const int shift = 4 * p;
        hipLaunchKernelGGL(radix_hist_kernel, dim3(nblk), dim3(256), 0, s, ka, n, shift, nblk, hist);
        hipError_t e = launch_exclusive_scan(hist, 16 * (int64_t)nblk, hoff, tsum, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(radix_scatter_kernel, dim3(nblk), dim3(256), 0, s, ka, va, n, shift, nblk, hoff, kb, vb);
        uint32_t* tk = ka; ka = kb; kb = tk;
        uint32_t* tv = va; va = vb; vb = tv;
    }
    *out_k = ka;
    *out_v = va;
    return hipGetLastError();
}

// ------------------------------------------------------------ gather + offsets
__global__ __launch_bounds__(256) void gather_kernel(GatherArgs a) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= a.n) return;
    const uint32_t i = a.vals[p];
    if (a.keys[p] >= (uint32_t)a.nkeys || (int64_t)i >= a.n) return;   // dropped lines sit at the end
    const PrepRec r = a.p_rec[i];
    a.nu[p] = r.nu;
    a.elow[p] = r.elow;
    a.cA[p] = r.cA;
    a.gref[p] = r.gref;
    a.nexp[p] = r.nexp;
    a.kc[p] = r.kc;
    a.klo[p] = r.klo;
    a.khi[p] = r.khi;
    a.orig[p] = (int)i;
}

// off[v] = first sorted position whose key is >= v, for v = 0..nkeys.
__global__ __launch_bounds__(256) void offsets_kernel(const uint32_t* __restrict__ keys, int64_t n, int nkeys,
                                                      int* __restrict__ off) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v > nkeys) return;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)keys[mid] < v) lo = mid + 1; else hi = mid;
    }
    off[v] = (int)lo;
}

hipError_t launch_prep(const PrepArgs& a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    hipLaunchKernelGGL(prep_kernel, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_gather(const GatherArgs& a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    hipLaunchKernelGGL(gather_kernel, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_offsets(const uint32_t* keys, int64_t n, int nkeys, int* off, hipStream_t s) {
    hipLaunchKernelGGL(offsets_kernel, dim3((unsigned)((nkeys + 1 + 255) / 256)), dim3(256), 0, s, keys, n, nkeys, off);
    return hipGetLastError();
}

}  // namespace xs
