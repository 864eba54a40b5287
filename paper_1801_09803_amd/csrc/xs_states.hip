// State reductions (Sec. "Radiative lifetime", Sec. "Cooling function", and the specific
// heat from the moments of the partition function, Sec. "Partition function").
//
// The cooling function is a sum over transitions of the emissivity; every transition
// leaving state i carries the same population factor g_i exp(-c2 E_i/T)/Q, so
//     W(T) = h c / (4 pi Q(T)) sum_i g_i exp(-c2 E_i/T) P_i,   P_i = sum_f A_fi nu_fi.
// One pass over the transitions accumulates P_i (and sum_f A_fi, the inverse lifetime)
// per state (bucketed through LDS, or with global atomics beyond the bucketed range);
// each temperature then costs a pass over the states only, not the lines.
//
// Also here: the per-state vibrational energies of non-LTE populations (Sec. "Treating
// non-local thermodynamic equilibrium") and their gather onto the sorted lines.
#include "xs_states.hpp"
#include "xs_reduce.hpp"
#include "xs_lineprep.hpp"

#include <cmath>

namespace xs {

namespace {

constexpr double kR_GAS = kKB * 6.02214076e23;   // J / (K mol), the exact SI value

__global__ __launch_bounds__(256) void fill_kernel(double* x, int64_t n, double v) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) x[i] = v;
}

__global__ __launch_bounds__(256) void rates_kernel(const RateArgs a) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= a.n) return;
    const int up = a.upper[i] - a.index_base;
    if (up < 0 || up >= a.n_states) { atomicOr(a.flag, kFlagIndex); return; }
    const double Aein = a.a_is_log ? exp((double)a.A[i]) : (double)a.A[i];
    if (a.power) {
        const int lo = a.lower[i] - a.index_base;
        if (lo < 0 || lo >= a.n_states) { atomicOr(a.flag, kFlagIndex); return; }
        const double nu = a.E[up] - a.E[lo];
        if (!(nu > 0.0)) { atomicOr(a.flag, kFlagNu); return; }
        unsafeAtomicAdd(a.power + up, Aein * nu);
    }
    if (a.sum_A) unsafeAtomicAdd(a.sum_A + up, Aein);
}

__global__ __launch_bounds__(256) void lifetime_kernel(const double* __restrict__ sum_A, int64_t n,
                                                       double* __restrict__ tau) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double s = sum_A[i];
    tau[i] = s > 0.0 ? 1.0 / s : HUGE_VAL;
}

// Partial sums over the states for temperature blockIdx.y: block b sums the states
// b*256 + t + k*nb*256.  MOM: (w, w x, w x^2) with w = g exp(-x), x = c2 E/T; otherwise
// (w, w P).
template <bool MOM>
__global__ __launch_bounds__(256) void state_partial_kernel(const double* __restrict__ E, const int* __restrict__ g,
                                                            const double* __restrict__ power, int64_t n,
                                                            const double* __restrict__ T, int nb,
                                                            double* __restrict__ part) {
    __shared__ double lds[4];
    const double t = T[blockIdx.y];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    const int64_t stride = (int64_t)nb * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
        const double x = (kC2 * E[i]) / t;
        const double w = (double)g[i] * exp(-x);
        s0 += w;
        if constexpr (MOM) {
            s1 += w * x;
            s2 += (w * x) * x;
        } else {
            s1 += w * power[i];
        }
    }
    constexpr int NS = MOM ? 3 : 2;
    const double r0 = block_sum256(s0, lds);
    const double r1 = block_sum256(s1, lds);
    const double r2 = MOM ? block_sum256(s2, lds) : 0.0;
    if (threadIdx.x == 0) {
        double* p = part + (int64_t)NS * blockIdx.y * nb + blockIdx.x;
        p[0] = r0;
        p[nb] = r1;
        if (MOM) p[2 * nb] = r2;
    }
}

// Per temperature blockIdx.x: the nb partials of each sum, added in a fixed order.
template <bool MOM>
__global__ __launch_bounds__(256) void state_final_kernel(const double* __restrict__ part, int nb, double* Q,
                                                          double* Q1, double* Q2, double* Cp, double* W) {
    __shared__ double lds[4];
    constexpr int NS = MOM ? 3 : 2;
    const double* p = part + (int64_t)NS * blockIdx.x * nb;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) {
        s0 += p[i];
        s1 += p[nb + i];
        if (MOM) s2 += p[2 * nb + i];
    }
    const double q = block_sum256(s0, lds);
    const double q1 = block_sum256(s1, lds);
    const double q2 = MOM ? block_sum256(s2, lds) : 0.0;
    if (threadIdx.x != 0) return;
    const int t = blockIdx.x;
    if (MOM) {
        if (Q) Q[t] = q;
        if (Q1) Q1[t] = q1;
        if (Q2) Q2[t] = q2;
        // C_p = R [Q''/Q - (Q'/Q)^2] + 5R/2: the internal states' heat capacity (the variance
        // of x under the Boltzmann populations) plus the ideal gas's translation and pV
        if (Cp) {
            const double m1 = q1 / q;
            Cp[t] = kR_GAS * (q2 / q - m1 * m1) + 2.5 * kR_GAS;
        }
    } else {
        W[t] = (kH_CGS * kC_CGS) * q1 / (4.0 * kPI * q);
    }
}

// Manifold minima: the bit patterns of non-negative doubles order as the values do, so
// an unsigned 64-bit atomic minimum finds the lowest energy (order-independent).
__global__ __launch_bounds__(256) void vib_min_kernel(const double* __restrict__ E, const int* __restrict__ lab,
                                                      int64_t n, int n_labels, unsigned long long* vmin,
                                                      int* flag) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int l = lab[i];
    const double e = E[i];
    if (l < 0 || l >= n_labels) { atomicOr(flag, kFlagIndex); return; }
    if (!(e >= 0.0)) { atomicOr(flag, kFlagNu); return; }
    atomicMin(vmin + l, (unsigned long long)__double_as_longlong(e));
}

__global__ __launch_bounds__(256) void vib_assign_kernel(const int* __restrict__ lab, int64_t n, int n_labels,
                                                         const unsigned long long* __restrict__ vmin,
                                                         double* __restrict__ Ev) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int l = lab[i];
    Ev[i] = (l >= 0 && l < n_labels) ? __longlong_as_double((long long)vmin[l]) : 0.0;
}

__global__ __launch_bounds__(256) void u64_fill_kernel(unsigned long long* x, int64_t n, unsigned long long v) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) x[i] = v;
}

__global__ __launch_bounds__(256) void vib_gather_kernel(int64_t n, const int* __restrict__ orig, int64_t n_lines,
                                                         const int* __restrict__ upper,
                                                         const int* __restrict__ lower, int base,
                                                         const double* __restrict__ Ev, int64_t n_states,
                                                         double* __restrict__ evl, double* __restrict__ evu) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    const int o = orig[p];
    if (o < 0 || o >= n_lines) { evl[p] = 0.0; evu[p] = 0.0; return; }
    const int up = upper[o] - base, lo = lower[o] - base;
    evl[p] = (lo >= 0 && lo < n_states) ? Ev[lo] : 0.0;
    evu[p] = (up >= 0 && up < n_states) ? Ev[up] : 0.0;
}

dim3 grid_of(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

// ------------------------------------------------------- bucketed per-state sums
constexpr int kBItems = 16;
constexpr int kBTile = 256 * kBItems;     // transitions per block of the count and scatter
constexpr int kBucketStates = 1 << kBucketBits;

struct BRec {
    int local;        // upper state - bucket start
    float araw;       // the A array's value (ln A when a_is_log)
    double anu;       // A nu in double (when the power sum is wanted)
};

static_assert(sizeof(BRec) == 16, "bucket records are 16 B");

// Upper state of transition i, or -1 (flag set) when it is out of range.  Both passes
// place a transition by its upper state alone; the scatter checks the rest.
__device__ __forceinline__ int checked_upper(const RateArgs& a, int64_t i) {
    const int up = a.upper[i] - a.index_base;
    if (up < 0 || up >= a.n_states) { atomicOr(a.flag, kFlagIndex); return -1; }
    return up;
}

// hist[b * nblk + blk] = valid transitions of block blk whose upper state is in bucket b
__global__ __launch_bounds__(256) void bucket_count_kernel(const RateArgs a, int nbk, int nblk,
                                                           uint32_t* __restrict__ hist) {
    extern __shared__ uint32_t cnt[];
    for (int b = threadIdx.x; b < nbk; b += 256) cnt[b] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kBTile;
    for (int k = 0; k < kBItems; ++k) {
        const int64_t i = base + (int64_t)k * 256 + threadIdx.x;   // coalesced
        if (i >= a.n) break;
        const int up = checked_upper(a, i);
        if (up >= 0) atomicAdd(&cnt[up >> kBucketBits], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nbk; b += 256) hist[(int64_t)b * nblk + blockIdx.x] = cnt[b];
}

// Each valid transition to rec[hoff[b * nblk + blk] + rank], rank from an LDS counter
// (the order inside a block's bucket run is not fixed).
__global__ __launch_bounds__(256) void bucket_scatter_kernel(const RateArgs a, int nbk, int nblk,
                                                             const uint32_t* __restrict__ hoff,
                                                             BRec* __restrict__ rec) {
    extern __shared__ uint32_t cnt[];
    for (int b = threadIdx.x; b < nbk; b += 256) cnt[b] = hoff[(int64_t)b * nblk + blockIdx.x];
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kBTile;
    for (int k = 0; k < kBItems; ++k) {
        const int64_t i = base + (int64_t)k * 256 + threadIdx.x;
        if (i >= a.n) break;
        const int up = checked_upper(a, i);
        if (up < 0) continue;
        const uint32_t pos = atomicAdd(&cnt[up >> kBucketBits], 1u);
        BRec r;
        r.local = up & (kBucketStates - 1);
        r.araw = a.A[i];
        r.anu = 0.0;
        if (a.power) {
            // a transition with a bad lower state or nu <= 0 flags the call and adds nothing
            const int lo = a.lower[i] - a.index_base;
            if (lo < 0 || lo >= a.n_states) {
                atomicOr(a.flag, kFlagIndex);
            } else {
                const double nu = a.E[up] - a.E[lo];
                if (!(nu > 0.0)) atomicOr(a.flag, kFlagNu);
                else r.anu = (a.a_is_log ? exp((double)r.araw) : (double)r.araw) * nu;
            }
        }
        rec[pos] = r;
    }
}

// One workgroup per bucket: LDS sums of its records, then the bucket's states written.
__global__ __launch_bounds__(256) void bucket_sum_kernel(const RateArgs a, int nblk, int64_t nhist,
                                                         const uint32_t* __restrict__ hist,
                                                         const uint32_t* __restrict__ hoff,
                                                         const BRec* __restrict__ rec) {
    __shared__ double sa[kBucketStates], sp[kBucketStates];
    for (int j = threadIdx.x; j < kBucketStates; j += 256) { sa[j] = 0.0; sp[j] = 0.0; }
    __syncthreads();
    const int64_t h0 = (int64_t)blockIdx.x * nblk;
    const uint32_t r0 = hoff[h0];
    const uint32_t r1 = h0 + nblk < nhist ? hoff[h0 + nblk] : hoff[nhist - 1] + hist[nhist - 1];
    for (uint32_t q = r0 + threadIdx.x; q < r1; q += 256) {
        const BRec r = rec[q];
        if (a.sum_A) atomicAdd(&sa[r.local], a.a_is_log ? exp((double)r.araw) : (double)r.araw);
        if (a.power) atomicAdd(&sp[r.local], r.anu);
    }
    __syncthreads();
    const int64_t s0 = (int64_t)blockIdx.x * kBucketStates;
    for (int j = threadIdx.x; j < kBucketStates; j += 256) {
        const int64_t st = s0 + j;
        if (st >= a.n_states) break;
        if (a.sum_A) a.sum_A[st] = sa[j];
        if (a.power) a.power[st] = sp[j];
    }
}

}  // namespace

int64_t bucket_count_of(int64_t n_states) { return (n_states + kBucketStates - 1) >> kBucketBits; }

int64_t bucket_hist_len(int64_t n, int64_t n_states) {
    return bucket_count_of(n_states) * ((n + kBTile - 1) / kBTile);
}

bool bucket_rates_fits(int64_t n, int64_t n_states) {
    return n > 0 && bucket_count_of(n_states) <= 8192 && bucket_hist_len(n, n_states) <= kMaxBucketHist &&
           n < ((int64_t)1 << 32);
}

hipError_t launch_bucket_rates(const RateArgs& a, uint32_t* hist, uint32_t* hoff, uint32_t* tsum, void* rec,
                               hipStream_t s) {
    const int nbk = (int)bucket_count_of(a.n_states);
    const int nblk = (int)((a.n + kBTile - 1) / kBTile);
    const int64_t nh = (int64_t)nbk * nblk;
    const size_t lds = (size_t)nbk * sizeof(uint32_t);
    hipLaunchKernelGGL(bucket_count_kernel, dim3(nblk), dim3(256), lds, s, a, nbk, nblk, hist);
    hipError_t e = launch_exclusive_scan(hist, nh, hoff, tsum, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(bucket_scatter_kernel, dim3(nblk), dim3(256), lds, s, a, nbk, nblk, (const uint32_t*)hoff,
                       static_cast<BRec*>(rec));
    hipLaunchKernelGGL(bucket_sum_kernel, dim3(nbk), dim3(256), 0, s, a, nblk, nh, (const uint32_t*)hist,
                       (const uint32_t*)hoff, (const BRec*)rec);
    return hipGetLastError();
}

hipError_t launch_vib_energies(const double* E, const int* labels, int64_t n, int n_labels,
                               unsigned long long* vmin, double* Ev, int* flag, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(u64_fill_kernel, grid_of(n_labels), dim3(256), 0, s, vmin, (int64_t)n_labels,
                       0x7FF0000000000000ull);   // +inf
    hipLaunchKernelGGL(vib_min_kernel, grid_of(n), dim3(256), 0, s, E, labels, n, n_labels, vmin, flag);
    hipLaunchKernelGGL(vib_assign_kernel, grid_of(n), dim3(256), 0, s, labels, n, n_labels,
                       (const unsigned long long*)vmin, Ev);
    return hipGetLastError();
}

hipError_t launch_vib_gather(int64_t n, const int* orig, int64_t n_lines, const int* upper, const int* lower,
                             int index_base, const double* Ev, int64_t n_states, double* evl, double* evu,
                             hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(vib_gather_kernel, grid_of(n), dim3(256), 0, s, n, orig, n_lines, upper, lower, index_base,
                       Ev, n_states, evl, evu);
    return hipGetLastError();
}

hipError_t launch_fill(double* x, int64_t n, double v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_kernel, grid_of(n), dim3(256), 0, s, x, n, v);
    return hipGetLastError();
}

hipError_t launch_rates(const RateArgs& a, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(rates_kernel, grid_of(a.n), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_lifetimes(const double* sum_A, int64_t n, double* tau, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(lifetime_kernel, grid_of(n), dim3(256), 0, s, sum_A, n, tau);
    return hipGetLastError();
}

hipError_t launch_moments(const double* E, const int* g, int64_t n, const double* T_dev, int nT, double* part,
                          int nb, double* Q, double* Q1, double* Q2, double* Cp, hipStream_t s) {
    hipLaunchKernelGGL(state_partial_kernel<true>, dim3(nb, nT), dim3(256), 0, s, E, g, (const double*)nullptr, n,
                       T_dev, nb, part);
    hipLaunchKernelGGL(state_final_kernel<true>, dim3(nT), dim3(256), 0, s, part, nb, Q, Q1, Q2, Cp,
                       (double*)nullptr);
    return hipGetLastError();
}

hipError_t launch_cooling(const double* E, const int* g, const double* power, int64_t n, const double* T_dev,
                          int nT, double* part, int nb, double* W, hipStream_t s) {
    hipLaunchKernelGGL(state_partial_kernel<false>, dim3(nb, nT), dim3(256), 0, s, E, g, power, n, T_dev, nb, part);
    hipLaunchKernelGGL(state_final_kernel<false>, dim3(nT), dim3(256), 0, s, part, nb, (double*)nullptr,
                       (double*)nullptr, (double*)nullptr, (double*)nullptr, W);
    return hipGetLastError();
}

}  // namespace xs
