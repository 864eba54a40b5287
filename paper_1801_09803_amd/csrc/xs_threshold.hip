// Intensity thresholds (Sec. "Intensity thresholds"): per (T, P), the sorted lines whose
// intensity (Eq. 1) reaches the threshold at their wavenumber,
//     constant:  I_cut = I_crit;
//     HITRAN:    I_cut = I_crit (nu/nu_crit) tanh(c2 nu/(2T)) for nu <= nu_crit, else I_crit,
// compacted in sorted order so that the tile kernels sweep only kept lines.
//   cull_count: per 256 lines, the number kept;            (exclusive scan of the counts)
//   cull_map:   per line, its compacted position pos and, if kept, map[pos] = line;
//   cull_offs:  the offsets table of the kept lines, offs[v] = pos[off[v]].
// The keep decision is recomputed identically in both passes (same double arithmetic).
#include "xs_forward_common.hpp"

namespace xs {

namespace {

__device__ __forceinline__ bool keep_line(const CullArgs& A, const TPParam& tp, double Q, int g) {
    const double nu = A.L.nu[g];
    // the intensity the cross section sums: Eq. 1, or the emissivity for emission
    const double S = line_intensity(A.L, g, A.L.elow[g], nu, tp, Q);
    double cut = A.i_crit;
    if (A.mode == 2 && nu <= A.nu_crit) cut = A.i_crit * (nu / A.nu_crit) * tanh(kC2 * nu / (2.0 * tp.T));
    return S >= cut;
}

__device__ __forceinline__ unsigned block_scan_u32(unsigned v, unsigned* lds4, unsigned* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    unsigned incl = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const unsigned o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
    }
    __syncthreads();
    if (lane == 63) lds4[wave] = incl;
    __syncthreads();
    unsigned wbase = 0;
    for (int w = 0; w < wave; ++w) wbase += lds4[w];
    *total = lds4[0] + lds4[1] + lds4[2] + lds4[3];
    return wbase + incl - v;
}

__global__ __launch_bounds__(256) void cull_count_kernel(const CullArgs A) {
    __shared__ unsigned lds4[4];
    const int g = blockIdx.x * 256 + threadIdx.x;
    const TPParam tp = *A.tp;
    const unsigned k = (g < A.n_lines && keep_line(A, tp, A.Q[tp.iq], g)) ? 1u : 0u;
    unsigned tot;
    block_scan_u32(k, lds4, &tot);
    if (threadIdx.x == 0) A.bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void cull_map_kernel(const CullArgs A) {
    __shared__ unsigned lds4[4];
    const int g = blockIdx.x * 256 + threadIdx.x;
    const TPParam tp = *A.tp;
    const bool k = g < A.n_lines && keep_line(A, tp, A.Q[tp.iq], g);
    unsigned tot;
    const unsigned ex = block_scan_u32(k ? 1u : 0u, lds4, &tot);
    const unsigned long long p = A.bsum[blockIdx.x] + ex;
    if (g < A.n_lines) {
        A.pos[g] = (unsigned)p;
        if (k) A.map[p] = g;
    }
    if (g == A.n_lines - 1) A.pos[A.n_lines] = (unsigned)A.scan_tmp[4096];
}

__global__ __launch_bounds__(256) void cull_offs_kernel(const CullArgs A) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v > A.G.nkeys) return;
    A.offs[v] = (int)A.pos[A.off[v]];
}

}  // namespace

hipError_t launch_cull(const CullArgs& a, hipStream_t s) {
    if (a.n_lines <= 0) return hipSuccess;
    const int64_t nb = ((int64_t)a.n_lines + 255) / 256;
    hipLaunchKernelGGL(cull_count_kernel, dim3((unsigned)nb), dim3(256), 0, s, a);
    hipError_t e = launch_scan64(a.bsum, nb, a.scan_tmp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(cull_map_kernel, dim3((unsigned)nb), dim3(256), 0, s, a);
    const int64_t nk = (int64_t)a.G.nkeys + 1;
    hipLaunchKernelGGL(cull_offs_kernel, dim3((unsigned)((nk + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace xs
