// Fixed-order block reductions of the state and line sums (the same inputs give the
// same bits on every run).
#pragma once

#include <hip/hip_runtime.h>

namespace xs {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Sum over a 256-thread block (wave shuffles, then the 4 wave sums in a fixed order);
// the result is valid in thread 0.  lds4: 4 doubles of shared memory.
__device__ __forceinline__ double block_sum256(double v, double* lds4) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds4[wave] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = (lds4[0] + lds4[1]) + (lds4[2] + lds4[3]);
    return r;
}

}  // namespace xs
