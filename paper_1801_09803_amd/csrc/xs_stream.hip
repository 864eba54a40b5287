// Accumulators of line-list streaming: the cross sections of successive chunks of a
// line list are added into device-resident compensated sums (sum, compensation) per
// (T, P) and grid point, then read out as sum + compensation.
#include "xs_forward.hpp"

namespace xs {

namespace {

template <class R2>
__global__ __launch_bounds__(256) void acc_zero_kernel(R2* acc, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) {
        R2 z;
        z.x = 0;
        z.y = 0;
        acc[i] = z;
    }
}

// TwoSum of the running sum and the chunk's value; the rounding error goes to the
// compensation term.
template <class R, class R2>
__global__ __launch_bounds__(256) void acc_add_kernel(const R* x, R2* acc, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const R v = x[i];
    R2 a = acc[i];
    const R t = a.x + v;
    const R bp = t - a.x;
    a.y += (a.x - (t - bp)) + (v - bp);
    a.x = t;
    acc[i] = a;
}

template <class R, class R2>
__global__ __launch_bounds__(256) void acc_finish_kernel(const R2* acc, R* out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = acc[i].x + acc[i].y;
}

dim3 grid_of(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

}  // namespace

hipError_t launch_acc_zero(int fp64, void* acc, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (fp64) hipLaunchKernelGGL(acc_zero_kernel<double2>, grid_of(n), dim3(256), 0, s, static_cast<double2*>(acc), n);
    else hipLaunchKernelGGL(acc_zero_kernel<float2>, grid_of(n), dim3(256), 0, s, static_cast<float2*>(acc), n);
    return hipGetLastError();
}

hipError_t launch_acc_add(int fp64, const void* x, void* acc, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (fp64)
        hipLaunchKernelGGL((acc_add_kernel<double, double2>), grid_of(n), dim3(256), 0, s,
                           static_cast<const double*>(x), static_cast<double2*>(acc), n);
    else
        hipLaunchKernelGGL((acc_add_kernel<float, float2>), grid_of(n), dim3(256), 0, s,
                           static_cast<const float*>(x), static_cast<float2*>(acc), n);
    return hipGetLastError();
}

hipError_t launch_acc_finish(int fp64, const void* acc, void* out, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (fp64)
        hipLaunchKernelGGL((acc_finish_kernel<double, double2>), grid_of(n), dim3(256), 0, s,
                           static_cast<const double2*>(acc), static_cast<double*>(out), n);
    else
        hipLaunchKernelGGL((acc_finish_kernel<float, float2>), grid_of(n), dim3(256), 0, s,
                           static_cast<const float2*>(acc), static_cast<float*>(out), n);
    return hipGetLastError();
}

}  // namespace xs
