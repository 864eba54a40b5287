// Measurement aid: a kernel of known vector-instruction count that keeps the vector ALUs
// busy, against which the VALU-issue counters of the cross-section kernels are calibrated
// (as a device copy of known size calibrates the HBM byte counters).
#include <climits>
#include <cstdint>
#include <string>

#include "xs_internal.hpp"

namespace xs {
namespace {

constexpr int kProbeChains = 16;

// Each thread runs iters iterations of kProbeChains independent FP32 FMA chains (one
// v_fma_f32 each per iteration: enough independent work to hide the FMA latency within a
// wavefront), then writes the chains' sum so that none is dead code.
__global__ __launch_bounds__(256) void valu_probe_kernel(float* out, int iters) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    float a[kProbeChains];
#pragma unroll
    for (int q = 0; q < kProbeChains; ++q) a[q] = (float)((t + q) & 1023) * 1.0e-7f;
    const float m = 0.9999999f, c = 1.0e-7f;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int q = 0; q < kProbeChains; ++q) a[q] = __builtin_fmaf(a[q], m, c);
    }
    float s = 0.0f;
#pragma unroll
    for (int q = 0; q < kProbeChains; ++q) s += a[q];
    out[t] = s;
}

}  // namespace
}  // namespace xs

extern "C" xs_status xs_valu_probe(float* out, int64_t n_threads, int32_t iters, void* stream) {
    if (!out) return xs::set_error(XS_ERR_ARG, "xs_valu_probe: out is NULL");
    if (n_threads <= 0 || n_threads % 256 != 0 || n_threads / 256 > INT32_MAX)
        return xs::set_error(XS_ERR_ARG, "xs_valu_probe: n_threads must be a positive multiple of 256");
    if (iters < 1) return xs::set_error(XS_ERR_ARG, "xs_valu_probe: iters must be at least 1");
    hipLaunchKernelGGL(xs::valu_probe_kernel, dim3((unsigned)(n_threads / 256)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), out, (int)iters);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return xs::set_error(XS_ERR_HIP, std::string("xs_valu_probe: ") + hipGetErrorString(e));
    return XS_OK;
}
