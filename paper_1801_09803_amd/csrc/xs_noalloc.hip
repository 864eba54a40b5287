// Q(T) and dQ/dT (Eq. 2 and its temperature derivative) without any device allocation,
// for callers that cannot allocate (code under HIP graph capture, tight serving loops).
//
// xs_partition_function copies its temperatures into plan-owned device memory and keeps
// the per-block partial sums there, growing both on demand.  This variant takes that
// scratch from `scratch`, a file-scope device array of fixed size, so it never calls
// hipMalloc: the temperatures go to the device as a kernel argument and the partial sums
// live in the array.  The reduction kernels and their launch shape are those of
// xs_partition_function, so the results are bitwise the same.
//
// In host code `scratch` names a host-side stand-in, not device memory: its device
// address is taken with hipGetSymbolAddress, once per device, on the first call made
// with that device current, and only that address is passed to kernels.
#include "../../include/xsec.h"
#include "xs_internal.hpp"
#include "xs_lineprep.hpp"

#include <cmath>
#include <mutex>
#include <string>

namespace {

constexpr int kNoAllocMaxT = XS_NOALLOC_MAX_T;
constexpr int kNoAllocBlocks = 256;   // partial sums per temperature (xs_partition_function's count)
// layout: temperatures [kNoAllocMaxT], then partial sums [2 kNoAllocMaxT][kNoAllocBlocks]
constexpr size_t kScratchDoubles = kNoAllocMaxT + (size_t)2 * kNoAllocMaxT * kNoAllocBlocks;

static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};   // device address of `scratch` per device (nullptr: not looked up yet)

// temperatures travel by value (kernel argument), so the call copies nothing from host memory
struct Temperatures {
    double T[kNoAllocMaxT];
    int n;
};

__global__ __launch_bounds__(kNoAllocMaxT) void put_temperatures(const Temperatures t, double* dst) {
    const int i = threadIdx.x;
    if (i < t.n) dst[i] = t.T[i];
}

// Device address of `scratch` on the current device; XS_OK and *out, or an error.
xs_status scratch_address(double** out, std::string* err) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) { *err = std::string("hipGetDevice: ") + hipGetErrorString(e); return XS_ERR_HIP; }
    if (dev < 0 || dev >= kMaxDevices) { *err = "device index beyond the library's table"; return XS_ERR_UNSUPPORTED; }
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            *err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return XS_ERR_HIP;
        }
        g_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_ptr[dev];
    return XS_OK;
}

}  // namespace

extern "C" xs_status xs_partition_function_noalloc(xs_plan* plan, int32_t n_T, const double* T, double* Q,
                                                   double* dQdT, void* stream) {
    if (n_T <= 0 || n_T > kNoAllocMaxT)
        return xs::set_error(XS_ERR_ARG, "n_T must be in [1, " + std::to_string(kNoAllocMaxT) +
                                             "] for xs_partition_function_noalloc (its fixed scratch holds " +
                                             std::to_string(kNoAllocMaxT) + " temperatures)");
    if (!plan || !T) return xs::set_error(XS_ERR_ARG, "NULL argument");
    const double* E = nullptr;
    const int* g = nullptr;
    int64_t n_states = 0;
    if (!xs::plan_states(plan, &E, &g, &n_states) || n_states <= 0)
        return xs::set_error(XS_ERR_STATE, "xs_set_states must come first");
    Temperatures t{};
    t.n = n_T;
    for (int i = 0; i < n_T; ++i) {
        if (!(T[i] > 0.0) || !std::isfinite(T[i]))
            return xs::set_error(XS_ERR_ARG, "temperatures must be finite and > 0");
        t.T[i] = T[i];
    }
    double* base = nullptr;
    std::string err;
    const xs_status st = scratch_address(&base, &err);
    if (st != XS_OK) return xs::set_error(st, err);
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* dT = base;                      // temperatures
    double* part = base + kNoAllocMaxT;     // partial sums, every entry written before it is read
    hipLaunchKernelGGL(put_temperatures, dim3(1), dim3(kNoAllocMaxT), 0, s, t, dT);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = xs::launch_partition(E, g, nullptr, n_states, dT, nullptr, n_T, part, kNoAllocBlocks, Q, dQdT, s);
    if (e != hipSuccess) return xs::set_error(XS_ERR_HIP, std::string("partition sums: ") + hipGetErrorString(e));
    return XS_OK;
}
