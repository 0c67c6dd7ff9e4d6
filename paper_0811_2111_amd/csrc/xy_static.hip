// xy_static.hip -- the allocation-free sweep entry point (xy_sweep_noalloc).
//
// For callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops, harnesses that forbid it): the workspace of the sweep
// (ping-pong copy of the state, accept and arrival counters, FP64 partial
// records and chunk sums) is a file-scope device array of fixed size instead of
// a caller buffer.  Each device the library runs on holds its own copy of the
// array from module load to process end; the host learns each copy's address
// once per device with hipGetSymbolAddress and passes only that address to the
// kernels.  Calls on one device share the array: calls that overlap in time on
// one device (two streams, two threads) race on it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "xy.h"
#include "xy_launch.hpp"
#include "xy_runtime.hpp"

namespace {

constexpr size_t kScratchBytes = (size_t)XY_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices];   // device address of `scratch` on each device (nullptr: not looked up yet)

// Address of the current device's copy of `scratch`, looked up on the first call
// on that device (with that device current).
hipError_t scratch_ptr(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" int xy_sweep_noalloc(uint64_t seed, int32_t L, double beta, double delta, int32_t precision,
                                uint64_t sweep, int64_t n_sweeps, int32_t measure_every, void* state_dev,
                                size_t state_len, xy_obs* obs_dev, void* hip_stream)
{
    if (!xyr::valid_L(L) || (precision != XY_FP32 && precision != XY_FP16)) return XY_EINVAL;
    const size_t need = xyk::work_bytes(L, precision);
    if (need > kScratchBytes) return XY_ESIZE;
    void* work = nullptr;
    hipError_t e = scratch_ptr(&work);
    if (e != hipSuccess) return xyr::hip_fail(e, "xy_sweep_noalloc: hipGetSymbolAddress(scratch)");
    return xyr::sweep_on_work(seed, L, beta, delta, precision, sweep, n_sweeps, measure_every, state_dev, state_len,
                              work, kScratchBytes, obs_dev, (hipStream_t)hip_stream);
}
