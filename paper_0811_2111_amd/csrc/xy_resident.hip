// xy_resident.hip -- single-lattice sweeps with the whole lattice resident in LDS
// (L <= 128): every sweep of a call in one launch of one workgroup.
#include <hip/hip_runtime.h>

#include "xy_launch.hpp"
#include "xy_resident.hpp"

using namespace xyd;

namespace xyk {

template <typename T>
__global__ void __launch_bounds__(256)
k_resident(const T* __restrict__ src, T* __restrict__ dst, int L, uint32_t sweep0, int n, int me, uint32_t k0,
           uint32_t k1, Params p, xy_obs* __restrict__ obs)
{
    extern __shared__ __align__(16) char smem[];
    resident_program<T, 256>(src, dst, L, sweep0, n, me, k0, k1, p, obs, smem);
}

bool resident_supported(int L) { return L >= 4 && L <= kResidentMaxL && L % 4 == 0; }

template <typename T>
static hipError_t run_resident(const SweepArgs& a, int n, int me, xy_obs* obs, hipStream_t s)
{
    static bool attr_set = false;
    auto kern = k_resident<T>;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)resident_lds_bytes(kResidentMaxL, 256));
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const Params p{a.delta, a.nbl2e};
    hipLaunchKernelGGL(kern, dim3(1), dim3(256), resident_lds_bytes(a.L, 256), s, (const T*)a.src, (T*)a.dst, a.L,
                       a.sweep, n, me, a.key0, a.key1, p, obs);
    return hipGetLastError();
}

hipError_t launch_resident(const SweepArgs& a, int n, int me, xy_obs* obs, hipStream_t s)
{
    if (!resident_supported(a.L) || n < 0) return hipErrorInvalidValue;
    if (a.precision == XY_FP16) return run_resident<__half>(a, n, me, obs, s);
    return run_resident<float>(a, n, me, obs, s);
}

}  // namespace xyk
