// xy_reduce.hpp -- the workgroup-level step of the fixed-order FP64 reductions,
// shared by the sweep's record reduction and the hybrid Monte Carlo sums.
#pragma once

#include "xy_device.hpp"

namespace xyd {

// Seven sums over a workgroup of 256 threads: each wave's sum (wave_sum), then the
// four wave sums as (w0 + w1) + (w2 + w3); thread 0 gets the totals.  `red` is 28
// doubles of LDS.
__device__ __forceinline__ void block_sum7_256(double v[7], double* red /* [4][7] */)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 7; ++q) v[q] = wave_sum(v[q]);
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < 7; ++q) red[wid * 7 + q] = v[q];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < 7; ++q) v[q] = (red[q] + red[7 + q]) + (red[14 + q] + red[21 + q]);
}

}  // namespace xyd
