// xy_strip.hip -- single-lattice sweep by strip segments: one workgroup walks down
// TX columns x SH rows, one sweep per launch.
#include <hip/hip_runtime.h>

#include "xy_launch.hpp"
#include "xy_strip.hpp"

using namespace xyd;

namespace xyk {

// Workgroups are dispatched round-robin over the 8 XCDs (block b -> XCD b % 8).
// Remap so that each XCD takes a band of whole segment rows and walks it segment
// row by segment row, every strip of a row side by side: the workgroups resident
// on an XCD at one time hold the segments on both sides of each strip edge, so the
// edge columns a segment loads before its walk are lines its neighbours load in
// the same XCD's L2, and only the 8 band boundaries cross XCDs.  (With bands of
// whole strips instead, the lines beside a band's outer strips come from another
// XCD: reads 1.22 x one load per angle at L = 16384 against 1.08 x.)  A lattice
// whose segment rows do not split into 8 equal bands takes bands of whole strips
// if its strips do, else the plain order.
__device__ __forceinline__ void xcd_strip(int b, int nsx, int nsy, int& sx, int& sy)
{
    if ((nsy & 7) == 0) {
        const int i = b >> 3;
        sx = i % nsx;
        sy = (b & 7) * (nsy >> 3) + i / nsx;
        return;
    }
    if ((nsx & 7) == 0) {
        const int spx = nsx >> 3, i = b >> 3;
        sx = (b & 7) * spx + i % spx;
        sy = i / spx;
        return;
    }
    sx = b / nsy;
    sy = b - sx * nsy;
}

template <typename T, int TX, int SH, bool MEAS>
__global__ void __launch_bounds__(256)
k_strip(const T* __restrict__ src, T* __restrict__ dst, int L, uint32_t sweep, uint32_t k0, uint32_t k1, Params p,
        double* __restrict__ partials)
{
    extern __shared__ __align__(16) char smem[];
    int sx, sy;
    xcd_strip((int)blockIdx.x, L / TX, L / SH, sx, sy);
    strip_program<T, TX, SH, 256, MEAS>(src, dst, (unsigned)((size_t)L * L * sizeof(T)), L, sx * TX, sy * SH, sweep,
                                       k0, k1, p, partials + (size_t)blockIdx.x * 4 * 8, smem);
}

template <typename T, int TX, int SH, bool MEAS>
static hipError_t run_strip_k(const SweepArgs& a, double* partials, hipStream_t s)
{
    constexpr size_t lds = Strip<TX, SH, 256>::lds_bytes;
    static bool attr_set = false;
    auto kern = k_strip<T, TX, SH, MEAS>;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const int n = (a.L / TX) * (a.L / SH);
    const Params p{a.delta, a.nbl2e};
    hipLaunchKernelGGL(kern, dim3(n), dim3(256), lds, s, (const T*)a.src, (T*)a.dst, a.L, a.sweep, a.key0, a.key1,
                       p, partials);
    return hipGetLastError();
}

// The (strip width, segment height) pairs the autotuner chooses from.
#define XY_STRIP_SHAPES(X) \
    X(128, 32)             \
    X(128, 64)             \
    X(128, 128)            \
    X(256, 32)             \
    X(256, 64)             \
    X(256, 128)            \
    X(256, 256)            \
    X(512, 64)             \
    X(512, 128)            \
    X(512, 256)

bool strip_supported(int L, int tile_x, int tile_y)
{
    if (L < 4 || (L % 4) != 0 || tile_x <= 0 || tile_y <= 0) return false;
    if ((long long)L * L * 4 >= (1LL << 32)) return false;
    if (L % tile_x != 0 || L % tile_y != 0) return false;
#define X(tx, sh) \
    if (tile_x == tx && tile_y == sh) return true;
    XY_STRIP_SHAPES(X)
#undef X
    return false;
}

int strip_records(int L, int tile_x, int tile_y) { return (L / tile_x) * (L / tile_y) * 4; }

hipError_t launch_strip(const SweepArgs& a, int tile_x, int tile_y, bool meas, double* partials, hipStream_t s)
{
#define X(tx, sh)                                                                                     \
    if (tile_x == tx && tile_y == sh) {                                                               \
        if (a.precision == XY_FP16)                                                                   \
            return meas ? run_strip_k<__half, tx, sh, true>(a, partials, s)                           \
                        : run_strip_k<__half, tx, sh, false>(a, partials, s);                         \
        return meas ? run_strip_k<float, tx, sh, true>(a, partials, s)                                \
                    : run_strip_k<float, tx, sh, false>(a, partials, s);                              \
    }
    XY_STRIP_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

}  // namespace xyk
