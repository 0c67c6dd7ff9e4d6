// xy_fused.hip -- single-lattice fused sweep: one workgroup per tile, M sweeps per launch.
#include <hip/hip_runtime.h>

#include "xy_launch.hpp"
#include "xy_tile.hpp"
#include "xy_tile1.hpp"

using namespace xyd;

namespace xyk {

// Workgroups are dispatched round-robin over the 8 XCDs (block b -> XCD b % 8).
// Remap so that each XCD works on one contiguous band of tile rows and the halo
// rows two neighbouring tiles share stay in that XCD's L2.
__device__ __forceinline__ int xcd_tile(int b, int ntiles)
{
    if ((ntiles & 7) != 0) return b;
    const int per = ntiles >> 3;
    return (b & 7) * per + (b >> 3);
}

// LDS bytes of a fused launch: the single-sweep tile keeps (cos, sin) only, the
// two-sweep tile also the angles.
template <int TX, int TY, int M, int NT>
constexpr size_t fused_lds()
{
    if constexpr (M == 1) return Tile1<TX, TY, NT>::lds_bytes;
    else return TileShape<TX, TY, M, NT>::lds_bytes;
}

// Lattices whose two buffers (state and ping-pong) together exceed the 256 MiB
// MALL are read back from HBM every sweep; their single-sweep tiles store with
// the non-temporal hint, so the stored rows do not crowd the halo rows the tiles
// beside still have to read out of the L2 (L = 8192 in FP32: 5% less time per
// sweep).  Within the MALL the hint costs more than it saves (L = 4096: 12% more).
constexpr size_t kStreamBytes = (size_t)256 << 20;

// MEAS (single-sweep tiles only): 1 = this sweep is measured, one partial record
// per wave (tile-major); 0 = not measured.  The two-sweep tile takes the mask of
// measured sub-sweeps at run time, one record per tile and sub-sweep.  ST
// (single-sweep tiles only): non-temporal stores.
template <typename T, int TX, int TY, int M, int NT, int MEAS, bool ST>
__global__ void __launch_bounds__(NT)
k_fused(const T* __restrict__ src, T* __restrict__ dst, int L, uint32_t sweep0, uint32_t k0, uint32_t k1, Params p,
        unsigned meas_mask, double* __restrict__ partials)
{
    extern __shared__ __align__(16) char smem[];
    const int tiles_x = L / TX;
    const int ntiles = tiles_x * (L / TY);
    const int b = xcd_tile((int)blockIdx.x, ntiles);
    const int ty = b / tiles_x, tx = b - ty * tiles_x;
    double* red = (double*)(smem + fused_lds<TX, TY, M, NT>());
    if constexpr (M == 1)
        tile1_program<T, TX, TY, NT, MEAS, ST>(src, dst, (unsigned)((size_t)L * L * sizeof(T)), L, tx * TX, ty * TY,
                                           sweep0, k0, k1, p, MEAS != 0, partials + (size_t)b * (NT / 64) * 8, smem,
                                           red);
    else
        tile_program<T, TX, TY, M, NT>(src, dst, L, tx * TX, ty * TY, sweep0, k0, k1, p, meas_mask,
                                       partials + (size_t)b * 8, (size_t)ntiles * 8, smem, red);
}

template <typename T, int TX, int TY, int M, int NT, int MEAS, bool ST>
static hipError_t run_fused_k(const SweepArgs& a, unsigned meas_mask, double* partials, hipStream_t s)
{
    constexpr size_t lds = fused_lds<TX, TY, M, NT>() + (size_t)(NT / 64) * 7 * sizeof(double);
    static bool attr_set = false;
    auto kern = k_fused<T, TX, TY, M, NT, MEAS, ST>;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const int ntiles = (a.L / TX) * (a.L / TY);
    const Params p{a.delta, a.nbl2e};
    hipLaunchKernelGGL(kern, dim3(ntiles), dim3(NT), lds, s, (const T*)a.src, (T*)a.dst,
                       a.L, a.sweep, a.key0, a.key1, p, meas_mask, partials);
    return hipGetLastError();
}

template <typename T, int TX, int TY, int M, int NT>
static hipError_t run_fused(const SweepArgs& a, unsigned meas_mask, double* partials, hipStream_t s)
{
    if constexpr (M == 1) {
        const bool st = 2 * (size_t)a.L * (size_t)a.L * sizeof(T) > kStreamBytes;
        if (meas_mask & 1u)
            return st ? run_fused_k<T, TX, TY, M, NT, 1, true>(a, meas_mask, partials, s)
                      : run_fused_k<T, TX, TY, M, NT, 1, false>(a, meas_mask, partials, s);
        return st ? run_fused_k<T, TX, TY, M, NT, 0, true>(a, meas_mask, partials, s)
                  : run_fused_k<T, TX, TY, M, NT, 0, false>(a, meas_mask, partials, s);
    } else {
        return run_fused_k<T, TX, TY, M, NT, -1, false>(a, meas_mask, partials, s);
    }
}

// The tile shapes the autotuner chooses from.
#define XY_FUSED_SHAPES(X) \
    X(64, 16, 1, 256)      \
    X(64, 32, 1, 256)      \
    X(128, 16, 1, 256)     \
    X(128, 32, 1, 256)     \
    X(128, 64, 1, 256)     \
    X(256, 16, 1, 256)     \
    X(256, 32, 1, 256)     \
    X(64, 32, 2, 256)      \
    X(128, 32, 2, 256)

bool fused_supported(int L, int tile_x, int tile_y, int m)
{
    if (L < 4 || (L % 4) != 0 || tile_x <= 0 || tile_y <= 0) return false;
    // buffer descriptors address the FP32 state with 32-bit byte offsets
    if ((long long)L * L * 4 >= (1LL << 32)) return false;
    if (L % tile_x != 0 || L % tile_y != 0) return false;
    if (2 * m > L || m > L / 2) return false;
#define X(tx, ty, mm, nt) \
    if (tile_x == tx && tile_y == ty && m == mm) return true;
    XY_FUSED_SHAPES(X)
#undef X
    return false;
}

int fused_tiles(int L, int tile_x, int tile_y) { return (L / tile_x) * (L / tile_y); }

int fused_records(int L, int tile_x, int tile_y, int m)
{
    // single-sweep tiles: one record per wave of the 256-thread workgroup
    return fused_tiles(L, tile_x, tile_y) * (m == 1 ? 4 : 1);
}

hipError_t launch_fused(const SweepArgs& a, int tile_x, int tile_y, int m, unsigned meas_mask, double* partials,
                        hipStream_t s)
{
#define X(tx, ty, mm, nt)                                                                          \
    if (tile_x == tx && tile_y == ty && m == mm) {                                                 \
        if (a.precision == XY_FP16) return run_fused<__half, tx, ty, mm, nt>(a, meas_mask, partials, s); \
        return run_fused<float, tx, ty, mm, nt>(a, meas_mask, partials, s);               \
    }
    XY_FUSED_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

}  // namespace xyk
