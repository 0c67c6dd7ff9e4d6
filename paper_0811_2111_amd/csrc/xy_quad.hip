// xy_quad.hip -- four replicas of one lattice in one float4 state: hot start,
// fused sweeps, measurement records, and the xy_quad_* C ABI.
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>

#include "xy.h"
#include "xy_launch.hpp"
#include "xy_runtime.hpp"
#include "xy_tile4.hpp"

using namespace xyd;

namespace xyk {

namespace {

// Hot start: replica r of entry (c, y, k) takes u of word X0 (even k) or X2 (odd
// k) of Philox(0, c, 1, y P + k/2) keyed by seed_r, exactly as a single lattice
// with seed_r; cold start: 0.
__global__ void __launch_bounds__(256) k_quad_init(float4* __restrict__ st, int L, Params4 p, int hot)
{
    const int Hh = L >> 1, P = (Hh + 1) >> 1;
    const int j = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    const int c = blockIdx.z;
    if (j >= P || y >= L) return;
    float4* row = st + ((size_t)c * L + y) * Hh;
    const int ka = 2 * j, kb = 2 * j + 1;
    float4 a = make_float4(0.f, 0.f, 0.f, 0.f), b = a;
    if (hot) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const u32x4 w = philox10(0u, (uint32_t)c, 1u, (uint32_t)(y * P + j), p.k0[r], p.k1[r]);
            f4set(a, r, u01(w.x));
            f4set(b, r, u01(w.z));
        }
    }
    row[ka] = a;
    if (kb < Hh) row[kb] = b;
}

__global__ void __launch_bounds__(256) k_quad_copy(const float4* __restrict__ src, float4* __restrict__ dst, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) dst[i] = src[i];
}

__device__ __forceinline__ int xcd_tile4(int b, int ntiles)
{
    if ((ntiles & 7) != 0) return b;
    const int per = ntiles >> 3;
    return (b & 7) * per + (b >> 3);
}

template <int TX, int TY, bool MEAS>
__global__ void __launch_bounds__(256)
k_quad_fused(const float4* __restrict__ src, float4* __restrict__ dst, int L, uint32_t sweep, Params4 p,
             double* __restrict__ partials)
{
    extern __shared__ __align__(16) char smem[];
    const int tiles_x = L / TX;
    const int ntiles = tiles_x * (L / TY);
    const int b = xcd_tile4((int)blockIdx.x, ntiles);
    const int ty = b / tiles_x, tx = b - ty * tiles_x;
    tile4_program<TX, TY, 256, MEAS>(src, dst, (unsigned)((size_t)L * L * sizeof(float4)), L, tx * TX, ty * TY, sweep,
                                     p, partials + (size_t)b * 4 * 8, (size_t)ntiles * 4, smem);
}

template <int TX, int TY, bool MEAS>
hipError_t run_quad(const float4* src, float4* dst, int L, uint32_t sweep, const Params4& p, double* partials,
                    hipStream_t s)
{
    constexpr size_t lds = Tile4<TX, TY, 256>::lds_bytes;
    static bool attr_set = false;
    auto kern = k_quad_fused<TX, TY, MEAS>;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const int ntiles = (L / TX) * (L / TY);
    hipLaunchKernelGGL(kern, dim3(ntiles), dim3(256), lds, s, src, dst, L, sweep, p, partials);
    return hipGetLastError();
}

}  // namespace

// Tile shapes (256 threads, TX/4 pairs per row; one or two pair items per thread
// and half-sweep, each item eight independent updates).
#define XY_QUAD_SHAPES(X) \
    X(32, 16)             \
    X(64, 8)              \
    X(64, 16)             \
    X(128, 4)             \
    X(128, 8)

static bool quad_shape_ok(int L, int tx, int ty)
{
#define X(a, b) \
    if (tx == a && ty == b) return L % a == 0 && L % b == 0;
    XY_QUAD_SHAPES(X)
#undef X
    return false;
}

static hipError_t launch_quad(const float4* src, float4* dst, int L, int tx, int ty, uint32_t sweep,
                              const Params4& p, bool meas, double* partials, hipStream_t s)
{
#define X(a, b)                                                                                   \
    if (tx == a && ty == b)                                                                       \
        return meas ? run_quad<a, b, true>(src, dst, L, sweep, p, partials, s)                    \
                    : run_quad<a, b, false>(src, dst, L, sweep, p, partials, s);
    XY_QUAD_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

}  // namespace xyk

// ----------------------------------------------------------------------- C ABI

namespace {

constexpr uint32_t kQuadMagic = 0x51554144u;   // "QUAD"

size_t quad_state_bytes(int L) { return (size_t)L * (size_t)L * sizeof(float4); }
// one partial record per wave (4 per 256-thread tile) and replica; the smallest
// tiles (32 x 16, 64 x 8, 128 x 4) hold 512 sites
size_t quad_max_records(int L) { return (size_t)L * (size_t)L / 512 * 4 * 4; }
size_t quad_chunks(int L) { return (quad_max_records(L) / 4 + 255) / 256 * 4; }
// ping-pong state, 256 bytes for the finalize's arrival counter, partials, chunks
size_t quad_work_bytes(int L)
{
    return ((quad_state_bytes(L) + 255) & ~(size_t)255) + 256 +
           (quad_max_records(L) + quad_chunks(L)) * 8 * sizeof(double);
}

bool quad_L_ok(int32_t L)
{
    // float4 entries addressed with 32-bit byte offsets; tiles need L % 32 == 0
    return L >= 32 && L % 32 == 0 && (long long)L * L * 16 < (1LL << 32);
}

}  // namespace

struct xy_quad {
    uint32_t magic;
    int32_t L;
    uint64_t seed[4];
    double beta[4], delta[4];
    float4* state;
    float4* pingpong;
    double* partials;
    double* chunks;
    unsigned* arrive;      // arrival counter of the one-launch record reduction (zero between calls)
    hipStream_t stream;
    uint64_t sweep;
    int32_t tile_x, tile_y;
    int32_t hmc_steps;     // leap-frog steps per pass of xy_quad_hmc (1 .. 4)
};

static bool quad_live(const xy_quad* q) { return q && q->magic == kQuadMagic; }

static xyd::Params4 quad_params(const xy_quad* q)
{
    xyd::Params4 p;
    for (int r = 0; r < 4; ++r) {
        const xyk::SweepArgs a = xyr::sweep_args(q->seed[r], q->L, XY_FP32, q->beta[r], q->delta[r]);
        p.delta[r] = a.delta;
        p.nbl2e[r] = a.nbl2e;
        p.k0[r] = a.key0;
        p.k1[r] = a.key1;
    }
    return p;
}

extern "C" {

int xy_quad_state_bytes(int32_t L, size_t* state, size_t* workspace)
{
    if (!quad_L_ok(L)) return XY_EINVAL;
    if (state) *state = quad_state_bytes(L);
    if (workspace) *workspace = quad_work_bytes(L);
    return XY_OK;
}

int xy_quad_init(xy_quad** out, const uint64_t* seeds, int32_t L, const double* beta, const double* delta,
                 int32_t start, void* state_dev, size_t state_len, void* work_dev, size_t work_len, void* hip_stream)
{
    if (!out) return XY_ESTATE;
    *out = nullptr;
    if (!seeds || !beta || !delta || !state_dev || !work_dev) return XY_ESTATE;
    if (!quad_L_ok(L) || (start != XY_HOT && start != XY_COLD)) return XY_EINVAL;
    for (int r = 0; r < 4; ++r)
        if (!xyr::valid_beta_delta(beta[r], delta[r])) return XY_EINVAL;
    if (state_len < quad_state_bytes(L) || work_len < quad_work_bytes(L)) return XY_ESIZE;
    xy_quad* q = new (std::nothrow) xy_quad();
    if (!q) return XY_ENOMEM;
    q->magic = kQuadMagic;
    q->L = L;
    for (int r = 0; r < 4; ++r) {
        q->seed[r] = seeds[r];
        q->beta[r] = beta[r];
        q->delta[r] = delta[r];
    }
    q->state = (float4*)state_dev;
    char* w = (char*)work_dev;
    q->pingpong = (float4*)w;
    w += (quad_state_bytes(L) + 255) & ~(size_t)255;
    q->arrive = (unsigned*)w;
    w += 256;
    q->partials = (double*)w;
    q->chunks = q->partials + quad_max_records(L) * 8;
    q->stream = (hipStream_t)hip_stream;
    q->sweep = 0;
    q->tile_x = L % 128 == 0 ? 128 : 32;
    q->tile_y = L % 128 == 0 ? 8 : 16;
    q->hmc_steps = 4;
    const int Hh = L / 2, P = (Hh + 1) / 2;
    hipLaunchKernelGGL(xyk::k_quad_init, dim3((P + 63) / 64, (L + 3) / 4, 2), dim3(64, 4), 0, q->stream, q->state, L,
                       quad_params(q), start == XY_HOT ? 1 : 0);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = xyk::launch_zero_u64((unsigned long long*)q->arrive, 4, q->stream);
    if (e != hipSuccess) {
        q->magic = 0;
        delete q;
        return xyr::hip_fail(e, "xy_quad_init: launch");
    }
    *out = q;
    return XY_OK;
}

int xy_quad_sweep(xy_quad* q, int64_t n_sweeps, int32_t measure_every, xy_obs* obs_dev)
{
    if (!quad_live(q)) return XY_ESTATE;
    if (n_sweeps < 0 || measure_every < 0) return XY_EINVAL;
    if (q->sweep + (uint64_t)n_sweeps >= 0xffffffffull) return XY_ERANGE;
    const bool meas = measure_every > 0 && obs_dev != nullptr;
    const xyd::Params4 p = quad_params(q);
    const int ntiles = (q->L / q->tile_x) * (q->L / q->tile_y);
    const int nrec = ntiles * 4;                      // records per replica
    const size_t nchunk = ((size_t)nrec + 255) / 256;
    for (int64_t j = 1; j <= n_sweeps; ++j) {
        const bool mj = meas && (j % measure_every) == 0;
        const float4* src = (j & 1) ? q->state : q->pingpong;
        float4* dst = (j & 1) ? q->pingpong : q->state;
        hipError_t e = xyk::launch_quad(src, dst, q->L, q->tile_x, q->tile_y, (uint32_t)q->sweep, p, mj, q->partials,
                                        q->stream);
        if (e != hipSuccess) return xyr::hip_fail(e, "xy_quad_sweep: launch");
        q->sweep += 1;
        if (mj) {
            xy_obs* rec = obs_dev + (size_t)(j / measure_every - 1) * 4;
            for (int r = 0; r < 4; ++r) {
                e = xyk::launch_finalize(q->partials + (size_t)r * nrec * 8, nrec, nullptr, rec + r, q->sweep,
                                         q->stream, q->chunks + (size_t)r * nchunk * 8, q->arrive);
                if (e != hipSuccess) return xyr::hip_fail(e, "xy_quad_sweep: finalize");
            }
        }
    }
    if (n_sweeps & 1) {                               // the last sweep wrote the second buffer
        const size_t n = (size_t)q->L * q->L;
        hipLaunchKernelGGL(xyk::k_quad_copy, dim3(2048), dim3(256), 0, q->stream, q->pingpong, q->state, n);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return xyr::hip_fail(e, "xy_quad_sweep: copy");
    }
    return XY_OK;
}

int xy_quad_set_params(xy_quad* q, const double* beta, const double* delta)
{
    if (!quad_live(q)) return XY_ESTATE;
    if (!beta || !delta) return XY_ESTATE;
    for (int r = 0; r < 4; ++r)
        if (!xyr::valid_beta_delta(beta[r], delta[r])) return XY_EINVAL;
    for (int r = 0; r < 4; ++r) {
        q->beta[r] = beta[r];
        q->delta[r] = delta[r];
    }
    return XY_OK;
}

int xy_quad_get_sweep(const xy_quad* q, uint64_t* sweep)
{
    if (!quad_live(q) || !sweep) return XY_ESTATE;
    *sweep = q->sweep;
    return XY_OK;
}

int xy_quad_set_sweep(xy_quad* q, uint64_t sweep)
{
    if (!quad_live(q)) return XY_ESTATE;
    if (sweep >= 0xffffffffull) return XY_ERANGE;
    q->sweep = sweep;
    return XY_OK;
}

int xy_quad_set_tile(xy_quad* q, int32_t tile_x, int32_t tile_y)
{
    if (!quad_live(q)) return XY_ESTATE;
    if (!xyk::quad_shape_ok(q->L, tile_x, tile_y)) return XY_EINVAL;
    q->tile_x = tile_x;
    q->tile_y = tile_y;
    return XY_OK;
}

int xy_quad_get_tile(const xy_quad* q, int32_t* tile_x, int32_t* tile_y)
{
    if (!quad_live(q) || !tile_x || !tile_y) return XY_ESTATE;
    *tile_x = q->tile_x;
    *tile_y = q->tile_y;
    return XY_OK;
}

int xy_quad_hmc_work_bytes(int32_t L, size_t* bytes)
{
    if (!bytes) return XY_ESTATE;
    if (!quad_L_ok(L)) return XY_EINVAL;
    *bytes = xyk::quad_hmc_work_bytes(L);
    return XY_OK;
}

int xy_quad_hmc(xy_quad* q, int64_t n_traj, int32_t n_md, double eps, void* hmc_work, size_t hmc_len,
                xy_hmc_obs* obs_dev)
{
    if (!quad_live(q)) return XY_ESTATE;
    if (n_traj < 0 || n_md < 1 || !std::isfinite(eps) || !(eps > 0.0)) return XY_EINVAL;
    if (!hmc_work) return XY_ESTATE;
    if (hmc_len < xyk::quad_hmc_work_bytes(q->L)) return XY_ESIZE;
    if (q->sweep + (uint64_t)n_traj >= 0xffffffffull) return XY_ERANGE;
    const xyd::Params4 p = quad_params(q);
    xyk::QHmcKeys keys;
    for (int r = 0; r < 4; ++r) {
        keys.k0[r] = p.k0[r];
        keys.k1[r] = p.k1[r];
    }
    const xyk::QuadHmcWork w = xyk::quad_hmc_carve(hmc_work, q->L);
    for (int64_t j = 0; j < n_traj; ++j) {
        hipError_t e = XY_LAUNCH(xyk::launch_quad_hmc_trajectory(q->state, q->pingpong, w, q->L, q->beta, eps, n_md,
                                                                 q->hmc_steps, (uint32_t)q->sweep, keys,
                                                                 obs_dev ? obs_dev + (size_t)j * 4 : nullptr,
                                                                 q->stream));
        if (e != hipSuccess) return xyr::hip_fail(e, "xy_quad_hmc: launch");
        q->sweep += 1;
    }
    return XY_OK;
}

int xy_quad_hmc_set_steps_per_pass(xy_quad* q, int32_t steps)
{
    if (!quad_live(q)) return XY_ESTATE;
    if (steps < 1 || steps > 4) return XY_EINVAL;
    q->hmc_steps = steps;
    return XY_OK;
}

int xy_quad_hmc_get_steps_per_pass(const xy_quad* q, int32_t* steps)
{
    if (!quad_live(q) || !steps) return XY_ESTATE;
    *steps = q->hmc_steps;
    return XY_OK;
}

int xy_quad_free(xy_quad* q)
{
    if (!quad_live(q)) return XY_ESTATE;
    q->magic = 0;
    delete q;
    return XY_OK;
}

}  // extern "C"
