// xy_kernels.hip -- gfx950 kernels for checkerboard Metropolis sweeps of the 2-d XY model.
//
// State layout: two half-lattices (red c = 0, black c = 1), L rows of L/2 entries
// each; entry (c, y, k) is site x = 2k + ((c + y) & 1).  In this layout the four
// neighbours of entry (c, y, k) are, in the other half-lattice,
//     left (y, k + o - 1), right (y, k + o), up (y - 1, k), down (y + 1, k),
// with o = (c + y) & 1, all periodic.  A thread owns the two entries 2j, 2j+1 of
// a half-row, which share one Philox call (counter (sweep, colour, purpose,
// y * P + j)) and their middle horizontal neighbour.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "xy_device.hpp"
#include "xy_launch.hpp"
#include "xy_reduce.hpp"

using namespace xyd;

namespace xyk {

static constexpr int kMaxPartialsFloor = 4096;

size_t state_bytes(int L, int precision)
{
    const size_t elem = precision == XY_FP16 ? 2 : 4;
    return (size_t)L * (size_t)L * elem;
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

int max_partials_for(int L)
{
    // enough for one partial per wave (4 per tile) of the smallest single-sweep
    // tile (64 x 16), for one per tile and sub-sweep of the two-sweep tiles, and
    // for the grid-stride measurement kernel
    const long long t = 4LL * (long long)L * (long long)L / (64 * 16);
    return (int)(t > kMaxPartialsFloor ? t : kMaxPartialsFloor);
}

size_t work_bytes(int L, int precision)
{
    const size_t np = (size_t)max_partials_for(L);
    return align256(state_bytes(L, precision)) + 256 + np * 8 * sizeof(double) + ((np + 255) / 256) * 8 * sizeof(double);
}

Work carve(void* work, int L, int precision)
{
    Work w;
    char* p = (char*)work;
    w.pingpong = p;
    p += align256(state_bytes(L, precision));
    w.counter = (unsigned long long*)p;
    w.arrive = (unsigned*)(w.counter + 2);    // within the 4 u64 zeroed at init
    p += 256;
    w.partials = (double*)p;
    w.max_partials = max_partials_for(L);
    w.chunks = w.partials + (size_t)w.max_partials * 8;
    return w;
}

// --------------------------------------------------------------------- init
template <typename T>
__global__ void __launch_bounds__(256) k_init(T* __restrict__ st, int L, uint32_t k0, uint32_t k1, int hot)
{
    const int Hh = L >> 1;
    const int P = (Hh + 1) >> 1;
    const int j = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    const int c = blockIdx.z;
    if (j >= P || y >= L) return;
    T* row = st + ((size_t)c * L + y) * Hh;
    const int ka = 2 * j, kb = 2 * j + 1;
    if (!hot) {
        row[ka] = store<T>::st(0.0f);
        if (kb < Hh) row[kb] = store<T>::st(0.0f);
        return;
    }
    const u32x4 r = philox10(0u, (uint32_t)c, 1u, (uint32_t)(y * P + j), k0, k1);
    // phi = u (theta = 2 pi u), exact in FP32; binary16 storage rounds it once
    row[ka] = store<T>::st(u01(r.x));
    if (kb < Hh) row[kb] = store<T>::st(u01(r.z));
}

hipError_t launch_init(void* st, int L, int precision, uint32_t k0, uint32_t k1, int hot, hipStream_t s)
{
    const int P = ((L >> 1) + 1) >> 1;
    dim3 grid((P + 63) / 64, (L + 3) / 4, 2), block(64, 4);
    if (precision == XY_FP16)
        hipLaunchKernelGGL(k_init<__half>, grid, block, 0, s, (__half*)st, L, k0, k1, hot);
    else
        hipLaunchKernelGGL(k_init<float>, grid, block, 0, s, (float*)st, L, k0, k1, hot);
    return hipGetLastError();
}

// --------------------------------------------------------------------- zero
__global__ void k_zero_u64(unsigned long long* p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_u64, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

// ------------------------------------------------------ streaming half-sweep
// One colour per launch, in place (a colour reads only the other colour).  The
// neighbours' (cos, sin) are recomputed per thread; this is the schedule for any
// even L and the reference schedule of the debug export.
__device__ __forceinline__ int wrapk(int k, int Hh)
{
    return k < 0 ? k + Hh : (k >= Hh ? k - Hh : k);
}

template <typename T>
__global__ void __launch_bounds__(256)
k_half_sweep(T* __restrict__ st, int L, int col, uint32_t sweep, uint32_t k0, uint32_t k1, Params p,
             unsigned long long* __restrict__ counter, uint8_t* __restrict__ dbg_acc,
             float* __restrict__ dbg_dE)
{
    __shared__ unsigned long long wacc[4];
    const int Hh = L >> 1;
    const int P = (Hh + 1) >> 1;
    const int j = blockIdx.x * 64 + threadIdx.x;
    int acc = 0;
    // rows in a grid-stride loop: the grid stays a few thousand blocks, and so does
    // the number of accept-counter atomics (one per block)
    for (int y = blockIdx.y * 4 + threadIdx.y; y < L; y += gridDim.y * 4) {
        if (j >= P) continue;
        const int o = (col + y) & 1;
        T* own = st + ((size_t)col * L + y) * Hh;
        const T* oth = st + ((size_t)(1 - col) * L + y) * Hh;
        const T* up = st + ((size_t)(1 - col) * L + (y == 0 ? L - 1 : y - 1)) * Hh;
        const T* dn = st + ((size_t)(1 - col) * L + (y == L - 1 ? 0 : y + 1)) * Hh;
        const int ka = 2 * j;
        const bool has_b = ka + 1 < Hh;
        const int kb = has_b ? ka + 1 : ka;
        // horizontal neighbours: h0 = left of a, h1 = right of a = left of b, h2 = right of b
        const float h0 = store<T>::ld(oth[wrapk(ka + o - 1, Hh)]);
        const float h1 = store<T>::ld(oth[wrapk(ka + o, Hh)]);
        const float h2 = store<T>::ld(oth[wrapk(kb + o, Hh)]);
        const float ua = store<T>::ld(up[ka]), ub = store<T>::ld(up[kb]);
        const float da = store<T>::ld(dn[ka]), db = store<T>::ld(dn[kb]);
        float s0, c0, s1, c1, s2, c2, sua, cua, sub, cub, sda, cda, sdb, cdb;
        sincos_turn(h0, s0, c0);
        sincos_turn(h1, s1, c1);
        sincos_turn(h2, s2, c2);
        sincos_turn(ua, sua, cua);
        sincos_turn(ub, sub, cub);
        sincos_turn(da, sda, cda);
        sincos_turn(db, sdb, cdb);
        const u32x4 r = philox10(sweep, (uint32_t)col, 0u, (uint32_t)(y * P + j), k0, k1);
        float tha = store<T>::ld(own[ka]);
        float sa, ca;
        sincos_turn(tha, sa, ca);
        float dEa;
        const int acca = site_update<T>(tha, ca, sa, nsum(c0, c1, cua, cda), nsum(s0, s1, sua, sda),
                                        r.x, r.y, p, &dEa);
        own[ka] = store<T>::st(tha);
        acc += acca;
        const size_t ia = ((size_t)col * L + y) * Hh + ka;
        if (dbg_acc) dbg_acc[ia] = (uint8_t)acca;
        if (dbg_dE) dbg_dE[ia] = dEa;
        if (has_b) {
            float thb = store<T>::ld(own[kb]);
            float sb, cb;
            sincos_turn(thb, sb, cb);
            float dEb;
            const int accb = site_update<T>(thb, cb, sb, nsum(c1, c2, cub, cdb), nsum(s1, s2, sub, sdb),
                                            r.z, r.w, p, &dEb);
            own[kb] = store<T>::st(thb);
            acc += accb;
            if (dbg_acc) dbg_acc[ia + 1] = (uint8_t)accb;
            if (dbg_dE) dbg_dE[ia + 1] = dEb;
        }
    }
    if (counter) {
        const unsigned long long w = wave_sum_u64((unsigned long long)acc);
        if ((threadIdx.x & 63) == 0) wacc[threadIdx.y] = w;
        __syncthreads();
        if (threadIdx.x == 0 && threadIdx.y == 0) {
            const unsigned long long t = (wacc[0] + wacc[1]) + (wacc[2] + wacc[3]);
            if (t) atomicAdd(counter, t);
        }
    }
}

hipError_t launch_half_sweep(const SweepArgs& a, int colour, unsigned long long* counter, uint8_t* dbg_acc,
                             float* dbg_dE, hipStream_t s)
{
    const int P = ((a.L >> 1) + 1) >> 1;
    // about 8192 blocks at most: the row loop covers the rest
    const int gx = (P + 63) / 64;
    const int gy = std::max(1, std::min((a.L + 3) / 4, 8192 / gx));
    dim3 grid(gx, gy), block(64, 4);
    const Params p{a.delta, a.nbl2e};
    if (a.precision == XY_FP16)
        hipLaunchKernelGGL(k_half_sweep<__half>, grid, block, 0, s, (__half*)a.dst, a.L, colour, a.sweep,
                           a.key0, a.key1, p, counter, dbg_acc, dbg_dE);
    else
        hipLaunchKernelGGL(k_half_sweep<float>, grid, block, 0, s, (float*)a.dst, a.L, colour, a.sweep,
                           a.key0, a.key1, p, counter, dbg_acc, dbg_dE);
    return hipGetLastError();
}

// ------------------------------------------------------------- measurement
// Block-level FP64 reduction of the six sums; thread 0 gets the totals.
template <int NT>
__device__ __forceinline__ void block_sum6(double v[6], double* red /* [NT/64][6] */)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 6; ++q) v[q] = wave_sum(v[q]);
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < 6; ++q) red[wid * 6 + q] = v[q];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            double t = 0.0;
            for (int w = 0; w < NT / 64; ++w) t += red[w * 6 + q];
            v[q] = t;
        }
    }
}

// Grid-stride loop over black pairs; every black site adds its four bonds, its own
// spin and that of its right-hand red neighbour.  FP32 per-site terms, FP64 sums.
template <typename T>
__global__ void __launch_bounds__(256) k_measure(const T* __restrict__ st, int L, double* __restrict__ partials)
{
    __shared__ double red[4 * 6];
    const int Hh = L >> 1;
    const int P = (Hh + 1) >> 1;
    const long long npairs = (long long)L * P;
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < npairs; t += (long long)gridDim.x * 256) {
        const int y = (int)(t / P), j = (int)(t - (long long)y * P);
        const int o = (1 + y) & 1;
        const T* own = st + ((size_t)L + y) * Hh;
        const T* oth = st + (size_t)y * Hh;
        const T* up = st + (size_t)(y == 0 ? L - 1 : y - 1) * Hh;
        const T* dn = st + (size_t)(y == L - 1 ? 0 : y + 1) * Hh;
        const int ka = 2 * j;
        const bool has_b = ka + 1 < Hh;
        Meas m{0, 0, 0, 0, 0, 0};
        for (int q = 0; q < (has_b ? 2 : 1); ++q) {
            const int k = ka + q;
            float sb, cb, sl, cl, sr, cr, su, cu, sd, cd;
            sincos_turn(store<T>::ld(own[k]), sb, cb);
            sincos_turn(store<T>::ld(oth[wrapk(k + o - 1, Hh)]), sl, cl);
            sincos_turn(store<T>::ld(oth[wrapk(k + o, Hh)]), sr, cr);
            sincos_turn(store<T>::ld(up[k]), su, cu);
            sincos_turn(store<T>::ld(dn[k]), sd, cd);
            meas_black(m, cb, sb, cl, sl, cr, sr, cu, su, cd, sd);
        }
        v[0] += (double)m.cx; v[1] += (double)m.cy; v[2] += (double)m.ix;
        v[3] += (double)m.iy; v[4] += (double)m.mx; v[5] += (double)m.my;
    }
    block_sum6<256>(v, red);
    if (threadIdx.x == 0) {
        double* o = partials + (size_t)blockIdx.x * 8;
#pragma unroll
        for (int q = 0; q < 6; ++q) o[q] = v[q];
        o[6] = 0.0; o[7] = 0.0;
    }
}

hipError_t launch_measure(const void* st, int L, int precision, double* partials, int max_parts, int* nparts,
                          hipStream_t s)
{
    const int P = ((L >> 1) + 1) >> 1;
    const long long npairs = (long long)L * P;
    long long nb = (npairs + 255) / 256;
    if (nb > 2048) nb = 2048;
    if (nb > max_parts) nb = max_parts;
    *nparts = (int)nb;
    if (precision == XY_FP16)
        hipLaunchKernelGGL(k_measure<__half>, dim3((unsigned)nb), dim3(256), 0, s, (const __half*)st, L, partials);
    else
        hipLaunchKernelGGL(k_measure<float>, dim3((unsigned)nb), dim3(256), 0, s, (const float*)st, L, partials);
    return hipGetLastError();
}

// Fixed-order reduction of nparts partial records (8 doubles: six sums, accepts,
// unused) -> one xy_obs.  Large counts take two levels: k_reduce_chunks sums
// consecutive chunks of 256 records (thread t takes record t of its chunk, then a
// fixed tree, block_sum7_256), k_finalize sums the chunk results.  Both levels are
// deterministic.

__global__ void __launch_bounds__(256)
k_reduce_chunks(const double* __restrict__ partials, int nparts, double* __restrict__ out)
{
    __shared__ double red[4 * 7];
    const int i = blockIdx.x * 256 + threadIdx.x;
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    if (i < nparts) {
        const double* q = partials + (size_t)i * 8;
#pragma unroll
        for (int k = 0; k < 7; ++k) v[k] = q[k];
    }
    block_sum7_256(v, red);
    if (threadIdx.x == 0) {
        double* o = out + (size_t)blockIdx.x * 8;
#pragma unroll
        for (int k = 0; k < 7; ++k) o[k] = v[k];
        o[7] = 0.0;
    }
}

__global__ void __launch_bounds__(256)
k_finalize(const double* __restrict__ partials, int nparts, unsigned long long* __restrict__ counter,
           xy_obs* __restrict__ out, uint64_t sweep_after)
{
    __shared__ double red[4 * 7];
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int i = threadIdx.x; i < nparts; i += 256) {
        const double* q = partials + (size_t)i * 8;
#pragma unroll
        for (int k = 0; k < 7; ++k) v[k] += q[k];
    }
    block_sum7_256(v, red);
    if (threadIdx.x == 0) {
        xy_obs o;
        o.sweep = sweep_after;
        o.n_accept = (counter ? *counter : 0ull) + (unsigned long long)v[6];
        o.cx = v[0]; o.cy = v[1]; o.ix = v[2]; o.iy = v[3]; o.mx = v[4]; o.my = v[5];
        *out = o;
        if (counter) *counter = 0ull;
    }
}

hipError_t launch_reduce_chunks(const double* partials, int nparts, double* out, hipStream_t s)
{
    const int nb = (nparts + 255) / 256;
    hipLaunchKernelGGL(k_reduce_chunks, dim3(nb), dim3(256), 0, s, partials, nparts, out);
    return hipGetLastError();
}

// Both levels in one launch: every workgroup sums its chunk of 256 records as
// k_reduce_chunks does and writes the result to `chunks`; the workgroup that
// arrives last (a counter in device memory, released and acquired at device
// scope) sums the chunk results as k_finalize does, writes the record and sets
// the counter back to zero.  The sums, and their order, are those of the two
// separate kernels.
__global__ void __launch_bounds__(256)
k_reduce_finalize(const double* __restrict__ partials, int nparts, double* __restrict__ chunks,
                  unsigned* __restrict__ arrive, unsigned long long* __restrict__ counter, xy_obs* __restrict__ out,
                  uint64_t sweep_after)
{
    __shared__ double red[4 * 7];
    __shared__ int last;
    const int i = blockIdx.x * 256 + threadIdx.x;
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    if (i < nparts) {
        const double* q = partials + (size_t)i * 8;
#pragma unroll
        for (int k = 0; k < 7; ++k) v[k] = q[k];
    }
    block_sum7_256(v, red);
    if (threadIdx.x == 0) {
        double* o = chunks + (size_t)blockIdx.x * 8;
#pragma unroll
        for (int k = 0; k < 7; ++k) o[k] = v[k];
        o[7] = 0.0;
        __threadfence();
        last = atomicAdd(arrive, 1u) == gridDim.x - 1u;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    const int nb = (int)gridDim.x;
    double w[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int c = threadIdx.x; c < nb; c += 256) {
        const double* q = chunks + (size_t)c * 8;
#pragma unroll
        for (int k = 0; k < 7; ++k) w[k] += q[k];
    }
    block_sum7_256(w, red);
    if (threadIdx.x == 0) {
        xy_obs o;
        o.sweep = sweep_after;
        o.n_accept = (counter ? *counter : 0ull) + (unsigned long long)w[6];
        o.cx = w[0]; o.cy = w[1]; o.ix = w[2]; o.iy = w[3]; o.mx = w[4]; o.my = w[5];
        *out = o;
        if (counter) *counter = 0ull;
        *arrive = 0u;
    }
}

hipError_t launch_finalize(const double* partials, int nparts, unsigned long long* counter, xy_obs* out,
                           uint64_t sweep_after, hipStream_t s, double* scratch, unsigned* arrive)
{
    if (nparts > 2048 && scratch && arrive) {
        const int nb = (nparts + 255) / 256;
        hipLaunchKernelGGL(k_reduce_finalize, dim3(nb), dim3(256), 0, s, partials, nparts, scratch, arrive, counter,
                           out, sweep_after);
    } else if (nparts > 2048 && scratch) {
        const int nb = (nparts + 255) / 256;
        hipLaunchKernelGGL(k_reduce_chunks, dim3(nb), dim3(256), 0, s, partials, nparts, scratch);
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, scratch, nb, counter, out, sweep_after);
    } else {
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, partials, nparts, counter, out, sweep_after);
    }
    return hipGetLastError();
}

}  // namespace xyk
