// xy_batch.hip -- many lattices of uneven size and temperature advanced together.
//
// The replicas of the paper's GLSL variant (four lattices, possibly at different
// temperatures, in one RGBA texture, section 3.2) and its remark that the device
// performs well only with enough work in flight motivate running a whole
// temperature scan as one work list: small lattices alone cannot fill 256 CUs.
//
// Work list (persistent schedule): the lattices are split into eight groups of
// about equal area, one per XCD, and every lattice is cut into TX x TY tiles.
// The workgroups of the one launch find out which XCD they run on, and those on
// XCD x split group x's tiles into contiguous ranges.  The grid never exceeds
// what the GPU holds at once, so every workgroup is resident and the waits
// below cannot deadlock.  One pass = one fused sweep of a tile (state ->
// ping-pong or back).  Every tile has a counter of the passes it has finished;
// before a workgroup starts pass p on its range of a lattice it waits until the
// tiles around the range (those whose halos it reads and those that read its
// halos) have finished pass p-1, which orders both the new reads after the old
// writes and the new writes after the old halo reads.  Workgroups wait only
// for their neighbours, lattices never for each other; a lattice's records wait
// for all of its tiles.  Every workgroup that touches a lattice runs on one XCD
// and so shares one L2: a wait needs no L2 write-back, only the completion of
// the workgroup's stores before it publishes and a drop of its L1 lines after
// it waits.
//
// The second schedule (XY_BATCH_PASSES) launches one kernel per pass over the
// whole work list instead, one workgroup per tile, and lets the kernel boundary
// order the passes.  A workgroup-level barrier needs an agent-scope release and
// acquire per workgroup and pass, i.e. write-backs and invalidations of the
// XCD's L2 cache, whereas a kernel boundary does that once per pass; when many
// workgroups share a lattice the boundary is the cheaper barrier.  Records of a
// measured pass are one partial per tile, summed per lattice in a fixed order by
// a second small kernel.  Under these schedules lattices of L <= 32 are not cut
// into tiles: one workgroup per such lattice holds it in LDS for every sweep of
// the call (xy_resident.hpp), on a second stream that runs beside the per-sweep
// launches and joins them before the copy back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "xy.h"
#include "xy_launch.hpp"
#include "xy_resident.hpp"
#include "xy_runtime.hpp"
#include "xy_tile.hpp"
#include "xy_tile1.hpp"

using namespace xyd;

namespace xyb {

struct LatDesc {
    long long off;        // element offset of the lattice in the state buffer
    int L;
    int tiles_x;
    int first_tile;
    int ntiles;
    int xfirst;           // persistent schedule: first tile within its XCD group's list
    int xcd;              // persistent schedule: the XCD group
    int wide;             // tiles of kWideX x kWideY instead of the batch's shape (not under XY_BATCH_PASSES)
    int resident;         // held in one workgroup's LDS for a whole call (per-sweep schedules, L <= 32)
    uint32_t key0, key1;
    float delta, nbl2e;
};

// Tile shape of the lattices that take wide tiles (XY_BATCH_PASSES_WIDE, XY_BATCH_PERSISTENT):
// the fastest single-lattice shape.
constexpr int kWideX = 256, kWideY = 16;
// Lattices up to this size are LDS-resident under the per-sweep schedules.
constexpr int kBatchResidentMaxL = 32;
// XCDs of the GPU (workgroups of a launch are spread over all of them).
constexpr int kXcd = 8;

// Lattice groups of the persistent schedule: group x (run on XCD x) holds the
// lattices ord[beg[x] .. beg[x+1]) (ord follows this struct in device memory)
// with tiles[x] tiles in all.
struct XcdPlan {
    int beg[kXcd + 1];
    int tiles[kXcd];
    int pad[7];
};

struct Ctrl {
    uint32_t sweep0;      // absolute sweep index of the next pass (advanced by k_batch_advance)
    uint32_t timed_out;   // set if a barrier wait gave up (sticky: the batch's results are void)
    uint32_t spin_limit;  // polls before a barrier wait gives up
    uint32_t hmc_round;   // index of the next HMC trajectory within an xy_batch_hmc call
    uint32_t pad[60];
};

// Default spin limit of one barrier wait: 2^27 polls with s_sleep 2 (~128
// cycles each), several seconds at 2.4 GHz, far beyond any legitimate wait.
static constexpr unsigned kSpinLimit = 1u << 27;

// The XCD a wave runs on: hardware register XCC_ID (20), bits 0..3.
__device__ __forceinline__ int xcc_id()
{
    return (int)(__builtin_amdgcn_s_getreg(20 | (0 << 6) | ((4 - 1) << 11)) & (kXcd - 1));
}

// Bounded poll of a counter by thread 0: relaxed agent-scope loads (no cache
// maintenance per poll) until it reaches target.  A wait that reaches the spin
// limit flags ctrl->timed_out and gives up; every wait, before and while it
// polls, leaves at once once that flag is set, so after one wait has given up
// the whole grid drains without waiting again (the sweeps then run on stale data,
// whose indices never depend on it, and xy_batch_status reports XY_EBARRIER).
__device__ __forceinline__ void poll_at_least(unsigned* ctr, unsigned target, Ctrl* ctrl)
{
    const unsigned limit = ctrl->spin_limit;
    unsigned spins = 0;
    while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (__hip_atomic_load(&ctrl->timed_out, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) break;
        __builtin_amdgcn_s_sleep(2);
        if (++spins >= limit) {
            __hip_atomic_store(&ctrl->timed_out, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
    }
}

// Barrier between workgroups of one XCD.  They share the XCD's L2 and the vector
// L1 is write-through, so a release only has to wait until the workgroup's
// stores have reached the L2: no L2 write-back, which an agent-scope release
// would do (of the whole L2, for every workgroup and pass).  The acquire has to
// drop the stale lines of the CU's L1 cache; outside thread-group-split mode the
// workgroup-scope invalidate does not do that (stale halo rows were read with
// it), so it is the agent-scope one, which drops this XCD's L2 copies of memory
// it does not own as well.
__device__ __forceinline__ void xcd_wait(unsigned* ctr, unsigned target, Ctrl* ctrl)
{
    if (threadIdx.x == 0) {
        poll_at_least(ctr, target, ctrl);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __builtin_amdgcn_s_waitcnt(0);
    }
    __syncthreads();
}

// Wait until every tile in the neighbourhood of this workgroup's range [la, lb)
// of a lattice (lattice-local tile indices, n tiles, tx per tile row) has
// finished `target` passes: the tiles up to 2 tx before the range and after it,
// modulo n, which hold every halo the range reads and every tile that reads the
// range.  The workgroup's threads poll the counters side by side; a poll that
// reaches the spin limit flags ctrl->timed_out, and every wait leaves at once
// once that flag is set.  Then the acquire of xcd_wait.
__device__ __forceinline__ void window_wait(const unsigned* __restrict__ td, int la, int lb, int n, int tx,
                                            unsigned target, Ctrl* ctrl)
{
    const int w = 2 * tx;
    const unsigned limit = ctrl->spin_limit;
    for (unsigned spins = 0;; ++spins) {
        int ok = 1;
        for (int k = threadIdx.x; k < 2 * w; k += 256) {
            int lt = k < w ? la - w + k : lb + (k - w);
            lt %= n;
            if (lt < 0) lt += n;
            if (lt >= la && lt < lb) continue;          // this workgroup's own tile
            if (__hip_atomic_load(&td[lt], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) ok = 0;
        }
        const int stop = __hip_atomic_load(&ctrl->timed_out, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
        if (__syncthreads_and(ok | stop)) break;
        if (threadIdx.x == 0 && spins + 1 >= limit)
            __hip_atomic_store(&ctrl->timed_out, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_s_sleep(2);
    }
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __builtin_amdgcn_s_waitcnt(0);
    }
    __syncthreads();
}

// Wait until all n tile counters of a lattice have reached `target` (the
// workgroup polls them side by side, as window_wait), then the acquire.  A sum
// of counters would not do: with only neighbours coupled, one workgroup can be
// a pass ahead while another is a pass behind.
__device__ __forceinline__ void all_wait(const unsigned* __restrict__ td, int n, unsigned target, Ctrl* ctrl)
{
    const unsigned limit = ctrl->spin_limit;
    for (unsigned spins = 0;; ++spins) {
        int ok = 1;
        for (int k = threadIdx.x; k < n; k += 256)
            if (__hip_atomic_load(&td[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) ok = 0;
        const int stop = __hip_atomic_load(&ctrl->timed_out, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
        if (__syncthreads_and(ok | stop)) break;
        if (threadIdx.x == 0 && spins + 1 >= limit)
            __hip_atomic_store(&ctrl->timed_out, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_s_sleep(2);
    }
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __builtin_amdgcn_s_waitcnt(0);
    }
    __syncthreads();
}

// Position in ord[beg .. end) of the lattice whose group-local tiles hold tile t.
__device__ __forceinline__ int xlattice_of(const LatDesc* d, const int* ord, int beg, int end, int t)
{
    int lo = beg, hi = end - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (d[ord[mid]].xfirst <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Reduce the partials of lattice i for one measured pass (fixed order) into its record.
template <int NT>
__device__ void reduce_lattice(const LatDesc& d, const double* part, xy_obs* out, uint64_t sweep_after, double* red)
{
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int t = threadIdx.x; t < d.ntiles; t += NT) {
        const double* q = part + (size_t)(d.first_tile + t) * 8;
#pragma unroll
        for (int k = 0; k < 7; ++k) v[k] += q[k];
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 7; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < 7; ++k) red[wid * 7 + k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        double s[7];
        for (int k = 0; k < 7; ++k) {
            s[k] = 0.0;
            for (int w = 0; w < NT / 64; ++w) s[k] += red[w * 7 + k];
        }
        xy_obs o;
        o.sweep = sweep_after;
        o.n_accept = (uint64_t)s[6];
        o.cx = s[0]; o.cy = s[1]; o.ix = s[2]; o.iy = s[3]; o.mx = s[4]; o.my = s[5];
        *out = o;
    }
    __syncthreads();
}

// LDS of a batch kernel: the larger of the two tile programs it may run (the
// batch's shape, and 256 x 16 for the lattices flagged wide), then the
// workgroup's reduction slots.
template <int TX, int TY, bool WIDE>
constexpr size_t pass_lds()
{
    constexpr size_t a = Tile1<TX, TY, 256>::lds_bytes, w = Tile1<kWideX, kWideY, 256>::lds_bytes;
    return (WIDE && w > a ? w : a) + Tile1<TX, TY, 256>::red_bytes;
}

// The persistent kernel.  Lattices flagged wide are cut into kWideX x kWideY tiles,
// the others into TX x TY.  bar: records written per lattice, then kXcd + 1
// registration counters (workgroups per XCD, all workgroups); tdone: passes
// finished per tile (work-list order); all zero at launch.
// Start: each workgroup takes a rank among the workgroups of its XCD and waits
// until the whole grid has registered, so that it knows how many share its
// group's tiles.  A group whose XCD runs no workgroup of the grid would be left
// undone: that is flagged like a barrier time-out (it does not happen while the
// grid, a multiple of 8 workgroups, is dealt out over the XCDs in turn).
template <typename T, int TX, int TY, int NT>
__global__ void __launch_bounds__(NT)
k_batch(T* __restrict__ state, T* __restrict__ pp, const LatDesc* __restrict__ lat, const XcdPlan* __restrict__ plan,
        int nlat, int total_tiles, unsigned* __restrict__ bar, unsigned* __restrict__ tdone, Ctrl* __restrict__ ctrl,
        int npass, int measure_every, double* __restrict__ part /* [2][total_tiles][8] */, xy_obs* __restrict__ obs,
        int nrec)
{
    extern __shared__ __align__(16) char smem[];
    __shared__ int s_pos[2];
    static_assert(NT == 256, "four waves");
    // 7 doubles per wave, after the tile programs' LDS
    double* red = (double*)(smem + pass_lds<TX, TY, true>() - Tile1<TX, TY, NT>::red_bytes);
    const int* ord = (const int*)(plan + 1);
    unsigned* rdone = bar;                    // records written per lattice
    unsigned* reg = bar + nlat;
    const int x = xcc_id();
    if (threadIdx.x == 0) {
        const unsigned r = __hip_atomic_fetch_add(&reg[x], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // the rank is taken (the returning atomic has completed) before the
        // workgroup counts as registered
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __hip_atomic_fetch_add(&reg[kXcd], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        poll_at_least(&reg[kXcd], gridDim.x, ctrl);
        for (int y = 0; y < kXcd; ++y)
            if (plan->tiles[y] > 0 && __hip_atomic_load(&reg[y], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u)
                __hip_atomic_store(&ctrl->timed_out, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_pos[0] = (int)r;
        s_pos[1] = (int)__hip_atomic_load(&reg[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);   // > r
    }
    __syncthreads();
    const int rank = s_pos[0], nx = s_pos[1];
    const int nt = plan->tiles[x], beg = plan->beg[x], end = plan->beg[x + 1];
    const int t0 = (int)((long long)nt * rank / nx);
    const int t1 = (int)((long long)nt * (rank + 1) / nx);
    const uint32_t sweep0 = ctrl->sweep0;
    const int qlo = t1 > t0 ? xlattice_of(lat, ord, beg, end, t0) : 0;
    const int qhi = t1 > t0 ? xlattice_of(lat, ord, beg, end, t1 - 1) : -1;
    // measured passes: pass p is measured if (p + 1) % measure_every == 0; its
    // records go to half (p / measure_every) & 1 of the partials
    auto measured = [&](int p) { return measure_every > 0 && obs != nullptr && ((p + 1) % measure_every) == 0; };
    auto slots = [&](int p) {
        return part + (size_t)((p / (measure_every > 0 ? measure_every : 1)) & 1) * (size_t)total_tiles * 8;
    };
    // the workgroup holding a lattice's first tile writes its records once every
    // tile of the lattice has finished the measured pass (a lattice-wide wait,
    // only at measured passes), and counts them in rdone
    auto reduce_if_owner = [&](const LatDesc& d, int i, int p) {
        if (measured(p - 1) && t0 <= d.xfirst && d.xfirst < t1) {
            all_wait(tdone + d.first_tile, d.ntiles, (unsigned)p, ctrl);
            reduce_lattice<NT>(d, slots(p - 1), obs + (size_t)i * nrec + (p / measure_every - 1),
                               (uint64_t)sweep0 + (uint64_t)p, red);
            if (threadIdx.x == 0) __hip_atomic_fetch_add(&rdone[i], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    };

    // A workgroup starts pass p on its tiles of a lattice as soon as the tiles
    // around them have finished pass p-1 (tdone), not the whole lattice, so
    // workgroups wait only for their neighbours.
    for (int p = 0; p < npass; ++p) {
        T* src = (p & 1) ? pp : state;
        T* dst = (p & 1) ? state : pp;
        const bool meas = measured(p);
        double* cur = slots(p);
        for (int q = qlo; q <= qhi; ++q) {
            const int i = ord[q];
            const LatDesc d = lat[i];
            const int a = max(t0, d.xfirst), b = min(t1, d.xfirst + d.ntiles);
            unsigned* td = tdone + d.first_tile;
            if (p > 0) {
                window_wait(td, a - d.xfirst, b - d.xfirst, d.ntiles, d.tiles_x, (unsigned)p, ctrl);
                reduce_if_owner(d, i, p);   // pass p-1 is complete
            }
            // this measured pass reuses the partials half of the records two
            // before it: those must have been read (a read before a write: no
            // cache maintenance needed)
            if (meas && p / measure_every >= 2) {
                if (threadIdx.x == 0) poll_at_least(&rdone[i], (unsigned)(p / measure_every - 1), ctrl);
                __syncthreads();
            }
            const Params prm{d.delta, d.nbl2e};
            const unsigned bytes = (unsigned)((size_t)d.L * d.L * sizeof(T));
            for (int t = a; t < b; ++t) {
                const int lt = t - d.xfirst;
                const int ty = lt / d.tiles_x, tx = lt - ty * d.tiles_x;
                double* rec = cur + (size_t)(d.first_tile + lt) * 8;
                if (d.wide)
                    tile1_program<T, kWideX, kWideY, NT>(src + d.off, dst + d.off, bytes, d.L, tx * kWideX,
                                                         ty * kWideY, sweep0 + (uint32_t)p, d.key0, d.key1, prm, meas,
                                                         rec, smem, red);
                else
                    tile1_program<T, TX, TY, NT>(src + d.off, dst + d.off, bytes, d.L, tx * TX, ty * TY,
                                                 sweep0 + (uint32_t)p, d.key0, d.key1, prm, meas, rec, smem, red);
                __syncthreads();   // the next tile reuses the LDS
            }
            // done with lattice i in pass p: its stores complete, then the tiles' counters
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __syncthreads();
            for (int k = threadIdx.x; k < b - a; k += NT)
                __hip_atomic_store(&td[a - d.xfirst + k], (unsigned)(p + 1), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
    }

    // Epilogue: wait for the last pass, write the last record, and if the pass
    // count is odd copy this workgroup's tiles back into the caller's buffer.
    if (npass > 0) {
        for (int q = qlo; q <= qhi; ++q) {
            const int i = ord[q];
            const LatDesc d = lat[i];
            const int a = max(t0, d.xfirst), b = min(t1, d.xfirst + d.ntiles);
            // the neighbours have finished the last pass (and its reads of `state`)
            window_wait(tdone + d.first_tile, a - d.xfirst, b - d.xfirst, d.ntiles, d.tiles_x, (unsigned)npass, ctrl);
            reduce_if_owner(d, i, npass);
            if (npass & 1) {
                const int Hh = d.L >> 1;
                const int hx = (d.wide ? kWideX : TX) / 2, ry = d.wide ? kWideY : TY;   // tile: ry rows of hx entries
                for (int t = a; t < b; ++t) {
                    const int lt = t - d.xfirst;
                    const int ty = lt / d.tiles_x, tx = lt - ty * d.tiles_x;
                    for (int idx = threadIdx.x; idx < 2 * ry * hx; idx += NT) {
                        const int c = idx / (ry * hx);
                        const int rem = idx - c * (ry * hx);
                        const int rr = rem / hx, k = rem - rr * hx;
                        const size_t e = (size_t)d.off + ((size_t)c * d.L + ty * ry + rr) * Hh + tx * hx + k;
                        state[e] = pp[e];
                    }
                }
            }
        }
    }
}

__global__ void k_batch_advance(Ctrl* ctrl, uint32_t n) { ctrl->sweep0 += n; }

// Batched HMC: the trajectory's records of all lattices from the staging area to
// obs[i * n_traj + r] (r = trajectory within the call), then the sweep counter
// (the trajectory index every lattice's next trajectory reads) advances by one.
__global__ void k_bhmc_finish(const xy_hmc_obs* __restrict__ staging, xy_hmc_obs* __restrict__ obs, int n,
                              int n_traj, Ctrl* __restrict__ ctrl)
{
    __shared__ uint32_t r;
    if (threadIdx.x == 0) r = ctrl->hmc_round;
    __syncthreads();
    if (obs)
        for (int i = threadIdx.x; i < n; i += blockDim.x) obs[(size_t)i * n_traj + r] = staging[i];
    __syncthreads();
    if (threadIdx.x == 0) {
        ctrl->hmc_round = r + 1u;
        ctrl->sweep0 += 1u;
    }
}

__global__ void k_bhmc_start(Ctrl* ctrl) { ctrl->hmc_round = 0u; }

// One pass of the per-pass schedule: workgroup b sweeps tile t (XCD-aware order:
// each XCD takes a contiguous run of the work list, so neighbouring tiles share
// its L2).  WIDE: lattices flagged wide are cut into kWideX x kWideY tiles.
// MEAS = -1: measured, one record per tile at part[t * 8]; 0: not.
template <typename T, int TX, int TY, int MEAS, bool WIDE>
__global__ void __launch_bounds__(256)
k_batch_pass(const T* __restrict__ src, T* __restrict__ dst, const LatDesc* __restrict__ lat,
             const int* __restrict__ tile_lat, int total_tiles, const Ctrl* __restrict__ ctrl, int p,
             double* __restrict__ part)
{
    extern __shared__ __align__(16) char smem[];
    double* red = (double*)(smem + pass_lds<TX, TY, WIDE>() - Tile1<TX, TY, 256>::red_bytes);
    // the grid is the tile count rounded up to a multiple of 8; the last blocks of
    // XCD 7's run have no tile
    const int b = (int)blockIdx.x;
    const int t = (b & 7) * (int)(gridDim.x >> 3) + (b >> 3);
    if (t >= total_tiles) return;
    const LatDesc d = lat[tile_lat[t]];      // a table, not a search: two loads before the tile starts
    const int lt = t - d.first_tile;
    const int ty = lt / d.tiles_x, tx = lt - ty * d.tiles_x;
    const Params prm{d.delta, d.nbl2e};
    const unsigned bytes = (unsigned)((size_t)d.L * d.L * sizeof(T));
    const uint32_t sweep = ctrl->sweep0 + (uint32_t)p;
    if (WIDE && d.wide)
        tile1_program<T, kWideX, kWideY, 256, MEAS>(src + d.off, dst + d.off, bytes, d.L, tx * kWideX, ty * kWideY,
                                                    sweep, d.key0, d.key1, prm, MEAS != 0, part + (size_t)t * 8,
                                                    smem, red);
    else
        tile1_program<T, TX, TY, 256, MEAS>(src + d.off, dst + d.off, bytes, d.L, tx * TX, ty * TY, sweep, d.key0,
                                            d.key1, prm, MEAS != 0, part + (size_t)t * 8, smem, red);
}

// Records of measured pass p (one workgroup per lattice, fixed order): record r of
// lattice i at obs[i * nrec + r], sweep count sweep0 + p + 1.  LDS-resident
// lattices write their own records.
__global__ void __launch_bounds__(256)
k_batch_reduce(const LatDesc* __restrict__ lat, const Ctrl* __restrict__ ctrl, int p, const double* __restrict__ part,
               xy_obs* __restrict__ obs, int nrec, int r)
{
    __shared__ double red[4 * 7];
    const int i = (int)blockIdx.x;
    if (lat[i].resident) return;
    reduce_lattice<256>(lat[i], part, obs + (size_t)i * nrec + r, (uint64_t)ctrl->sweep0 + (uint64_t)p + 1u, red);
}

// The LDS-resident lattices of a per-sweep call: workgroup b runs every sweep of
// lattice ridx[b] from `state`, writes the result to `out` (the buffer that holds
// the other lattices after the last pass) and its records to obs[i * nrec ..].
template <typename T>
__global__ void __launch_bounds__(256)
k_batch_resident(const T* __restrict__ state, T* __restrict__ out, const LatDesc* __restrict__ lat,
                 const int* __restrict__ ridx, const Ctrl* __restrict__ ctrl, int npass, int me,
                 xy_obs* __restrict__ obs, int nrec)
{
    extern __shared__ __align__(16) char smem[];
    const int i = ridx[blockIdx.x];
    const LatDesc d = lat[i];
    const Params prm{d.delta, d.nbl2e};
    resident_program<T, 256>(state + d.off, out + d.off, d.L, ctrl->sweep0, npass, me, d.key0, d.key1, prm,
                             (me > 0 && obs) ? obs + (size_t)i * nrec : nullptr, smem);
}

// dst <- src, n16 16-byte words
__global__ void __launch_bounds__(256) k_batch_copy(uint4* __restrict__ dst, const uint4* __restrict__ src, size_t n16)
{
    for (size_t k = (size_t)blockIdx.x * 256 + threadIdx.x; k < n16; k += (size_t)gridDim.x * 256) dst[k] = src[k];
}

// ---------------------------------------------------------- parallel tempering
// Lattices of equal L form a ladder (ladders ordered by L); rung t of ladder g
// has the temperature (beta, delta) of rung_param[start_g + t]; member[start_g +
// t] is the lattice on it.  After a round (its last sweep measured into
// round_obs[i]), the lattices a, b on rungs t, t+1 (t = parity, parity + 2, ...)
// exchange rungs iff u < exp((beta_t - beta_t+1)(E_a - E_b)), E = -(Cx + Cy),
// u = u(X0) of Philox counter (round, g, 4, t) keyed by the tempering seed; an
// exchange rewrites the two lattices' descriptors (delta, -beta log2 e).
struct Rung {
    double beta;
    float delta, nbl2e;      // as in LatDesc
};

// One workgroup; slots k = 0 .. n-1 of `member` (ladders are contiguous runs of
// slots).  First every slot's record and rung of the round are written, then the
// exchanges run one thread per pair of slots (the pairs of a round are disjoint,
// and each decision depends only on its own pair).
__device__ __forceinline__ int ladder_of(const int2* __restrict__ ladders, int nlad, int k)
{
    int g = 0;
    while (g + 1 < nlad && ladders[g + 1].x <= k) ++g;
    return g;
}

__global__ void __launch_bounds__(256)
k_batch_exchange(LatDesc* __restrict__ lat, int* __restrict__ member, const int2* __restrict__ ladders, int nlad,
                 const Rung* __restrict__ rung, const xy_obs* __restrict__ round_obs, uint32_t round, uint32_t k0,
                 uint32_t k1, xy_obs* __restrict__ obs_out, int32_t* __restrict__ rung_out)
{
    const int n = ladders[nlad - 1].x + ladders[nlad - 1].y;
    for (int k = threadIdx.x; k < n; k += 256) {
        const int i = member[k];
        if (obs_out) obs_out[i] = round_obs[i];
        if (rung_out) rung_out[i] = k - ladders[ladder_of(ladders, nlad, k)].x;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < n; k += 256) {
        const int g = ladder_of(ladders, nlad, k);
        const int start = ladders[g].x, len = ladders[g].y, t = k - start;
        if (((t ^ (int)round) & 1) != 0 || t + 1 >= len) continue;
        const int a = member[k], b = member[k + 1];
        const double ea = -(round_obs[a].cx + round_obs[a].cy), eb = -(round_obs[b].cx + round_obs[b].cy);
        const Rung ra = rung[k], rb = rung[k + 1];
        const u32x4 w = philox10(round, (uint32_t)g, 4u, (uint32_t)t, k0, k1);
        if ((double)u01(w.x) < exp((ra.beta - rb.beta) * (ea - eb))) {
            member[k] = b;
            member[k + 1] = a;
            lat[a].delta = rb.delta;
            lat[a].nbl2e = rb.nbl2e;
            lat[b].delta = ra.delta;
            lat[b].nbl2e = ra.nbl2e;
        }
    }
}

__global__ void k_zero_u32(unsigned* p, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

__global__ void k_set_sweep(Ctrl* ctrl, uint32_t v)
{
    ctrl->sweep0 = v;
    ctrl->timed_out = 0u;
    ctrl->spin_limit = kSpinLimit;
}

__global__ void k_set_spin_limit(Ctrl* ctrl, uint32_t v) { ctrl->spin_limit = v; }

}  // namespace xyb

// ===================================================================== host side
namespace xyb {

struct Shape {
    int tx, ty;
};
// Batch tile shapes, largest first.  Shapes of at least 512 sites are preferred;
// the small ones exist so that any batch of L % 4 == 0 lattices can run.
static const Shape kShapes[] = {{64, 32}, {64, 16}, {32, 16}, {16, 16}, {8, 8}, {4, 4}};
static constexpr int kNT = 256;
// Streams a batched HMC trajectory forks into (lattices run side by side).
static constexpr int kHmcStreams = 4;
// Longest per-sweep launch sequence captured in one graph (longer calls replay it).
static constexpr int kMaxGraphPasses = 16384;

static std::vector<Shape> candidates(int n, const int32_t* L)
{
    std::vector<Shape> big, all;
    for (const Shape& s : kShapes) {
        bool ok = true;
        for (int i = 0; i < n && ok; ++i) ok = (L[i] % s.tx == 0) && (L[i] % s.ty == 0);
        if (!ok) continue;
        all.push_back(s);
        if (s.tx * s.ty >= 512) big.push_back(s);
    }
    if (!big.empty()) return big;
    if (!all.empty()) return {all.front()};
    return {};
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct Layout {
    size_t state_bytes, pp_off, ctrl_off, bar_off, desc_off, xplan_off, res_off, tile_off, part_off, td_off, pt_off,
        total;
    long long max_tiles;
};

// Tempering area: per lattice one round record, one ladder member slot, one rung
// and one ladder-table entry.
struct PtArea {
    xy_obs* round_obs;
    int* member;
    Rung* rung;
    int2* ladders;
};

static size_t pt_bytes(int n) { return (size_t)n * (sizeof(xy_obs) + sizeof(int) + sizeof(Rung) + sizeof(int2)) + 4 * 256; }

static Layout layout(int n, const int32_t* L, int precision)
{
    Layout lo{};
    const size_t elem = precision == XY_FP16 ? 2 : 4;
    long long sites = 0;
    for (int i = 0; i < n; ++i) sites += (long long)L[i] * L[i];
    lo.state_bytes = (size_t)sites * elem;
    std::vector<Shape> c = candidates(n, L);
    int min_area = 1 << 30;
    for (const Shape& s : c) min_area = std::min(min_area, s.tx * s.ty);
    lo.max_tiles = c.empty() ? 0 : sites / min_area;
    lo.pp_off = 0;
    lo.ctrl_off = align256(lo.state_bytes);
    lo.bar_off = lo.ctrl_off + 256;
    lo.desc_off = align256(lo.bar_off + (size_t)(n + kXcd + 1) * sizeof(unsigned));
    lo.xplan_off = align256(lo.desc_off + (size_t)n * sizeof(LatDesc));
    lo.res_off = align256(lo.xplan_off + sizeof(XcdPlan) + (size_t)n * sizeof(int));
    lo.tile_off = align256(lo.res_off + (size_t)n * sizeof(int));
    lo.part_off = align256(lo.tile_off + (size_t)lo.max_tiles * sizeof(int));
    lo.td_off = align256(lo.part_off + (size_t)2 * lo.max_tiles * 8 * sizeof(double));
    lo.pt_off = align256(lo.td_off + (size_t)lo.max_tiles * sizeof(unsigned));
    lo.total = lo.pt_off + pt_bytes(n);
    return lo;
}

template <typename T, int TX, int TY>
static void* kernel_ptr()
{
    return (void*)k_batch<T, TX, TY, kNT>;
}

template <typename T, int TX, int TY, bool WIDE>
static void* pass_kernel_ptr(bool meas)
{
    return meas ? (void*)k_batch_pass<T, TX, TY, -1, WIDE> : (void*)k_batch_pass<T, TX, TY, 0, WIDE>;
}

// The per-pass kernel for shape s (wide tiles or not, measured or not) and its LDS bytes.
static void* pass_kernel(int precision, Shape s, bool wide, bool meas, size_t* lds)
{
#define XYB_CASE(TXV, TYV)                                                                          \
    if (s.tx == TXV && s.ty == TYV) {                                                               \
        *lds = wide ? pass_lds<TXV, TYV, true>() : pass_lds<TXV, TYV, false>();                     \
        if (precision == XY_FP16)                                                                   \
            return wide ? pass_kernel_ptr<__half, TXV, TYV, true>(meas)                             \
                        : pass_kernel_ptr<__half, TXV, TYV, false>(meas);                           \
        return wide ? pass_kernel_ptr<float, TXV, TYV, true>(meas) : pass_kernel_ptr<float, TXV, TYV, false>(meas); \
    }
    XYB_CASE(64, 32)
    XYB_CASE(64, 16)
    XYB_CASE(32, 16)
    XYB_CASE(16, 16)
    XYB_CASE(8, 8)
    XYB_CASE(4, 4)
#undef XYB_CASE
    return nullptr;
}

static void* batch_kernel(int precision, Shape s, size_t* lds)
{
#define XYB_CASE(TXV, TYV)                                                                         \
    if (s.tx == TXV && s.ty == TYV) {                                                              \
        *lds = pass_lds<TXV, TYV, true>();                                                          \
        return precision == XY_FP16 ? kernel_ptr<__half, TXV, TYV>() : kernel_ptr<float, TXV, TYV>(); \
    }
    XYB_CASE(64, 32)
    XYB_CASE(64, 16)
    XYB_CASE(32, 16)
    XYB_CASE(16, 16)
    XYB_CASE(8, 8)
    XYB_CASE(4, 4)
#undef XYB_CASE
    return nullptr;
}

}  // namespace xyb

using namespace xyb;

static const uint32_t kBatchMagic = 0x58594254u;  // "XYBT"

struct xy_batch {
    uint32_t magic;
    uint32_t pt_round;     // index of the next tempering round (exchange random numbers)
    int n;
    std::vector<int32_t> L;
    std::vector<uint64_t> seed;
    std::vector<double> beta, delta;
    int precision;
    char* state;
    char* work;
    size_t state_len, work_len;
    hipStream_t stream;
    hipStream_t cap;       // private stream used only for graph capture
    uint64_t sweep;
    Layout lo;
    Shape shape;
    int sched;             // XY_BATCH_PERSISTENT, XY_BATCH_PASSES or XY_BATCH_PASSES_WIDE
    hipStream_t cap2;      // second capture stream: the LDS-resident lattices
    hipEvent_t ev_fork, ev_join;
    int nres, res_maxL;    // LDS-resident lattices and their largest L
    int grid;
    int total_tiles;
    std::vector<LatDesc> desc;
    hipGraph_t graph;
    hipGraphExec_t exec;
    int64_t g_n;
    int32_t g_me;
    xy_obs* g_obs;
    int g_nrec;
    int g_grid;
    int g_sched;
    // batched HMC: extra capture streams, join events and the cached graph of one
    // trajectory of every lattice (key: n_md, eps, steps per pass, workspace, records on/off)
    hipStream_t hs[kHmcStreams];
    hipEvent_t hev[kHmcStreams];
    hipGraph_t hgraph;
    hipGraphExec_t hexec;
    int32_t h_nmd, h_steps;
    double h_eps;
    void* h_work;
    xy_hmc_obs* h_obs;
    int64_t h_ntraj;
    uint64_t h_pgen;
    int32_t hmc_steps;     // leap-frog steps per pass of xy_batch_hmc
    // batched HMC stages of the cached graph: descriptors and block offsets (host
    // copies; the graph reads them from the caller's HMC workspace, where every
    // call writes them again before its replays)
    std::vector<xyk::BhLat> h_desc;
    std::vector<uint32_t> h_start;
    uint64_t pgen;         // bumped whenever a lattice's beta or delta changes
};

static bool blive(const xy_batch* b) { return b && b->magic == kBatchMagic; }

static void drop_graph(xy_batch* b);

// Graph, streams and events of a batch, then the handle itself.
static void drop_hmc_graph(xy_batch* b)
{
    if (b->hexec) (void)hipGraphExecDestroy(b->hexec);
    if (b->hgraph) (void)hipGraphDestroy(b->hgraph);
    b->hexec = nullptr;
    b->hgraph = nullptr;
    // queued copies read the host descriptors: let them finish before they go
    if (!b->h_desc.empty()) (void)hipStreamSynchronize(b->stream);
    b->h_desc.clear();
    b->h_start.clear();
}

static void release(xy_batch* b)
{
    drop_graph(b);
    drop_hmc_graph(b);
    for (int k = 0; k < kHmcStreams; ++k) {
        if (b->hs[k]) (void)hipStreamDestroy(b->hs[k]);
        if (b->hev[k]) (void)hipEventDestroy(b->hev[k]);
    }
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->cap2) (void)hipStreamDestroy(b->cap2);
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    if (b->ev_join) (void)hipEventDestroy(b->ev_join);
    b->magic = 0;
    delete b;
}

static void drop_graph(xy_batch* b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

// Plan the work list for shape s: tiles per lattice, grid size (all workgroups
// resident), contiguous tile ranges, barrier arrival counts and reducers.
static int plan_batch(xy_batch* b, Shape s)
{
    size_t lds = 0;
    void* k = batch_kernel(b->precision, s, &lds);
    if (!k) return XY_EINVAL;
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return xyr::hip_fail(e, "hipFuncSetAttribute");
    for (int m = 0; m < 4; ++m) {
        size_t pl = 0;
        void* pk = pass_kernel(b->precision, s, (m & 2) != 0, (m & 1) != 0, &pl);
        if (!pk) return XY_EINVAL;
        if ((e = hipFuncSetAttribute(pk, hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl)) != hipSuccess)
            return xyr::hip_fail(e, "hipFuncSetAttribute");
    }
    int dev = 0, cus = 0, per_cu = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return xyr::hip_fail(e, "hipGetDevice");
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
        return xyr::hip_fail(e, "hipDeviceGetAttribute");
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kNT, lds)) != hipSuccess)
        return xyr::hip_fail(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
    if (per_cu < 1) return XY_EINVAL;
    int total = 0;
    b->desc.assign(b->n, LatDesc{});
    long long off = 0;
    for (int i = 0; i < b->n; ++i) {
        LatDesc& d = b->desc[i];
        d.off = off;
        d.L = b->L[i];
        d.resident = b->sched != XY_BATCH_PERSISTENT && d.L <= kBatchResidentMaxL && xyk::resident_supported(d.L);
        d.wide = b->sched != XY_BATCH_PASSES && d.L % kWideX == 0 && d.L % kWideY == 0;
        const int tx = d.wide ? kWideX : s.tx, ty = d.wide ? kWideY : s.ty;
        d.tiles_x = d.L / tx;
        d.first_tile = total;
        d.ntiles = d.resident ? 0 : (d.L / tx) * (d.L / ty);
        xyk::SweepArgs a = xyr::sweep_args(b->seed[i], d.L, b->precision, b->beta[i], b->delta[i]);
        d.key0 = a.key0;
        d.key1 = a.key1;
        d.delta = a.delta;
        d.nbl2e = a.nbl2e;
        total += d.ntiles;
        off += (long long)d.L * d.L;
    }
    if ((long long)total > b->lo.max_tiles) return XY_EINVAL;
    // Persistent schedule: lattices into kXcd groups of about equal tile count,
    // largest first onto the lightest group; within a group in lattice order.
    std::vector<int> by_size(b->n);
    for (int i = 0; i < b->n; ++i) by_size[i] = i;
    std::stable_sort(by_size.begin(), by_size.end(),
                     [&](int u, int v) { return b->desc[u].ntiles > b->desc[v].ntiles; });
    long long load[kXcd] = {0};
    for (int i : by_size) {
        int best = 0;
        for (int y = 1; y < kXcd; ++y)
            if (load[y] < load[best]) best = y;
        b->desc[i].xcd = best;
        load[best] += b->desc[i].ntiles;
    }
    XcdPlan plan{};
    std::vector<int> ord;
    for (int y = 0; y < kXcd; ++y) {
        plan.beg[y] = (int)ord.size();
        int t = 0;
        for (int i = 0; i < b->n; ++i)
            if (b->desc[i].xcd == y) {
                b->desc[i].xfirst = t;
                t += b->desc[i].ntiles;
                ord.push_back(i);
            }
        plan.tiles[y] = t;
    }
    plan.beg[kXcd] = (int)ord.size();
    // every workgroup must be resident at once for the barriers; keep a margin of
    // one resident slot in ten in case part of the GPU is busy with other work.
    // At most three workgroups per CU: more (up to the occupancy limit) were
    // slower, as each adds waits to every barrier of its lattices.  A multiple of
    // kXcd workgroups, so that each XCD gets the same number.
    const int G = std::max(kXcd, std::min(total, std::min(cus * 3, cus * per_cu * 9 / 10)) / kXcd * kXcd);
    b->shape = s;
    b->grid = G;
    b->total_tiles = total;
    std::vector<int> ridx;
    b->res_maxL = 0;
    for (int i = 0; i < b->n; ++i)
        if (b->desc[i].resident) {
            ridx.push_back(i);
            b->res_maxL = std::max(b->res_maxL, b->desc[i].L);
        }
    b->nres = (int)ridx.size();
    e = hipMemcpyAsync(b->work + b->lo.desc_off, b->desc.data(), sizeof(LatDesc) * b->n, hipMemcpyHostToDevice,
                       b->stream);
    if (e != hipSuccess) return xyr::hip_fail(e, "hipMemcpyAsync(desc)");
    e = hipMemcpyAsync(b->work + b->lo.xplan_off, &plan, sizeof(XcdPlan), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->work + b->lo.xplan_off + sizeof(XcdPlan), ord.data(), sizeof(int) * ord.size(),
                           hipMemcpyHostToDevice, b->stream);
    if (e != hipSuccess) return xyr::hip_fail(e, "hipMemcpyAsync(XCD groups)");
    if (b->nres > 0) {
        e = hipMemcpyAsync(b->work + b->lo.res_off, ridx.data(), sizeof(int) * ridx.size(), hipMemcpyHostToDevice,
                           b->stream);
        if (e != hipSuccess) return xyr::hip_fail(e, "hipMemcpyAsync(resident list)");
    }
    // tile -> lattice table of the work list (the per-sweep kernels read it)
    std::vector<int> tl((size_t)total);
    for (int i = 0; i < b->n; ++i)
        for (int t = 0; t < b->desc[i].ntiles; ++t) tl[(size_t)b->desc[i].first_tile + t] = i;
    if (total > 0) {
        e = hipMemcpyAsync(b->work + b->lo.tile_off, tl.data(), sizeof(int) * tl.size(), hipMemcpyHostToDevice,
                           b->stream);
        if (e != hipSuccess) return xyr::hip_fail(e, "hipMemcpyAsync(tile table)");
    }
    if ((e = hipStreamSynchronize(b->stream)) != hipSuccess) return xyr::hip_fail(e, "hipStreamSynchronize");
    drop_graph(b);
    return XY_OK;
}

static hipError_t enqueue_batch(xy_batch* b, hipStream_t s, int npass, int32_t me, xy_obs* obs, int nrec)
{
    size_t lds = 0;
    void* k = batch_kernel(b->precision, b->shape, &lds);
    unsigned* bar = (unsigned*)(b->work + b->lo.bar_off);
    Ctrl* ctrl = (Ctrl*)(b->work + b->lo.ctrl_off);
    const LatDesc* desc = (const LatDesc*)(b->work + b->lo.desc_off);
    double* part = (double*)(b->work + b->lo.part_off);
    const XcdPlan* plan = (const XcdPlan*)(b->work + b->lo.xplan_off);
    unsigned* tdone = (unsigned*)(b->work + b->lo.td_off);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(256), 0, s, bar, b->n + kXcd + 1);
    hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)std::min(1024, (b->total_tiles + 255) / 256 + 1)), dim3(256), 0, s,
                       tdone, b->total_tiles);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    void* pp = b->work + b->lo.pp_off;
    void* st = b->state;
    int nlat = b->n, tt = b->total_tiles;
    void* args[] = {&st, &pp, &desc, &plan, &nlat, &tt, &bar, &tdone, &ctrl, &npass, &me, &part, &obs, (void*)&nrec};
    e = hipLaunchKernel(k, dim3(b->grid), dim3(kNT), args, lds, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_batch_advance, dim3(1), dim3(1), 0, s, ctrl, (uint32_t)npass);
    return hipGetLastError();
}

// Per-pass schedule: one launch per pass over all tiles, a record kernel after each
// measured pass, a copy back for an odd pass count, then the sweep counter.
static hipError_t enqueue_passes(xy_batch* b, hipStream_t s, int npass, int32_t me, xy_obs* obs, int nrec)
{
    Ctrl* ctrl = (Ctrl*)(b->work + b->lo.ctrl_off);
    const LatDesc* desc = (const LatDesc*)(b->work + b->lo.desc_off);
    double* part = (double*)(b->work + b->lo.part_off);
    void* pp = b->work + b->lo.pp_off;
    int nlat = b->n, tt = b->total_tiles;
    hipError_t e = hipSuccess;
    if (b->nres > 0) {
        // the LDS-resident lattices on the second stream, beside the passes below
        if ((e = hipEventRecord(b->ev_fork, s)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(b->cap2, b->ev_fork, 0)) != hipSuccess) return e;
        void* out = (npass & 1) ? pp : (void*)b->state;
        const int* ridx = (const int*)(b->work + b->lo.res_off);
        const size_t lds = resident_lds_bytes(b->res_maxL, kNT);
        if (b->precision == XY_FP16)
            hipLaunchKernelGGL(k_batch_resident<__half>, dim3(b->nres), dim3(kNT), lds, b->cap2,
                               (const __half*)b->state, (__half*)out, desc, ridx, (const Ctrl*)ctrl, npass, me, obs,
                               nrec);
        else
            hipLaunchKernelGGL(k_batch_resident<float>, dim3(b->nres), dim3(kNT), lds, b->cap2,
                               (const float*)b->state, (float*)out, desc, ridx, (const Ctrl*)ctrl, npass, me, obs,
                               nrec);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = hipEventRecord(b->ev_join, b->cap2)) != hipSuccess) return e;
    }
    for (int p = 0; p < npass && tt > 0; ++p) {
        const bool meas = me > 0 && ((p + 1) % me) == 0;
        size_t lds = 0;
        void* k = pass_kernel(b->precision, b->shape, b->sched == XY_BATCH_PASSES_WIDE, meas, &lds);
        void* src = (p & 1) ? pp : (void*)b->state;
        void* dst = (p & 1) ? (void*)b->state : pp;
        int pv = p;
        const int* tile_lat = (const int*)(b->work + b->lo.tile_off);
        void* args[] = {&src, &dst, &desc, &tile_lat, &tt, &ctrl, &pv, &part};
        const unsigned grid = (unsigned)((tt + 7) & ~7);
        if ((e = hipLaunchKernel(k, dim3(grid), dim3(kNT), args, lds, s)) != hipSuccess) return e;
        if (meas) {
            hipLaunchKernelGGL(k_batch_reduce, dim3(nlat), dim3(kNT), 0, s, desc, (const Ctrl*)ctrl, p,
                               (const double*)part, obs, nrec, (p + 1) / me - 1);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    if (b->nres > 0 && (e = hipStreamWaitEvent(s, b->ev_join, 0)) != hipSuccess) return e;
    if (npass & 1) {
        const size_t n16 = b->lo.state_bytes / 16;
        const int grid = (int)std::min<size_t>((n16 + kNT - 1) / kNT, 4096);
        hipLaunchKernelGGL(k_batch_copy, dim3(grid), dim3(kNT), 0, s, (uint4*)b->state, (const uint4*)pp, n16);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_batch_advance, dim3(1), dim3(1), 0, s, ctrl, (uint32_t)npass);
    return hipGetLastError();
}

extern "C" {

int xy_batch_state_bytes(int32_t n, const int32_t* L, int32_t precision, size_t* state, size_t* workspace)
{
    if (n <= 0 || !L || (precision != XY_FP32 && precision != XY_FP16)) return XY_EINVAL;
    for (int i = 0; i < n; ++i)   // tiles address each lattice with 32-bit byte offsets
        if (!xyr::valid_L(L[i]) || L[i] % 4 != 0 || (long long)L[i] * L[i] * 4 >= (1LL << 32)) return XY_EINVAL;
    if (candidates(n, L).empty()) return XY_EINVAL;
    Layout lo = layout(n, L, precision);
    if (state) *state = lo.state_bytes;
    if (workspace) *workspace = lo.total;
    return XY_OK;
}

int xy_batch_init(xy_batch** out, int32_t n, const uint64_t* seeds, const int32_t* L, const double* beta,
                  const double* delta, int32_t start, int32_t precision, void* state_dev, size_t state_len,
                  void* work_dev, size_t work_len, void* hip_stream)
{
    if (!out) return XY_ESTATE;
    *out = nullptr;
    if (!seeds || !L || !beta || !delta) return XY_ESTATE;
    size_t need_s = 0, need_w = 0;
    int rc = xy_batch_state_bytes(n, L, precision, &need_s, &need_w);
    if (rc != XY_OK) return rc;
    if (start != XY_HOT && start != XY_COLD) return XY_EINVAL;
    for (int i = 0; i < n; ++i)
        if (!xyr::valid_beta_delta(beta[i], delta[i])) return XY_EINVAL;
    if (!state_dev || !work_dev) return XY_ESTATE;
    if (state_len < need_s || work_len < need_w) return XY_ESIZE;
    xy_batch* b = new (std::nothrow) xy_batch;
    if (!b) return XY_ENOMEM;
    b->magic = kBatchMagic;
    b->n = n;
    b->L.assign(L, L + n);
    b->seed.assign(seeds, seeds + n);
    b->beta.assign(beta, beta + n);
    b->delta.assign(delta, delta + n);
    b->precision = precision;
    b->state = (char*)state_dev;
    b->work = (char*)work_dev;
    b->state_len = state_len;
    b->work_len = work_len;
    b->stream = (hipStream_t)hip_stream;
    b->cap = nullptr;
    b->cap2 = nullptr;
    b->ev_fork = nullptr;
    b->ev_join = nullptr;
    b->nres = 0;
    b->res_maxL = 0;
    b->sweep = 0;
    b->pt_round = 0;
    b->lo = layout(n, L, precision);
    b->graph = nullptr;
    b->exec = nullptr;
    b->g_n = -1;
    b->g_me = -1;
    b->g_nrec = -1;
    b->g_obs = nullptr;
    b->g_grid = 0;
    b->g_sched = -1;
    for (int k = 0; k < kHmcStreams; ++k) {
        b->hs[k] = nullptr;
        b->hev[k] = nullptr;
    }
    b->hgraph = nullptr;
    b->hexec = nullptr;
    b->h_nmd = -1;
    b->h_steps = -1;
    b->h_eps = 0.0;
    b->h_work = nullptr;
    b->h_obs = nullptr;
    b->h_ntraj = -1;
    b->h_pgen = ~0ull;
    b->hmc_steps = 7;
    b->pgen = 0;
    b->sched = XY_BATCH_PASSES_WIDE;
    auto fail = [&](int code) {
        release(b);
        return code;
    };
    hipError_t e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        b->cap = nullptr;
        return fail(xyr::hip_fail(e, "hipStreamCreate"));
    }
    if ((e = hipStreamCreateWithFlags(&b->cap2, hipStreamNonBlocking)) != hipSuccess) {
        b->cap2 = nullptr;
        return fail(xyr::hip_fail(e, "hipStreamCreate"));
    }
    if ((e = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming)) != hipSuccess) {
        b->ev_fork = nullptr;
        return fail(xyr::hip_fail(e, "hipEventCreate"));
    }
    if ((e = hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming)) != hipSuccess) {
        b->ev_join = nullptr;
        return fail(xyr::hip_fail(e, "hipEventCreate"));
    }
    rc = plan_batch(b, candidates(n, L).front());
    if (rc != XY_OK) return fail(rc);
    for (int i = 0; i < n; ++i) {
        const size_t eb = precision == XY_FP16 ? 2 : 4;
        e = xyk::launch_init(b->state + b->desc[i].off * eb, L[i], precision, (uint32_t)(seeds[i] & 0xffffffffu),
                             (uint32_t)(seeds[i] >> 32), start == XY_HOT, b->stream);
        if (e != hipSuccess) return fail(xyr::hip_fail(e, "xy_batch_init: launch"));
    }
    hipLaunchKernelGGL(k_set_sweep, dim3(1), dim3(1), 0, b->stream, (Ctrl*)(b->work + b->lo.ctrl_off), 0u);
    if ((e = hipGetLastError()) != hipSuccess) return fail(xyr::hip_fail(e, "xy_batch_init: launch"));
    *out = b;
    return XY_OK;
}

// One launch sequence of n sweeps (graph captured once per (n, records, stride,
// grid, schedule) and replayed); records of lattice i at obs[i * nrec + r].
static int batch_sweep_chunk(xy_batch* b, int n, int32_t me, xy_obs* obs, int nrec)
{
    hipError_t e;
    if (!b->exec || b->g_n != n || b->g_me != me || b->g_obs != obs || b->g_nrec != nrec || b->g_grid != b->grid ||
        b->g_sched != b->sched) {
        drop_graph(b);
        if ((e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal)) != hipSuccess)
            return xyr::hip_fail(e, "hipStreamBeginCapture");
        hipError_t le = b->sched == XY_BATCH_PERSISTENT ? enqueue_batch(b, b->cap, n, me, obs, nrec)
                                                        : enqueue_passes(b, b->cap, n, me, obs, nrec);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(b->cap, &g);
        if (le != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return xyr::hip_fail(le, "batch launch (capture)");
        }
        if (e != hipSuccess) return xyr::hip_fail(e, "hipStreamEndCapture");
        b->graph = g;
        if ((e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0)) != hipSuccess) {
            b->exec = nullptr;
            drop_graph(b);
            return xyr::hip_fail(e, "hipGraphInstantiate");
        }
        b->g_n = n;
        b->g_me = me;
        b->g_obs = obs;
        b->g_nrec = nrec;
        b->g_grid = b->grid;
        b->g_sched = b->sched;
    }
    if ((e = XY_LAUNCH(hipGraphLaunch(b->exec, b->stream))) != hipSuccess) return xyr::hip_fail(e, "hipGraphLaunch");
    b->sweep += (uint64_t)n;
    return XY_OK;
}

int xy_batch_sweep(xy_batch* b, int64_t n_sweeps, int32_t measure_every, xy_obs* obs_dev)
{
    if (!blive(b)) return XY_ESTATE;
    if (n_sweeps < 0 || measure_every < 0) return XY_EINVAL;
    if (b->sweep + (uint64_t)n_sweeps >= 0xffffffffull) return XY_ERANGE;
    if (n_sweeps == 0) return XY_OK;
    const int32_t me = (obs_dev && measure_every > 0) ? measure_every : 0;
    xy_obs* obs = me ? obs_dev : nullptr;
    const int64_t nrec = me ? n_sweeps / me : 0;   // records per lattice: the stride of obs_dev
    if (nrec > INT32_MAX) return XY_EINVAL;
    // Split long calls: pass counts are ints and counters 32 bits (at most 2^30
    // sweeps per launch sequence, fewer for huge tile counts), and the per-sweep
    // schedules capture one launch per sweep (at most kMaxGraphPasses per graph).
    // Chunks are multiples of measure_every, so the records of chunk c start at
    // record done / measure_every of every lattice, with the call's stride.
    int max_tiles = 1;
    for (const LatDesc& d : b->desc) max_tiles = std::max(max_tiles, d.ntiles);
    int64_t cap = std::min<int64_t>((int64_t)1 << 30,
                                    std::max<int64_t>(1, (int64_t)(0xffffffffu / (unsigned)max_tiles) - 1));
    if (b->sched != XY_BATCH_PERSISTENT) cap = std::min<int64_t>(cap, kMaxGraphPasses);
    if (me) cap = std::max<int64_t>(cap / me, 1) * me;
    for (int64_t done = 0; done < n_sweeps;) {
        const int64_t m = std::min(cap, n_sweeps - done);
        int rc = batch_sweep_chunk(b, (int)m, me, obs ? obs + done / me : nullptr, (int)nrec);
        if (rc != XY_OK) return rc;
        done += m;
    }
    return XY_OK;
}

int xy_batch_get_sweep(const xy_batch* b, uint64_t* sweep)
{
    if (!blive(b) || !sweep) return XY_ESTATE;
    *sweep = b->sweep;
    return XY_OK;
}

int xy_batch_autotune(xy_batch* b, int32_t sweeps_per_trial, int32_t* tile_x, int32_t* tile_y)
{
    if (!blive(b)) return XY_ESTATE;
    if (sweeps_per_trial < 2) return XY_EINVAL;
    std::vector<Shape> cands = candidates(b->n, b->L.data());
    hipEvent_t e0, e1;
    hipError_t e;
    if ((e = hipEventCreate(&e0)) != hipSuccess) return xyr::hip_fail(e, "hipEventCreate");
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return xyr::hip_fail(e, "hipEventCreate");
    }
    double best = 1e300;
    Shape bs = b->shape;
    int bsched = b->sched;
    int rc = XY_OK;
    static const int scheds[3] = {XY_BATCH_PASSES_WIDE, XY_BATCH_PASSES, XY_BATCH_PERSISTENT};
    for (int ci = 0; ci < 3 * (int)cands.size(); ++ci) {
        const Shape s = cands[ci / 3];
        b->sched = scheds[ci % 3];
        if ((rc = plan_batch(b, s)) != XY_OK) break;
        if ((rc = xy_batch_sweep(b, sweeps_per_trial, 0, nullptr)) != XY_OK) break;   // warm-up, capture
        if ((e = hipEventRecord(e0, b->stream)) != hipSuccess) { rc = xyr::hip_fail(e, "hipEventRecord"); break; }
        if ((rc = xy_batch_sweep(b, sweeps_per_trial, 0, nullptr)) != XY_OK) break;
        if ((e = hipEventRecord(e1, b->stream)) != hipSuccess) { rc = xyr::hip_fail(e, "hipEventRecord"); break; }
        if ((e = hipEventSynchronize(e1)) != hipSuccess) { rc = xyr::hip_fail(e, "hipEventSynchronize"); break; }
        float ms = 0.f;
        if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) { rc = xyr::hip_fail(e, "hipEventElapsedTime"); break; }
        if (ms < best) {
            best = ms;
            bs = s;
            bsched = b->sched;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->sched = bsched;
    if (rc != XY_OK) return rc;
    if ((rc = plan_batch(b, bs)) != XY_OK) return rc;
    if (tile_x) *tile_x = bs.tx;
    if (tile_y) *tile_y = bs.ty;
    return XY_OK;
}

int xy_batch_set_tile(xy_batch* b, int32_t tile_x, int32_t tile_y)
{
    if (!blive(b)) return XY_ESTATE;
    for (const Shape& s : candidates(b->n, b->L.data()))
        if (s.tx == tile_x && s.ty == tile_y) return plan_batch(b, s);
    return XY_EINVAL;
}

int xy_batch_get_tile(const xy_batch* b, int32_t* tile_x, int32_t* tile_y)
{
    if (!blive(b)) return XY_ESTATE;
    if (tile_x) *tile_x = b->shape.tx;
    if (tile_y) *tile_y = b->shape.ty;
    return XY_OK;
}

int xy_batch_set_schedule(xy_batch* b, int32_t schedule)
{
    if (!blive(b)) return XY_ESTATE;
    if (schedule != XY_BATCH_PERSISTENT && schedule != XY_BATCH_PASSES && schedule != XY_BATCH_PASSES_WIDE)
        return XY_EINVAL;
    if (schedule == b->sched) return XY_OK;
    const int old = b->sched;
    b->sched = schedule;
    const int rc = plan_batch(b, b->shape);   // the work list depends on the schedule
    if (rc != XY_OK) b->sched = old;
    return rc;
}

int xy_batch_get_schedule(const xy_batch* b, int32_t* schedule)
{
    if (!blive(b) || !schedule) return XY_ESTATE;
    *schedule = b->sched;
    return XY_OK;
}

int xy_batch_tempering(xy_batch* b, int64_t n_rounds, int32_t sweeps_per_round, uint64_t pt_seed, xy_obs* obs_dev,
                       int32_t* rung_dev)
{
    if (!blive(b)) return XY_ESTATE;
    if (n_rounds < 0 || sweeps_per_round < 1) return XY_EINVAL;
    if (b->sweep + (uint64_t)n_rounds * (uint64_t)sweeps_per_round >= 0xffffffffull ||
        (uint64_t)b->pt_round + (uint64_t)n_rounds >= 0xffffffffull)
        return XY_ERANGE;
    if (n_rounds == 0) return XY_OK;
    const int n = b->n;
    // ladders: lattices of equal L in order of L, each ordered by (beta, index)
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        if (b->L[x] != b->L[y]) return b->L[x] < b->L[y];
        return b->beta[x] < b->beta[y];
    });
    std::vector<int> member(n);
    std::vector<Rung> rung(n);
    std::vector<int2> ladders;
    for (int k = 0; k < n; ++k) {
        const int i = order[k];
        if (k == 0 || b->L[i] != b->L[order[k - 1]]) ladders.push_back(make_int2(k, 0));
        ladders.back().y += 1;
        member[k] = i;
        const xyk::SweepArgs a = xyr::sweep_args(b->seed[i], b->L[i], b->precision, b->beta[i], b->delta[i]);
        rung[k].beta = b->beta[i];
        rung[k].delta = a.delta;
        rung[k].nbl2e = a.nbl2e;
    }
    std::vector<double> rbeta(n), rdelta(n);
    for (int k = 0; k < n; ++k) {
        rbeta[k] = b->beta[order[k]];
        rdelta[k] = b->delta[order[k]];
    }
    char* pt = b->work + b->lo.pt_off;
    PtArea area;
    area.round_obs = (xy_obs*)pt;
    area.member = (int*)(pt + align256((size_t)n * sizeof(xy_obs)));
    area.rung = (Rung*)((char*)area.member + align256((size_t)n * sizeof(int)));
    area.ladders = (int2*)((char*)area.rung + align256((size_t)n * sizeof(Rung)));
    hipError_t e;
    if ((e = hipMemcpyAsync(area.member, member.data(), sizeof(int) * n, hipMemcpyHostToDevice, b->stream)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(area.rung, rung.data(), sizeof(Rung) * n, hipMemcpyHostToDevice, b->stream)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(area.ladders, ladders.data(), sizeof(int2) * ladders.size(), hipMemcpyHostToDevice,
                            b->stream)) != hipSuccess)
        return xyr::hip_fail(e, "xy_batch_tempering: upload");
    const uint32_t k0 = (uint32_t)(pt_seed & 0xffffffffu), k1 = (uint32_t)(pt_seed >> 32);
    LatDesc* desc = (LatDesc*)(b->work + b->lo.desc_off);
    for (int64_t r = 0; r < n_rounds; ++r) {
        int rc = xy_batch_sweep(b, sweeps_per_round, sweeps_per_round, area.round_obs);
        if (rc != XY_OK) return rc;
        hipLaunchKernelGGL(k_batch_exchange, dim3(1), dim3(256), 0, b->stream, desc, area.member, area.ladders,
                           (int)ladders.size(), area.rung, area.round_obs, b->pt_round + (uint32_t)r, k0, k1,
                           obs_dev ? obs_dev + (size_t)r * n : nullptr, rung_dev ? rung_dev + (size_t)r * n : nullptr);
        if ((e = hipGetLastError()) != hipSuccess) return xyr::hip_fail(e, "xy_batch_tempering: exchange launch");
    }
    b->pt_round += (uint32_t)n_rounds;
    // the host copies of beta and delta follow the lattices to their new rungs
    if ((e = hipMemcpyAsync(member.data(), area.member, sizeof(int) * n, hipMemcpyDeviceToHost, b->stream)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(b->stream)) != hipSuccess)
        return xyr::hip_fail(e, "xy_batch_tempering: read back");
    for (int k = 0; k < n; ++k) {
        b->beta[member[k]] = rbeta[k];
        b->delta[member[k]] = rdelta[k];
    }
    b->pgen += 1;        // graphs that hold a lattice's beta are out of date
    return XY_OK;
}

int xy_batch_get_params(const xy_batch* b, double* beta, double* delta)
{
    if (!blive(b)) return XY_ESTATE;
    for (int i = 0; i < b->n; ++i) {
        if (beta) beta[i] = b->beta[i];
        if (delta) delta[i] = b->delta[i];
    }
    return XY_OK;
}

// ------------------------------------------------------------- batched HMC
// Workspace of lattice i at offset off[i] (its HMC areas sized for its L), then
// the trajectory's records of all lattices (staging), then the batched stages'
// descriptors (room for every lattice) and their block offsets.
static size_t bhmc_layout(const xy_batch* b, std::vector<size_t>* off, size_t* staging, size_t* desc = nullptr,
                          size_t* start = nullptr)
{
    size_t t = 0;
    if (off) off->resize(b->n);
    for (int i = 0; i < b->n; ++i) {
        if (off) (*off)[i] = t;
        t += align256(xyk::hmc_work_bytes_compact(b->L[i]));
    }
    if (staging) *staging = t;
    t += align256((size_t)b->n * sizeof(xy_hmc_obs));
    if (desc) *desc = t;
    t += align256((size_t)b->n * sizeof(xyk::BhLat));
    if (start) *start = t;
    return t + align256(3 * ((size_t)b->n + 1) * sizeof(uint32_t));
}

int xy_batch_hmc_work_bytes(const xy_batch* b, size_t* bytes)
{
    if (!blive(b) || !bytes) return XY_ESTATE;
    *bytes = bhmc_layout(b, nullptr, nullptr);
    return XY_OK;
}

int xy_batch_hmc(xy_batch* b, int64_t n_traj, int32_t n_md, double eps, void* hmc_work, size_t hmc_len,
                 xy_hmc_obs* obs_dev)
{
    if (!blive(b)) return XY_ESTATE;
    if (b->precision != XY_FP32 || n_traj < 0 || n_md < 1 || !std::isfinite(eps) || !(eps > 0.0)) return XY_EINVAL;
    if (!hmc_work) return XY_ESTATE;
    std::vector<size_t> off;
    size_t staging = 0, desc_off = 0, start_off = 0;
    if (hmc_len < bhmc_layout(b, &off, &staging, &desc_off, &start_off)) return XY_ESIZE;
    if (b->sweep + (uint64_t)n_traj >= 0xffffffffull || n_traj > INT32_MAX) return XY_ERANGE;
    if (n_traj == 0) return XY_OK;
    hipError_t e;
    for (int k = 1; k < kHmcStreams; ++k) {
        if (!b->hs[k] && (e = hipStreamCreateWithFlags(&b->hs[k], hipStreamNonBlocking)) != hipSuccess) {
            b->hs[k] = nullptr;
            return xyr::hip_fail(e, "xy_batch_hmc: hipStreamCreate");
        }
        if (!b->hev[k] && (e = hipEventCreateWithFlags(&b->hev[k], hipEventDisableTiming)) != hipSuccess) {
            b->hev[k] = nullptr;
            return xyr::hip_fail(e, "xy_batch_hmc: hipEventCreate");
        }
    }
    Ctrl* ctrl = (Ctrl*)(b->work + b->lo.ctrl_off);
    char* hw = (char*)hmc_work;
    xy_hmc_obs* stage = (xy_hmc_obs*)(hw + staging);
    xyk::BhLat* d_desc = (xyk::BhLat*)(hw + desc_off);
    uint32_t* d_start = (uint32_t*)(hw + start_off);
    if (!b->hexec || b->h_nmd != n_md || b->h_eps != eps || b->h_steps != b->hmc_steps || b->h_work != hmc_work ||
        b->h_obs != obs_dev || b->h_ntraj != n_traj || b->h_pgen != b->pgen) {
        // one trajectory of every lattice, captured once and replayed per
        // trajectory; the kernels read the trajectory index from the batch's device
        // counter.  Lattices with L % 64 == 0 (with passes of several steps) go
        // through the batched stages, one launch per stage for all of them; the
        // others are spread over kHmcStreams branches (greedy by L^2) with their
        // own single-lattice launches.
        if ((e = hipStreamSynchronize(b->stream)) != hipSuccess)     // a copy may still read the host descriptors
            return xyr::hip_fail(e, "xy_batch_hmc: hipStreamSynchronize");
        drop_hmc_graph(b);
        std::vector<int> fast;
        if (b->hmc_steps > 1)
            for (int i = 0; i < b->n; ++i)
                if (xyk::hmc_batch_supported(b->L[i])) fast.push_back(i);
        const int nf = (int)fast.size();
        uint32_t totals[3] = {0, 0, 0};
        std::vector<char> isfast(b->n, 0);
        double load[kHmcStreams] = {0.0};
        const size_t eb = sizeof(float);
        if (nf > 0) {
            std::vector<xyk::BhLat>& hd = b->h_desc;
            std::vector<uint32_t>& hs = b->h_start;
            hd.assign(nf, xyk::BhLat{});
            hs.assign(3 * (size_t)(nf + 1), 0u);
            for (int f = 0; f < nf; ++f) {
                const int i = fast[f];
                isfast[i] = 1;
                const LatDesc& ld = b->desc[i];
                xyk::BhLat& q = hd[f];
                q.st = (float*)(b->state + (size_t)ld.off * eb);
                q.pp = (float*)(b->work + b->lo.pp_off + (size_t)ld.off * eb);
                q.w = xyk::hmc_carve_compact(hw + off[i], b->L[i]);
                q.obs = stage + i;
                q.k0 = ld.key0;
                q.k1 = ld.key1;
                xyk::hmc_batch_describe(q, b->L[i], b->beta[i], eps);
                uint32_t nb[3];
                xyk::hmc_batch_blocks(b->L[i], nb);
                for (int g = 0; g < 3; ++g) {
                    hs[(size_t)g * (nf + 1) + f] = totals[g];
                    if ((uint64_t)totals[g] + nb[g] > 0x7fffffffull) {
                        drop_hmc_graph(b);
                        return XY_ESIZE;
                    }
                    totals[g] += nb[g];
                }
                load[0] += (double)b->L[i] * b->L[i];
            }
            for (int g = 0; g < 3; ++g) hs[(size_t)g * (nf + 1) + nf] = totals[g];
        }
        if ((e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
            drop_hmc_graph(b);
            return xyr::hip_fail(e, "xy_batch_hmc: hipStreamBeginCapture");
        }
        hipError_t le = hipEventRecord(b->ev_fork, b->cap);
        for (int k = 1; k < kHmcStreams && le == hipSuccess; ++k) le = hipStreamWaitEvent(b->hs[k], b->ev_fork, 0);
        if (le == hipSuccess && nf > 0)
            le = xyk::launch_hmc_batch_trajectory(d_desc, d_start, nf, totals, eps, n_md, b->hmc_steps,
                                                  &ctrl->sweep0, b->cap);
        for (int i = 0; i < b->n && le == hipSuccess; ++i) {
            if (isfast[i]) continue;
            int k = 0;
            for (int q = 1; q < kHmcStreams; ++q)
                if (load[q] < load[k]) k = q;
            load[k] += (double)b->L[i] * b->L[i];
            hipStream_t sk = k == 0 ? b->cap : b->hs[k];
            const LatDesc& d = b->desc[i];
            float* st = (float*)(b->state + (size_t)d.off * eb);
            float* pp = (float*)(b->work + b->lo.pp_off + (size_t)d.off * eb);
            const xyk::HmcWork w = xyk::hmc_carve_compact(hw + off[i], b->L[i]);
            le = xyk::launch_hmc_trajectory(st, pp, w, b->L[i], b->beta[i], eps, n_md, b->hmc_steps, 0u, d.key0,
                                            d.key1, stage + i, sk, &ctrl->sweep0);
        }
        for (int k = 1; k < kHmcStreams && le == hipSuccess; ++k) {
            le = hipEventRecord(b->hev[k], b->hs[k]);
            if (le == hipSuccess) le = hipStreamWaitEvent(b->cap, b->hev[k], 0);
        }
        if (le == hipSuccess) {
            hipLaunchKernelGGL(k_bhmc_finish, dim3(1), dim3(kNT), 0, b->cap, (const xy_hmc_obs*)stage, obs_dev, b->n,
                               (int)n_traj, ctrl);
            le = hipGetLastError();
        }
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(b->cap, &g);
        if (le != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            drop_hmc_graph(b);
            return xyr::hip_fail(le, "xy_batch_hmc: launch (capture)");
        }
        if (e != hipSuccess) {
            drop_hmc_graph(b);
            return xyr::hip_fail(e, "xy_batch_hmc: hipStreamEndCapture");
        }
        b->hgraph = g;
        if ((e = hipGraphInstantiate(&b->hexec, g, nullptr, nullptr, 0)) != hipSuccess) {
            b->hexec = nullptr;
            drop_hmc_graph(b);
            return xyr::hip_fail(e, "xy_batch_hmc: hipGraphInstantiate");
        }
        b->h_nmd = n_md;
        b->h_eps = eps;
        b->h_steps = b->hmc_steps;
        b->h_work = hmc_work;
        b->h_obs = obs_dev;
        b->h_ntraj = n_traj;
        b->h_pgen = b->pgen;
    }
    // the batched stages' descriptors into the caller's workspace, on every call
    // (the workspace is the caller's between calls), ordered before the replays
    if (!b->h_desc.empty() &&
        ((e = hipMemcpyAsync(d_desc, b->h_desc.data(), b->h_desc.size() * sizeof(xyk::BhLat),
                             hipMemcpyHostToDevice, b->stream)) != hipSuccess ||
         (e = hipMemcpyAsync(d_start, b->h_start.data(), b->h_start.size() * sizeof(uint32_t),
                             hipMemcpyHostToDevice, b->stream)) != hipSuccess))
        return xyr::hip_fail(e, "xy_batch_hmc: descriptor copy");
    hipLaunchKernelGGL(k_bhmc_start, dim3(1), dim3(1), 0, b->stream, ctrl);
    if ((e = hipGetLastError()) != hipSuccess) return xyr::hip_fail(e, "xy_batch_hmc: launch");
    for (int64_t t = 0; t < n_traj; ++t) {
        if ((e = XY_LAUNCH(hipGraphLaunch(b->hexec, b->stream))) != hipSuccess)
            return xyr::hip_fail(e, "xy_batch_hmc: hipGraphLaunch");
        b->sweep += 1;
    }
    return XY_OK;
}

int xy_batch_hmc_set_steps_per_pass(xy_batch* b, int32_t steps)
{
    if (!blive(b)) return XY_ESTATE;
    if (steps < 1 || steps > 8) return XY_EINVAL;
    b->hmc_steps = steps;
    return XY_OK;
}

int xy_batch_set_spin_limit(xy_batch* b, uint32_t polls)
{
    if (!blive(b)) return XY_ESTATE;
    if (polls == 0) return XY_EINVAL;
    hipLaunchKernelGGL(k_set_spin_limit, dim3(1), dim3(1), 0, b->stream, (Ctrl*)(b->work + b->lo.ctrl_off), polls);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return xyr::hip_fail(e, "xy_batch_set_spin_limit");
    return XY_OK;
}

int xy_batch_status(xy_batch* b)
{
    if (!blive(b)) return XY_ESTATE;
    Ctrl c;
    hipError_t e = hipMemcpyAsync(&c, b->work + b->lo.ctrl_off, sizeof(Ctrl), hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return xyr::hip_fail(e, "xy_batch_status");
    return c.timed_out ? XY_EBARRIER : XY_OK;
}

int xy_batch_free(xy_batch* b)
{
    if (!blive(b)) return XY_ESTATE;
    release(b);
    return XY_OK;
}

}  // extern "C"
