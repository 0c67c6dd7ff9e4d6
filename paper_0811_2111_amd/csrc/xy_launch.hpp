// xy_launch.hpp -- host-side launchers of the HIP kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "xy.h"

namespace xyk {

struct SweepArgs {
    void* src;          // state read by the sweep
    void* dst;          // state written (== src for in-place schedules)
    int L;
    int precision;      // XY_FP32 / XY_FP16
    uint32_t key0, key1;
    uint32_t sweep;     // absolute index of the (first) sweep
    float delta, nbl2e;   // proposal width in turns (FP32), -beta log2(e)
};

// Workspace carve-up shared by the runtime and the launchers.
struct Work {
    void* pingpong;                 // second state buffer (fused schedule)
    unsigned long long* counter;    // accept counter (one u64)
    unsigned* arrive;               // arrival counter of the one-launch finalize (zeroed with counter)
    double* partials;               // per-workgroup measurement partials, 8 doubles each
    int max_partials;
    double* chunks;                 // second-level sums of 256 partials each
};

size_t state_bytes(int L, int precision);
size_t work_bytes(int L, int precision);
Work carve(void* work, int L, int precision);
int max_partials_for(int L);

hipError_t launch_init(void* st, int L, int precision, uint32_t k0, uint32_t k1, int hot, hipStream_t s);

// One half-sweep of `colour`, in place.  counter != NULL adds the accepts to it;
// dbg_acc / dbg_dE != NULL write per-site decisions and FP32 dE in the state layout.
hipError_t launch_half_sweep(const SweepArgs& a, int colour, unsigned long long* counter,
                             uint8_t* dbg_acc, float* dbg_dE, hipStream_t s);

// FP64 partial sums of the observables of state `st` into partials[0..*nparts).
hipError_t launch_measure(const void* st, int L, int precision, double* partials, int max_parts,
                          int* nparts, hipStream_t s);

// Reduce partials in a fixed order, take the accept counter (and clear it) plus
// the accepts in slot 6 of the partials, write one xy_obs record.
// Sums of 256 consecutive records (slots 0..6) into out[chunk * 8 ..], fixed order.
hipError_t launch_reduce_chunks(const double* partials, int nparts, double* out, hipStream_t s);

// partials -> one record.  More than 2048 partials take two levels through
// `scratch`: in one launch when `arrive` (a zeroed u32 in device memory, zero again
// afterwards) is given, else in two.
hipError_t launch_finalize(const double* partials, int nparts, unsigned long long* counter,
                           xy_obs* out, uint64_t sweep_after, hipStream_t s, double* scratch,
                           unsigned* arrive = nullptr);

// Fused tiled sweep(s): `m` sweeps (1 or 2) per launch from a.src to a.dst.
// meas_mask bit j set: measure after sub-sweep j into the 8-double record
// partials[(j * ntiles + tile) * 8] (slot 6 = the tile's accepts).
hipError_t launch_fused(const SweepArgs& a, int tile_x, int tile_y, int m, unsigned meas_mask,
                        double* partials, hipStream_t s);
int fused_tiles(int L, int tile_x, int tile_y);
// Partial records one measured sweep of a fused launch writes (the sweep's
// records start at partials + j * fused_records(...) * 8 for sub-sweep j).
int fused_records(int L, int tile_x, int tile_y, int m);

// Strip sweep (xy_strip.hip): one sweep from a.src to a.dst by segments of
// tile_x columns x tile_y rows; measured: one record per wave (4 per segment) at
// partials[(segment * 4 + wave) * 8].
bool strip_supported(int L, int tile_x, int tile_y);
// Whole lattice resident in one workgroup's LDS (L <= 128, L % 4 == 0): n sweeps
// in place from a.src (= a.dst), records of every me-th sweep of the call to
// obs[0 ..] (none if me == 0 or obs == NULL).
bool resident_supported(int L);
hipError_t launch_resident(const SweepArgs& a, int n, int me, xy_obs* obs, hipStream_t s);
hipError_t launch_strip(const SweepArgs& a, int tile_x, int tile_y, bool meas, double* partials, hipStream_t s);
int strip_records(int L, int tile_x, int tile_y);

// ---- hybrid Monte Carlo (xy_hmc.hip)
constexpr int kHmcMaxRecords = 65536;   // partial records of one H sum (old or new)
constexpr int kHmcMaxChunks = kHmcMaxRecords / 256;
struct HmcWork {
    unsigned* flag;     // accept flag of the last trajectory
    float* p;           // momenta, state layout
    float* saved;       // angles at the start of the trajectory
    float* p2;          // second momentum buffer (passes of several steps)
    double* rec_old;    // partial records of H_old (8 doubles each)
    double* rec_new;    // partial records of H_new
    double* chunk_old;  // sums of 256 records each
    double* chunk_new;
};
size_t hmc_work_bytes(int L);
HmcWork hmc_carve(void* work, int L);
int hmc_records(int L);
// One trajectory from the FP32 angles in `state` (result back in `state`),
// `pingpong` a second state-sized buffer; record to obs if not NULL.
// steps_per_pass > 1 (and L % 32 == 0): leap-frog steps in passes of up to
// min(steps_per_pass, 8) steps (temporal blocking); else one step per launch.
// traj_dev != NULL: the trajectory index is read from device memory when the
// kernels run (graph replays), instead of `traj`.
hipError_t launch_hmc_trajectory(float* state, float* pingpong, const HmcWork& w, int L, double beta, double eps,
                                 int n_md, int steps_per_pass, uint32_t traj, uint32_t k0, uint32_t k1,
                                 xy_hmc_obs* obs, hipStream_t s, const uint32_t* traj_dev = nullptr);
// Workspace of one lattice with record arrays sized for its L only (batches).
size_t hmc_work_bytes_compact(int L);
HmcWork hmc_carve_compact(void* work, int L);
bool hmc_multi_supported(int L);

// One trajectory of many lattices, one launch per stage over all of them
// (batches).  Lattice i's numbers and arithmetic are those of
// launch_hmc_trajectory on it alone with the same steps per pass (> 1), so each
// lattice is bit for bit the single-lattice trajectory.
struct BhLat {
    float* st;          // the lattice's angles
    float* pp;          // its second angle buffer
    HmcWork w;          // its HMC areas (hmc_carve_compact)
    xy_hmc_obs* obs;    // where its trajectory record goes (may be NULL)
    double beta;
    int L, cols, rb, nrec;        // rb: row runs of the pair kernels (hmc_runs2)
    uint32_t k0, k1;
    float kick_half, kick_full;   // -beta eps / 2, -beta eps (FP32, as launch_hmc_trajectory forms them)
};
// Lattices this path takes: L % 64 == 0 (64 x 64 leap-frog tiles, pair ends).
bool hmc_batch_supported(int L);
// Fill the geometry fields of d (cols, rb, nrec, kicks) for lattice L at beta, eps.
void hmc_batch_describe(BhLat& d, int L, double beta, double eps);
// Workgroups lattice L takes in each stage grid: [0] ends, [1] leap-frog pass,
// [2] restore (each a multiple of 8, so that every lattice starts on XCD 0).
void hmc_batch_blocks(int L, uint32_t nb[3]);
// d: n descriptors in device memory; start: 3 (n + 1) block offsets in device
// memory (stage s, lattice i at start[s (n + 1) + i], each stage's total last),
// totals the three grid sizes; traj_dev: the trajectory index in device memory.
hipError_t launch_hmc_batch_trajectory(const BhLat* d, const uint32_t* start, int n, const uint32_t totals[3],
                                       double eps, int n_md, int steps_per_pass, const uint32_t* traj_dev,
                                       hipStream_t s);
bool fused_supported(int L, int tile_x, int tile_y, int m);

// ---- hybrid Monte Carlo on the four-replica texel (xy_quad_hmc.hip)
struct QHmcKeys {
    uint32_t k0[4], k1[4];        // Philox keys of the four replicas
};
struct QHmcBeta {
    double b[4];
};
struct QuadHmcWork {
    float4* p;          // momenta, one float4 per entry
    float4* saved;      // angles at the start of the trajectory
    float4* p2;         // second momentum buffer (passes of several steps)
    unsigned* flag;     // the four accept decisions of the last trajectory
    double* rec_old;    // partial records of H_old: replica r's at rec_old + r * records * 8
    double* rec_new;
    double* chunk_old;  // sums of 256 records each, per replica
    double* chunk_new;
};
int quad_hmc_records(int L);          // partial records per replica and H sum
size_t quad_hmc_work_bytes(int L);
QuadHmcWork quad_hmc_carve(void* work, int L);
// One trajectory of all four replicas of the float4 state (result back in
// `state`, `pingpong` a second state-sized buffer); obs: NULL or 4 records.
// steps_per_pass > 1: leap-frog steps in passes of up to min(steps_per_pass, 4)
// (L % 32 == 0, as every quad); 1: one step per launch.  Same trajectory.
hipError_t launch_quad_hmc_trajectory(float4* state, float4* pingpong, const QuadHmcWork& w, int L,
                                      const double beta[4], double eps, int n_md, int steps_per_pass, uint32_t traj,
                                      const QHmcKeys& keys, xy_hmc_obs* obs, hipStream_t s);

// Fill n u64 words with zero (kernel, not a memset node: safe inside graphs).
hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t s);

}  // namespace xyk
