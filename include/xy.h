/*
 * xy.h -- C ABI of the MI355X (gfx950) checkerboard Metropolis library for the
 * 2-d XY model.
 *
 * Model (section 1.2, eq. 1 of Anselmi, Conti, Di Renzo, "GPU computing for 2-d
 * spin systems: CUDA vs OpenGL", Lattice 2008): H = -J sum_<ij> cos(theta_i -
 * theta_j) over nearest-neighbour pairs of a periodic L x L square lattice, each
 * pair counted once, J = 1, Boltzmann weight exp(-beta H).  The paper samples it
 * with hybrid Monte Carlo; this library runs the same ensemble with
 * checkerboard single-site Metropolis:
 *
 *   one sweep = every red site ((x+y) even), then every black site; a site
 *   proposes theta' = theta + delta (2 u1 - 1), taken modulo 2 pi, and
 *   accepts iff u2 < exp(-beta dE), dE = -J sum_nn [cos(theta' - theta_j) -
 *   cos(theta - theta_j)].
 *
 * Angle unit: the state holds phi = theta / (2 pi) in turns, the argument the
 * hardware sine and cosine take.  delta is passed in radians and used as
 * Delta = fl32(delta / (2 pi)) turns.
 *
 * Random numbers: Philox4x32-10 (Salmon et al., SC'11), key = (seed mod 2^32,
 * seed >> 32), one call per two same-colour sites of a half-row: counter =
 * (sweep, colour, purpose, y * P + (k >> 1)) with k the half-row index and
 * P = ceil(L/4); words (X0, X1) for even k and (X2, X3) for odd k; u = (2 (w >> 9)
 * + 1) 2^-24.  Purpose 0 drives the updates, purpose 1 (sweep 0) the hot start
 * phi = u (theta = 2 pi u).  The stream depends on (seed, site, sweep) only, so every
 * schedule, tile shape and batch composition gives the same trajectory bit for
 * bit, and a run can be resumed from a saved state and sweep counter.
 *
 * FP32 proposal arithmetic, rounded exactly as written: step = fl(Delta * r),
 * t = fl(phi + step), phi' = fl(t - floor(t)), and phi' = 1 - 2^-24 where that
 * rounds to 1 (t a tiny negative number), so FP32 angles stay in [0, 1).  FP16
 * storage (XY_FP16) rounds phi' to IEEE binary16 (nearest-even; this may give
 * 1.0) before dE is evaluated.
 * Energies and decisions are FP32 on the device; observables are accumulated
 * in FP64 (the paper's "global sums of the energy", section 1.2).
 *
 * State layout (device memory, owned by the caller): two half-lattices,
 * colour c = 0 (red) then c = 1 (black), each L rows of L/2 entries, row-major:
 *     elem(c, y, k) = state[(c * L + y) * (L/2) + k],  x = 2k + ((c + y) & 1),
 * stored as float (XY_FP32) or IEEE binary16 (XY_FP16), turns in [0, 1] (FP32: [0, 1)).
 *
 * Conventions for every function:
 *   - returns XY_OK (0) or a negative error code; nothing throws or aborts;
 *   - a handle stays valid after any error;
 *   - all device memory (state, workspace, observables, debug buffers) belongs
 *     to the caller and must outlive the handle; the library never allocates
 *     device memory; host objects (handles, graphs) are freed by *_free;
 *   - work is enqueued on the caller's HIP stream and the call returns; launch
 *     and configuration errors are returned at once, asynchronous kernel faults
 *     surface at the caller's next synchronisation;
 *   - a handle is not thread-safe; distinct handles are independent.
 */
#ifndef XY_H
#define XY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- codes */
#define XY_OK      0
#define XY_EINVAL (-1)  /* L odd or < 4, L*L >= 2^31, beta not finite or < 0, delta not in (0, pi],
                           bad precision / start / plan / measure_every, n_sweeps < 0 */
#define XY_ESIZE  (-2)  /* a buffer is shorter than xy_state_bytes / xy_batch_state_bytes asks */
#define XY_ERANGE (-3)  /* sweep counter would pass 2^32 - 1 */
#define XY_EHIP   (-4)  /* a HIP runtime call failed; xy_last_hip_error() names it */
#define XY_ESTATE (-5)  /* NULL handle, NULL required pointer, or handle already freed */
#define XY_ENOMEM (-6)  /* host allocation of a handle failed */
#define XY_EBARRIER (-7) /* a batch barrier wait hit its spin limit (the GPU did not hold every
                            workgroup of the persistent launch at once), or an XCD with lattices
                            to sweep ran none of its workgroups; results are invalid */
#define XY_EIO    (-8)  /* a file (the tune cache) could not be written */

enum { XY_FP32 = 0, XY_FP16 = 1 };
enum { XY_HOT = 0, XY_COLD = 1 };

/* One measured configuration: raw FP64 sums over the lattice (64 bytes).
 *   cx = sum cos(theta(x,y) - theta(x+1,y)),  cy = sum cos(theta(x,y) - theta(x,y+1)),
 *   ix = sum sin(theta(x,y) - theta(x+1,y)),  iy = sum sin(theta(x,y) - theta(x,y+1)),
 *   mx = sum cos theta,  my = sum sin theta,
 *   sweep = sweep counter after the measured sweep, n_accept = accepted proposals in it
 *   (0 for xy_measure).  Derived: E = -(cx + cy), |m| = hypot(mx, my) / N, helicity
 *   modulus = (<cx + cy> - beta <ix^2 + iy^2>) / (2N). */
typedef struct xy_obs {
    uint64_t sweep;
    uint64_t n_accept;
    double cx, cy, ix, iy, mx, my;
} xy_obs;

/* Execution schedule of a sweep.  The trajectory does not depend on it.
 *   XY_PLAN_STREAM: two in-place half-sweep launches per sweep (any even L >= 4).
 *   XY_PLAN_FUSED : one launch per `sweeps_per_pass` sweeps; a workgroup loads a
 *                   tile_x x tile_y tile plus a halo of 2*sweeps_per_pass sites into
 *                   LDS, runs the red and black half-sweeps there (recomputing the
 *                   halo's red sites with their owners' random numbers) and writes
 *                   the tile to the other buffer of a ping-pong pair.  Needs
 *                   L % 4 == 0, tile_x % 4 == 0, tile_x | L, tile_y | L.
 *   XY_PLAN_STRIP : one launch per sweep; a workgroup walks down a segment of
 *                   tile_x columns (128, 256 or 512) and tile_y rows, a few rows
 *                   of each colour at a time, with (cos, sin) of the rows in
 *                   flight in LDS rings and the next rows' loads issued ahead;
 *                   the halo is one red row above and below the segment plus one
 *                   red entry per row beside it, recomputed.  Made for lattices
 *                   far beyond the caches: its row loads and stores carry the
 *                   non-temporal hint.  Needs tile_x | L, tile_y | L, (tile_x,
 *                   tile_y) one of (128, 32|64|128), (256, 32|64|128|256),
 *                   (512, 64|128|256), sweeps_per_pass = 1.
 *   XY_PLAN_RESIDENT: every sweep of a call in one launch of one workgroup that
 *                   holds the whole lattice in LDS (angles of both colours and the
 *                   (cos, sin) of one colour, 8 L^2 bytes): no halo and no HBM
 *                   traffic between sweeps.  Needs L <= 128, L % 4 == 0; tile_x,
 *                   tile_y ignored, sweeps_per_pass = 1.
 *   XY_PLAN_AUTO  : the tuned plan for (L, precision) if one is cached, else a
 *                   default: strip 512 x 64 for a lattice whose state and
 *                   ping-pong copy exceed 256 MiB, else the first fused tile of
 *                   256 x 16, 128 x 32, 64 x 32, 64 x 16 that L allows, else
 *                   XY_PLAN_STREAM. */
enum { XY_PLAN_AUTO = 0, XY_PLAN_STREAM = 1, XY_PLAN_FUSED = 2, XY_PLAN_STRIP = 3, XY_PLAN_RESIDENT = 4 };
typedef struct xy_plan {
    int32_t kind;
    int32_t tile_x;
    int32_t tile_y;
    int32_t sweeps_per_pass;   /* 1 or 2 */
} xy_plan;

typedef struct xy_lattice xy_lattice;
typedef struct xy_batch xy_batch;

/* Bytes of device memory a lattice needs: *state for the angles (layout above),
 * *workspace for the ping-pong copy and the reduction partials.  Either output
 * pointer may be NULL.  The lattice lives in device memory and is staged through
 * on-chip memory tile by tile (section 2.2).
 * XY_EINVAL: L odd, L < 4, L^2 >= 2^31, or a bad precision. */
int xy_state_bytes(int32_t L, int32_t precision, size_t* state, size_t* workspace);

/* Create a lattice of the model of section 1.2, eq. 1 on the caller's stream
 * (hipStream_t passed as void*, NULL = the null stream) and initialise the
 * angles: XY_HOT draws phi = u from the purpose-1 stream (exact in FP32; FP16
 * storage rounds it once), XY_COLD sets phi = 0.  The sweep counter starts at 0.
 * beta >= 0 finite (the weight exp(-beta H)); 0 < delta <= pi.
 * state_dev: xy_state_bytes' *state bytes, layout above; work_dev: its
 * *workspace bytes, contents owned by the library while the handle lives.
 * Both are caller-owned device memory and must outlive the handle.
 * XY_EINVAL: bad L, beta, delta, start or precision; XY_ESTATE: out, state_dev
 * or work_dev NULL; XY_ESIZE: a buffer too short; XY_EHIP: the initialising
 * launch failed (no handle is returned). */
int xy_init(xy_lattice** out, uint64_t seed, int32_t L, double beta, double delta,
            int32_t start, int32_t precision,
            void* state_dev, size_t state_len, void* work_dev, size_t work_len,
            void* hip_stream);

/* Same as xy_init (section 1.2, eq. 1) but keeps the angles already in
 * state_dev (a checkpoint) and sets the sweep counter to `sweep`.  Because the
 * random numbers depend only on (seed, sweep, site), the continued trajectory
 * is bit for bit the uninterrupted one.  XY_ERANGE: sweep >= 2^32 - 1; other
 * codes as xy_init. */
int xy_attach(xy_lattice** out, uint64_t seed, int32_t L, double beta, double delta,
              int32_t precision, uint64_t sweep,
              void* state_dev, size_t state_len, void* work_dev, size_t work_len,
              void* hip_stream);

/* Run n_sweeps Metropolis sweeps of the ensemble exp(-beta H), H of section
 * 1.2, eq. 1 (red sites, then black sites, the update in the preamble) from the
 * handle's sweep counter.  If measure_every > 0 and obs_dev != NULL, after every
 * sweep j (1-based within this call) with j % measure_every == 0 one xy_obs with
 * the FP64 global sums of section 1.2 is written to
 * obs_dev[j / measure_every - 1] (caller-owned device memory of
 * floor(n_sweeps / measure_every) * 64 bytes; the library does not know its
 * length).  On return (asynchronously, on the handle's stream) the angles are
 * in state_dev.  XY_EINVAL: n_sweeps < 0 or measure_every < 0; XY_ERANGE: the
 * counter would pass 2^32 - 1 (nothing is run); XY_EHIP: a launch failed (the
 * counter then stands after the last sweep enqueued). */
int xy_sweep(xy_lattice* h, int64_t n_sweeps, int32_t measure_every, xy_obs* obs_dev);

/* Measure the current state into obs_dev[0] (caller-owned device memory, 64
 * bytes): the global sums of the energy (section 1.2, in FP64 as the paper
 * keeps them), the bond sines of the helicity modulus and the magnetisation;
 * n_accept = 0.  XY_ESTATE: obs_dev NULL; XY_EHIP: a launch failed. */
int xy_measure(xy_lattice* h, xy_obs* obs_dev);

/* Handle accessors.  xy_set_params: the (beta, delta) of the update of section
 * 1.2 for later sweeps (XY_EINVAL as xy_init).  xy_get_sweep / xy_set_sweep: the
 * sweep counter that keys the random numbers (XY_ERANGE for >= 2^32 - 1).
 * xy_set_stream: later work goes to this stream.  xy_set_plan / xy_get_plan: the
 * schedule (XY_EINVAL if the plan does not fit L).  xy_free: releases the host
 * handle (never the caller's device memory).  XY_ESTATE for a NULL or freed
 * handle or a NULL output pointer. */
int xy_set_params(xy_lattice* h, double beta, double delta);
int xy_get_sweep(const xy_lattice* h, uint64_t* sweep);
int xy_set_sweep(xy_lattice* h, uint64_t sweep);
int xy_set_stream(xy_lattice* h, void* hip_stream);
int xy_set_plan(xy_lattice* h, const xy_plan* plan);
int xy_get_plan(const xy_lattice* h, xy_plan* plan);
int xy_free(xy_lattice* h);

/* Parallel tempering over a batch: the replicas at different temperatures of
 * section 3.2, which the paper keeps side by side, exchange temperatures
 * (standard parallel tempering; the paper gives no exchange rule).  Lattices of
 * equal L form a ladder (ladders in
 * order of L), its rungs ordered by the beta each lattice holds when the call
 * starts (ties by index); rung t keeps that (beta_t, delta_t).  Each of n_rounds
 * rounds runs sweeps_per_round sweeps of every lattice (the last one measured),
 * then the lattices a, b on rungs t, t+1 of every ladder, for t = p, p + 2, ...
 * (p = round index mod 2), exchange rungs iff u < exp((beta_t - beta_t+1)
 * (E_a - E_b)), E = -(cx + cy) of the round's record and u = u(X0) of Philox
 * counter (round, ladder, 4, t), key = (pt_seed mod 2^32, pt_seed >> 32).
 * Configurations stay in place; temperatures move.  Round indices continue
 * across calls on a batch.  obs_dev: NULL or device memory for n_rounds * n
 * records, [round][lattice]; rung_dev: NULL or n_rounds * n int32, the rung each
 * lattice held during the round.  Returns after the work has finished (the
 * lattices' new (beta, delta) are read back; see xy_batch_get_params).
 * XY_EINVAL: n_rounds < 0 or sweeps_per_round < 1; XY_ERANGE: the sweep or round
 * counter would pass 2^32 - 1. */
int xy_batch_tempering(xy_batch* b, int64_t n_rounds, int32_t sweeps_per_round, uint64_t pt_seed,
                       xy_obs* obs_dev, int32_t* rung_dev);

/* The (beta, delta) each lattice of the batch currently runs at after the
 * exchanges of section 3.2's replicas (host arrays of n; either may be NULL). */
int xy_batch_get_params(const xy_batch* b, double* beta, double* delta);

/* ------------------------------------------------ four-replica lattices
 * Four replicas of one L x L lattice (own seed, beta and delta each, e.g. four
 * temperatures) in one state array, the four-channel texel of section 3.2:
 * entry (c, y, k) of the layout above is four floats, component r holding
 * replica r's angle (turns), 16 bytes per entry.  Replica r draws exactly the
 * random numbers a single lattice with seed_r draws, so its trajectory is bit
 * for bit that of xy_init/xy_sweep with (seed_r, L, beta_r, delta_r) in FP32;
 * a sweep updates all four with one pass over the state.  FP32 only;
 * L % 32 == 0, 32 <= L and 16 L^2 < 2^32. */
typedef struct xy_quad xy_quad;

/* *state = 16 L^2 bytes; *workspace = the second state buffer plus partial sums
 * (16 L^2 + 2 L^2 + small). */
int xy_quad_state_bytes(int32_t L, size_t* state, size_t* workspace);

/* seeds, beta, delta: host arrays of 4.  start: XY_HOT (replica r: the hot start
 * of seed_r) or XY_COLD.  Counter starts at 0. */
int xy_quad_init(xy_quad** out, const uint64_t* seeds, int32_t L, const double* beta, const double* delta,
                 int32_t start, void* state_dev, size_t state_len, void* work_dev, size_t work_len,
                 void* hip_stream);

/* As xy_sweep; records go to obs_dev[(j / measure_every - 1) * 4 + r] for
 * replica r (4 xy_obs per measured sweep). */
int xy_quad_sweep(xy_quad* q, int64_t n_sweeps, int32_t measure_every, xy_obs* obs_dev);
int xy_quad_set_params(xy_quad* q, const double* beta, const double* delta);
int xy_quad_get_sweep(const xy_quad* q, uint64_t* sweep);
int xy_quad_set_sweep(xy_quad* q, uint64_t sweep);
/* Tile shape of the fused sweep: (32, 16), (64, 8), (64, 16), (128, 4), (128, 8),
 * dividing L (default (128, 8), or (32, 16) if 128 does not divide L).  The
 * trajectory does not depend on it. */
int xy_quad_set_tile(xy_quad* q, int32_t tile_x, int32_t tile_y);
int xy_quad_get_tile(const xy_quad* q, int32_t* tile_x, int32_t* tile_y);
int xy_quad_free(xy_quad* q);

/* ------------------------------------------------------ hybrid Monte Carlo
 * The paper's own update (section 1.2): Gaussian momenta converted from flat
 * random numbers, leap-frog integration of the equations of motion, and a
 * Metropolis step on global sums of the energy kept in double precision.
 *
 *   H = sum_i p_i^2 / 2 + beta E,  E = -sum_<ij> cos(theta_i - theta_j);
 *   force F_i = -beta sum_{j nn i} sin(theta_i - theta_j);
 *   trajectory: p_i = sqrt(-2 ln u1) cos(2 pi u2) with (u1, u2) the site's two
 *   uniforms of Philox purpose 2 (counter word 0 = the trajectory index, same
 *   site pairing as the Metropolis update); n_md leap-frog steps of size eps
 *   (p += eps/2 F, theta += eps p, p += eps/2 F; adjacent half kicks merged);
 *   dH = H_new - H_old from FP64 sums of FP32 per-site terms; accept iff
 *   u < exp(-dH), u = u(X0) of Philox counter (traj, 0, 3, 0); a rejected
 *   trajectory leaves the angles as they were.
 *
 * Trajectories and Metropolis sweeps share the handle's counter: trajectory t
 * uses counter word 0 = t and advances the counter by one.  FP32 lattices only.
 *
 * One record per trajectory, 72 bytes: */
typedef struct xy_hmc_obs {
    uint64_t traj;       /* counter after the trajectory */
    uint64_t accepted;   /* 1 if accepted */
    double dH;           /* H_new - H_old */
    double cx, cy, ix, iy, mx, my;   /* sums as in xy_obs, of the state after the Metropolis step */
} xy_hmc_obs;

/* Bytes of device workspace xy_hmc needs for an L x L lattice (two momentum
 * buffers, saved angles, partial sums, accept flag):
 * 12 L^2 + 256 + 2 * (65536 + 256) * 64. */
int xy_hmc_work_bytes(int32_t L, size_t* bytes);

/* Run n_traj trajectories of n_md leap-frog steps of size eps (> 0, finite) on
 * the lattice's angles, on its stream; the lattice workspace's ping-pong buffer
 * holds the second copy of the angles during a trajectory.  hmc_work: device
 * memory of at least xy_hmc_work_bytes (caller-owned, contents overwritten).
 * obs_dev: NULL, or device memory for n_traj records (record j after trajectory
 * j of the call).  XY_EINVAL for an FP16 lattice, n_traj < 0, n_md < 1 or a bad
 * eps; XY_ESIZE if hmc_len is too small; XY_ERANGE if the counter would pass
 * 2^32 - 1. */
int xy_hmc(xy_lattice* h, int64_t n_traj, int32_t n_md, double eps, void* hmc_work, size_t hmc_len,
           xy_hmc_obs* obs_dev);

/* Leap-frog steps per pass over the lattice (1 .. 8, default 7; XY_EINVAL
 * otherwise).  With more than one, for L % 32 == 0, a workgroup loads a 64 x 64
 * tile (32 x 32 if L % 64 != 0) grown by that many sites on every side, runs the
 * steps on it (the grown part shrinking by one site per step) and writes the
 * tile back, so HBM traffic per site and step falls by that factor; the
 * trajectory is bit for bit the same.  xy_hmc_get_steps_per_pass reports what
 * runs (1 if L % 32 != 0). */
int xy_hmc_set_steps_per_pass(xy_lattice* h, int32_t steps);
int xy_hmc_get_steps_per_pass(const xy_lattice* h, int32_t* steps);

/* Hybrid Monte Carlo on the four-replica texel (sections 1.2 and 3.2): the four
 * replicas of a quad run their trajectories together (each pass over the
 * float4 state advances all four by the same leap-frog steps; see
 * xy_quad_hmc_set_steps_per_pass), and the Metropolis step is a vector of four
 * decisions z_r, each from the replica's own FP64 dH; replica r keeps
 * z_r theta_new + (1 - z_r) theta_old.  Replica r follows bit for bit the
 * trajectory that xy_hmc gives a single lattice with (seed_r, L, beta_r) and the
 * same n_md and eps; its dH agrees to the rounding of FP64 sums taken in another
 * order (a decision could differ only where u and exp(-dH) agree to that
 * rounding).  Trajectories and xy_quad_sweep share the quad's counter, as for a
 * lattice.  hmc_work: caller-owned device memory of at least
 * xy_quad_hmc_work_bytes (two momentum buffers and the saved angles, 48 L^2
 * bytes, plus partial sums).  obs_dev: NULL, or device memory for 4 n_traj
 * records, replica r's record of trajectory j at obs_dev[j * 4 + r].  Errors as
 * xy_hmc. */
int xy_quad_hmc_work_bytes(int32_t L, size_t* bytes);
int xy_quad_hmc(xy_quad* q, int64_t n_traj, int32_t n_md, double eps, void* hmc_work, size_t hmc_len,
                xy_hmc_obs* obs_dev);
/* Leap-frog steps per pass of xy_quad_hmc (1 .. 4, default 4; XY_EINVAL
 * otherwise): with more than one, a workgroup loads a 32 x 32 tile grown by that
 * many sites on every side, runs the steps on it and writes the tile back, as
 * xy_hmc_set_steps_per_pass does for a lattice; 1: one step per pass over the
 * state.  The trajectory is bit for bit the same. */
int xy_quad_hmc_set_steps_per_pass(xy_quad* q, int32_t steps);
int xy_quad_hmc_get_steps_per_pass(const xy_quad* q, int32_t* steps);

/* Batched hybrid Monte Carlo: n_traj trajectories of every lattice of an FP32
 * batch, the paper's update (section 1.2; see xy_hmc) applied to the replicas at
 * several temperatures of section 3.2 with one Metropolis accept per replica
 * (the per-replica acceptance vector of section 3.2), decided on the device from
 * that lattice's own FP64 dH.  Lattice i runs at its current beta with its own
 * seed; trajectory t of the call uses counter word 0 = the batch's sweep counter,
 * which advances by one per trajectory (shared with sweeps, as for a single
 * lattice), so every lattice follows bit for bit the trajectory that xy_hmc
 * gives a single lattice with the same seed, beta, counter, n_md, eps and leap-
 * frog steps per pass.  One trajectory of all lattices is captured once into a
 * HIP graph and replayed: with passes of several leap-frog steps, the lattices
 * with L % 64 == 0 share one launch per stage of the trajectory (ends, passes,
 * decide, restore); the others run their own launches, spread over four
 * concurrent branches.  The graph is rebuilt when n_traj, n_md, eps, the steps
 * per pass, the workspace or obs_dev change, and after xy_batch_tempering has
 * moved betas between lattices.
 * hmc_work: caller-owned device memory of xy_batch_hmc_work_bytes bytes (per
 * lattice: momenta, second momenta, saved angles, partial records; then one
 * staging record per lattice and the batched stages' descriptors, which every
 * call writes on the stream before its trajectories); the batch workspace's
 * ping-pong area holds the second copy of the angles.  The library allocates no
 * device memory here either.  obs_dev: NULL, or device memory for n * n_traj
 * records, lattice-major (trajectory r of lattice i at obs_dev[i * n_traj + r]).
 * XY_EINVAL: FP16 batch, n_traj < 0, n_md < 1 or a bad eps; XY_ESIZE: hmc_len too
 * small; XY_ERANGE: the counter would pass 2^32 - 1. */
int xy_batch_hmc_work_bytes(const xy_batch* b, size_t* bytes);
int xy_batch_hmc(xy_batch* b, int64_t n_traj, int32_t n_md, double eps, void* hmc_work, size_t hmc_len,
                 xy_hmc_obs* obs_dev);
/* Leap-frog steps per pass of xy_batch_hmc (1 .. 8, default 7), as
 * xy_hmc_set_steps_per_pass.  XY_EINVAL otherwise. */
int xy_batch_hmc_set_steps_per_pass(xy_batch* b, int32_t steps);

/* Profiling support: time the tiled sweep kernel launches (XY_PLAN_FUSED and
 * XY_PLAN_STRIP; one launch per pass) of the handle's next calls with HIP events
 * recorded on its stream right before and after each launch, for up to
 * `capacity` launches (0 turns the timer off and frees its events; host objects
 * only).  xy_kernel_timer_read waits for the last timed launch, returns the sum
 * of their durations in ms and their number, and restarts the count.  The
 * events order each timed launch after the work before it, so timed calls lose
 * the little overlap between consecutive launches.  XY_EINVAL: capacity < 0. */
int xy_kernel_timer(xy_lattice* h, int32_t capacity);
int xy_kernel_timer_read(xy_lattice* h, double* total_ms, int64_t* launches);

/* Test support: run ONE sweep (section 1.2, eq. 1; the update in the preamble)
 * with the streaming schedule and write, per site in the state layout (red half
 * then black half), accept_dev[i] = 1/0 and dE_dev[i] = the FP32 energy change of
 * the proposal (caller-owned device buffers of L^2 entries).  Either output may
 * be NULL.  XY_ERANGE: the counter would pass 2^32 - 1. */
int xy_debug_sweep(xy_lattice* h, uint8_t* accept_dev, float* dE_dev);

/* Time each candidate plan for `sweeps_per_trial` sweeps (after one untimed
 * trial) on the handle's stream, in two rounds over the candidates, and select
 * the one with the fastest trial; *best receives it and
 * the handle keeps it.  The plans differ in how sublattices are staged through
 * on-chip memory with duplicated borders (section 2.2), never in the trajectory.
 * The trials advance the handle's state and counter: run it on a scratch
 * lattice.  If cache_path != NULL the result is merged into that JSON file under
 * the key "gfx950/L/precision".  XY_EINVAL: sweeps_per_trial < 2; XY_EIO: the
 * cache file could not be written (the handle still keeps the best plan). */
int xy_autotune(xy_lattice* h, int32_t sweeps_per_trial, const char* cache_path, xy_plan* best);

/* Look up a tuned plan for (L, precision) in the JSON cache file written by
 * xy_autotune; XY_EINVAL if the file or the entry is missing. */
int xy_tuned_plan(const char* cache_path, int32_t L, int32_t precision, xy_plan* plan);

/* ----------------------------------------------------------------- batches
 * Many lattices in one device launch, so that the device is "sufficiently
 * filled" (section 3.2, where four replicas at different temperatures share one
 * texture and the best performance came from the largest workload).
 * n lattices of sizes L[i] >= 4, L[i] % 4 == 0 (possibly different), with their own seed,
 * beta and delta, advanced together; the launches of one call are captured once
 * into a HIP graph and replayed.  Lattice i's angles start at element offset
 * sum_{j<i} L[j]^2 of state_dev, in the single-lattice layout.  A lattice
 * follows exactly the trajectory it would follow alone with the same seed.
 * Three schedules (xy_batch_set_schedule), the same trajectory:
 *   XY_BATCH_PERSISTENT: one persistent kernel per call; the lattices are split
 *     into eight groups of about equal area, one per XCD; the workgroups running
 *     on an XCD split its group's tiles into contiguous ranges, and each waits,
 *     before a pass over its range of a lattice, for the previous pass of the
 *     tiles around that range (a passes-done counter per tile in device memory,
 *     synchronised within the XCD only); 256 x 16 tiles for every lattice whose
 *     L is a multiple of 256;
 *   XY_BATCH_PASSES: one launch per sweep over all tiles of all lattices, one
 *     workgroup per tile; the kernel boundary orders the sweeps;
 *   XY_BATCH_PASSES_WIDE (default): the same, with 256 x 16 tiles for every
 *     lattice whose L is a multiple of 256 (the batch's shape for the others). */
enum { XY_BATCH_PERSISTENT = 0, XY_BATCH_PASSES = 1, XY_BATCH_PASSES_WIDE = 2 };
/* Device bytes of a batch (section 3.2's replicas, here of any sizes): *state =
 * sum of the lattices' state bytes (lattices back to back), *workspace = the
 * ping-pong copy, barrier counters, descriptors and partial sums.
 * XY_EINVAL: n < 1, a bad L[i] or precision; XY_ESTATE: L NULL. */
int xy_batch_state_bytes(int32_t n, const int32_t* L, int32_t precision,
                         size_t* state, size_t* workspace);
/* Create a batch of n lattices of section 1.2's model (seeds, L, beta, delta:
 * host arrays of n; the replicas at several temperatures of section 3.2) on the
 * caller's stream and initialise every lattice as xy_init does.  Buffers are
 * caller-owned device memory that must outlive the handle.  Error codes as
 * xy_init, for any lattice. */
int xy_batch_init(xy_batch** out, int32_t n, const uint64_t* seeds, const int32_t* L,
                  const double* beta, const double* delta, int32_t start, int32_t precision,
                  void* state_dev, size_t state_len, void* work_dev, size_t work_len,
                  void* hip_stream);
/* Run n_sweeps sweeps (section 1.2, eq. 1; the update in the preamble) of every
 * lattice of the batch.  obs_dev: NULL, or caller-owned device memory for
 * n * floor(n_sweeps / measure_every) records (FP64 global sums of section
 * 1.2), lattice-major (record r of lattice i at obs_dev[i * n_rec + r]).
 * XY_EINVAL: n_sweeps < 0 or measure_every < 0; XY_ERANGE: the counter would
 * pass 2^32 - 1; XY_EHIP: a launch or the graph failed. */
int xy_batch_sweep(xy_batch* b, int64_t n_sweeps, int32_t measure_every, xy_obs* obs_dev);
int xy_batch_get_sweep(const xy_batch* b, uint64_t* sweep);
/* Tile shape of the batch's work list (every L[i] is a multiple of it).  The
 * shape does not change the trajectory.  xy_batch_set_tile: XY_EINVAL if the
 * shape is not one of the batch's candidates (64x32, 64x16, 32x16 when every L
 * allows; else the largest of 16x16, 8x8, 4x4 that divides every L). */
int xy_batch_set_tile(xy_batch* b, int32_t tile_x, int32_t tile_y);
int xy_batch_get_tile(const xy_batch* b, int32_t* tile_x, int32_t* tile_y);
int xy_batch_set_schedule(xy_batch* b, int32_t schedule);   /* XY_EINVAL if not one of the three */
int xy_batch_get_schedule(const xy_batch* b, int32_t* schedule);
/* Time every candidate tile shape under every schedule for `sweeps_per_trial`
 * sweeps (after one untimed trial that also captures the graph) and keep the
 * fastest (shape and schedule).  The trials
 * advance the batch: run it on a scratch batch of the same sizes. */
int xy_batch_autotune(xy_batch* b, int32_t sweeps_per_trial, int32_t* tile_x, int32_t* tile_y);
/* Wait for the batch's stream and report whether any launch so far hit a barrier
 * spin limit (XY_EBARRIER) -- a guard for GPUs shared with other work.  The flag
 * is sticky: once set, the batch's later results are void as well. */
int xy_batch_status(xy_batch* b);
/* Test support (failure handling): the number of polls after which a barrier
 * wait of the persistent schedule gives up (default 2^27, several seconds).
 * After one wait has given up every later wait of the launch returns at once,
 * so the grid drains and the kernel exits normally; xy_batch_status then
 * reports XY_EBARRIER.  A limit of a few polls forces that path from the host.
 * XY_EINVAL: polls == 0. */
int xy_batch_set_spin_limit(xy_batch* b, uint32_t polls);
int xy_batch_free(xy_batch* b);

/* ------------------------------------------------ allocation-free entry point
 * For callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  Same as xy_attach(seed,
 * L, beta, delta, precision, sweep, ...) followed by xy_sweep(n_sweeps,
 * measure_every, obs_dev) and freeing the handle, with the same trajectory and
 * records bit for bit, but with no caller workspace and no handle: the
 * workspace is a fixed device array of XY_NOALLOC_SCRATCH_BYTES inside the
 * library, one per device, held from module load until the process ends.  The
 * call allocates nothing (no hipMalloc, hipFree or host heap) and reads no file;
 * it runs the default plan.  It enqueues its work on hip_stream and returns.
 * state_dev (xy_state_bytes bytes, caller-owned) holds the angles in and out;
 * obs_dev as in xy_sweep.  Every call on one device shares that device's array
 * (the counters in it are cleared at the start of each call): calls that overlap
 * in time on one device, from two streams or threads, race and give wrong
 * results.  XY_ESIZE: the workspace of (L, precision) exceeds the array (FP32:
 * L > 2432; FP16: L > 3342) or state_len is too small; XY_ERANGE: sweep +
 * n_sweeps would pass 2^32 - 1; XY_EINVAL / XY_ESTATE as xy_attach and xy_sweep;
 * XY_EHIP: the device address of the array could not be found or a launch
 * failed. */
#define XY_NOALLOC_SCRATCH_BYTES (24u << 20)
int xy_sweep_noalloc(uint64_t seed, int32_t L, double beta, double delta, int32_t precision,
                     uint64_t sweep, int64_t n_sweeps, int32_t measure_every, void* state_dev,
                     size_t state_len, xy_obs* obs_dev, void* hip_stream);

const char* xy_strerror(int code);
/* Name of the last failing HIP call and its error string (thread-local). */
const char* xy_last_hip_error(void);

/* Test support (failure handling): arm one injected failure.  The (after + 1)-th
 * launch point the library reaches from now on (a kernel launch of xy_init,
 * xy_attach, xy_sweep, xy_measure, xy_hmc or a batch graph launch, in any
 * thread) fails with hipErrorLaunchFailure without enqueueing anything, so the
 * call returns XY_EHIP and xy_last_hip_error() ends in "[injected]".  The
 * handle stays usable: its sweep counter counts exactly the sweeps that were
 * enqueued and their angles are in the caller's state buffer, so a later call
 * continues the same trajectory.  after = -1 disarms; XY_EINVAL below -1. */
int xy_test_inject_failure(int32_t after);

#ifdef __cplusplus
}
#endif

#endif /* XY_H */
