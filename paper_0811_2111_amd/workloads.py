"""Seeded synthetic workloads (inputs only; none of the method's arithmetic).

The paper's workloads are synthetic lattices of side 128..2048 (Table 1); the
configurations below are the ones the benchmarks and tests run.  Every random
choice is drawn from a named, seeded numpy generator so that it is reproducible.
"""
from __future__ import annotations

import numpy as np

# single lattice, MALL-resident: L = 4096, beta = 1.12, delta = 1.0,
# 1000 thermalisation + 10^4 sweeps, E/M every 10 sweeps
SINGLE_4096 = dict(L=4096, beta=1.12, delta=1.0, seed=1, therm=1000, sweeps=10000, measure_every=10)

# HBM-streaming: L = 16384 (1 GiB of FP32 angles), beta = 1.0, delta = 1.2, 500 sweeps,
# every observable every sweep
SINGLE_16384 = dict(L=16384, beta=1.0, delta=1.2, seed=1, therm=0, sweeps=500, measure_every=1)

# parity case: L = 32, beta = 1.0, delta = 1.0, seed 1, hot start, 1000 sweeps, every sweep
PARITY_32 = dict(L=32, beta=1.0, delta=1.0, seed=1, sweeps=1000, measure_every=1)

# precision study: L = 8192 at beta in {0.9, 1.0, 1.1}, FP16 vs FP32 storage, 2x10^4 sweeps,
# bias against the oracle on L = 256 with matched random numbers
PRECISION = dict(L=8192, betas=(0.9, 1.0, 1.1), delta=1.0, seed=1, sweeps=20000, discard=2000,
                 bias_L=256)


# four replicas of one L = 4096 lattice at four temperatures in one float4 state
# (the four-channel texel of section 3.2), records every 10 sweeps
QUAD_4096 = dict(L=4096, seeds=[1, 2, 3, 4], betas=[0.9, 1.0, 1.12, 1.3], delta=1.0, sweeps=1000, measure_every=10)

# hybrid Monte Carlo (the paper's update): n_md leap-frog steps of size eps per
# trajectory, after `therm` Metropolis sweeps from the hot start; eps falls with
# the lattice size (the mean energy violation grows like L^2 eps^4)
HMC_4096 = dict(L=4096, beta=1.0, eps=0.02, n_md=20, seed=1, therm=500, traj=50)
HMC_16384 = dict(L=16384, beta=1.0, eps=0.01, n_md=20, seed=1, therm=200, traj=20)
# batched HMC over the temperature scan (lattices of L = 64 .. 1024, their own beta)
HMC_SCAN = dict(eps=0.04, n_md=20, therm=100, traj=20, traj_per_lattice_timed=5)
# HMC on the four-replica texel: the quad's four temperatures, the L = 4096 step
QUAD_HMC_4096 = dict(L=4096, seeds=[1, 2, 3, 4], betas=[0.9, 1.0, 1.12, 1.3], eps=0.02, n_md=20, therm=200, traj=10)


def temperature_scan(n: int = 96, sizes=(64, 128, 256, 512, 1024), beta_lo: float = 0.80,
                     beta_hi: float = 1.30, seed: int = 1):
    """The batched temperature scan: n lattices with L drawn uniformly from `sizes`
    and beta uniform in [beta_lo, beta_hi], both from numpy PCG64(seed); lattice i
    uses Philox seed 1 + i and delta = 1.0; 5000 sweeps, a record every 10."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Ls = [int(v) for v in rng.choice(np.asarray(sizes), size=n)]
    betas = [float(v) for v in rng.uniform(beta_lo, beta_hi, size=n)]
    seeds = [1 + i for i in range(n)]
    deltas = [1.0] * n
    return dict(Ls=Ls, betas=betas, seeds=seeds, deltas=deltas, sweeps=5000, measure_every=10)
