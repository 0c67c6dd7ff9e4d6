"""Hybrid Monte Carlo on the four-replica texel (xy_quad_hmc through the C ABI).

Replica r must follow, bit for bit, the trajectory that xy_hmc gives a single
lattice with (seed_r, beta_r) and the same n_md and eps: the same angles and
decisions, and dH and the observables up to the rounding of FP64 sums taken in
another order (the quad sums each replica's per-site terms in its own record
layout).  Through the single-lattice path that is the oracle's trajectory
(test_gpu_hmc); the first trajectory from the hot start is also checked against
the FP64 HMC oracle directly.
"""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch

from gpu_helpers import natural, obs_tol

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_0811_2111_amd import xy
else:  # collected on CPU-only machines; skipped by the marker filter
    xy = None

SEEDS = [31, 32, 33, 34]
BETAS = [0.8, 1.0, 1.15, 1.4]
FIELDS = ["cx", "cy", "ix", "iy", "mx", "my"]
DECISION_EXEMPT = 1e-4


def turn_dist(a, b):
    d = np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)
    return np.abs(d - np.round(d))


def assert_replica_matches(qrec, srec, r, L):
    """Replica r's records against a single lattice's: counters and decisions
    exact, dH and sums to FP64 rounding (a decision could part only if u and
    exp(-dH) agreed to that rounding)."""
    assert np.array_equal(qrec["traj"][:, r], srec["traj"]), r
    assert np.array_equal(qrec["accepted"][:, r], srec["accepted"]), (r, qrec["dH"][:, r], srec["dH"])
    np.testing.assert_allclose(qrec["dH"][:, r], srec["dH"], rtol=0, atol=1e-9 * L * L)
    for f in FIELDS:
        np.testing.assert_allclose(qrec[f][:, r], srec[f], rtol=0, atol=1e-9 * L * L, err_msg=f)


@pytest.mark.parametrize("L", [32, 64, 96])
def test_quad_hmc_replicas_equal_single_lattices(L):
    """Metropolis sweeps, then trajectories with an odd step count (the final
    angles come back from the second buffer), then an even one with a larger
    step: every replica's angles bit for bit those of its single lattice."""
    q = xy.Quad(L, SEEDS, BETAS)
    q.sweep(2)
    q1 = xy.hmc_records(q.hmc(3, 9, 0.12))
    q2 = xy.hmc_records(q.hmc(2, 10, 0.3))
    assert q1.shape == (3, 4) and q.sweep_count == 7
    for r in range(4):
        lat = xy.Lattice(L, seed=SEEDS[r], beta=BETAS[r])
        lat.sweep(2)
        s1 = xy.hmc_records(lat.hmc(3, 9, 0.12))
        s2 = xy.hmc_records(lat.hmc(2, 10, 0.3))
        assert_replica_matches(q1, s1, r, L)
        assert_replica_matches(q2, s2, r, L)
        assert torch.equal(q.replica_state(r), lat.state), (L, r)
    q.sweep(1)                                       # and Metropolis goes on from the shared counter
    for r in range(4):
        lat = xy.Lattice(L, seed=SEEDS[r], beta=BETAS[r])
        lat.sweep(2)
        lat.hmc(3, 9, 0.12)
        lat.hmc(2, 10, 0.3)
        lat.sweep(1)
        assert torch.equal(q.replica_state(r), lat.state), (L, r)


def test_quad_hmc_vector_acceptance():
    """Replicas at very different temperatures in one trajectory: near-free ones
    (small beta) are accepted, cold ones with a long step rejected, and each
    keeps its own component (z theta_new + (1 - z) theta_old), as its single
    lattice does."""
    L, betas, eps, n = 64, [1e-4, 3.0, 1e-4, 3.0], 0.6, 8
    q = xy.Quad(L, SEEDS, betas)
    before = q.state.clone()
    rec = xy.hmc_records(q.hmc(2, n, eps))
    acc = rec["accepted"]
    assert acc[0].tolist() == [1, 0, 1, 0], rec["dH"]
    for r in range(4):
        lat = xy.Lattice(L, seed=SEEDS[r], beta=betas[r])
        srec = xy.hmc_records(lat.hmc(2, n, eps))
        assert_replica_matches(rec, srec, r, L)
        assert torch.equal(q.replica_state(r), lat.state), r
        if acc[0, r] == 0 and acc[1, r] == 0:
            assert torch.equal(q.replica_state(r), before[..., r]), r


def test_quad_hmc_first_trajectory_matches_oracle(orc):
    """From the hot start (L = 32), each replica's first trajectory against the
    FP64 HMC oracle with the replica's seed and beta: dH within the single-lattice
    tolerance, the decision outside the exemption band, the final angles and the
    record's sums."""
    L, eps, n = 32, 0.1, 10
    q = xy.Quad(L, SEEDS, BETAS)
    rec = xy.hmc_records(q.hmc(1, n, eps))
    for r in range(4):
        phi = orc.hot_start(SEEDS[r], L, "f32")
        acc, dH, _ = orc.hmc_trajectory(SEEDS[r], phi, BETAS[r], eps, n, 0)
        tol = 1e-4 + 1e-5 * abs(dH)
        assert abs(float(rec["dH"][0, r]) - dH) < tol, (r, float(rec["dH"][0, r]), dH)
        u = orc.hmc_accept_uniform(SEEDS[r], 0)
        st = natural(q.replica_state(r).contiguous())
        if abs(math.exp(-dH) - u) > DECISION_EXEMPT:
            assert bool(rec["accepted"][0, r]) == acc, r
            assert np.max(turn_dist(st, phi)) < 1e-5, r      # phi: the oracle's angles after its decision
        m = orc.measure(st)
        for name, ref in zip(FIELDS, m):
            assert abs(float(rec[name][0, r]) - ref) <= obs_tol(ref, L * L), (r, name)
    assert int(rec["traj"][0, 0]) == 1 and q.sweep_count == 1


def test_quad_hmc_error_codes():
    L = 32
    q = xy.Quad(L, SEEDS, BETAS)
    lib = xy.lib()
    with pytest.raises(xy.XYError) as ei:
        q.hmc(1, 0, 0.1)
    assert ei.value.code == xy.XY_EINVAL
    with pytest.raises(xy.XYError) as ei:
        q.hmc(1, 5, float("nan"))
    assert ei.value.code == xy.XY_EINVAL
    with pytest.raises(xy.XYError) as ei:
        q.hmc(-1, 5, 0.1)
    assert ei.value.code == xy.XY_EINVAL
    small = torch.empty((1024,), dtype=torch.uint8, device="cuda")
    assert lib.xy_quad_hmc(q.h, 1, 5, 0.1, small.data_ptr(), small.numel(), None) == xy.XY_ESIZE
    assert lib.xy_quad_hmc(q.h, 1, 5, 0.1, None, 1 << 30, None) == xy.XY_ESTATE
    q.set_sweep(2 ** 32 - 3)
    with pytest.raises(xy.XYError) as ei:
        q.hmc(3, 5, 0.1)
    assert ei.value.code == xy.XY_ERANGE
    assert q.sweep_count == 2 ** 32 - 3
    q.hmc(1, 5, 0.1)
    assert q.sweep_count == 2 ** 32 - 2
    torch.cuda.synchronize()


def test_quad_hmc_bench_size_equals_single_lattices():
    """The benchmark's configuration (L = 4096, beta 0.9 .. 1.3, eps = 0.02, 20
    steps) after Metropolis sweeps: two trajectories, every replica's angles bit
    for bit those of its single lattice (7-step passes on 64 x 64 tiles there,
    4-step passes on 32 x 32 tiles here)."""
    from paper_0811_2111_amd import workloads
    hc = workloads.QUAD_HMC_4096
    L = hc["L"]
    q = xy.Quad(L, hc["seeds"], hc["betas"])
    q.sweep(3)
    rec = xy.hmc_records(q.hmc(2, hc["n_md"], hc["eps"]))
    for r in range(4):
        lat = xy.Lattice(L, seed=hc["seeds"][r], beta=hc["betas"][r])
        lat.sweep(3)
        srec = xy.hmc_records(lat.hmc(2, hc["n_md"], hc["eps"]))
        assert lat.hmc_steps_per_pass == 7
        assert_replica_matches(rec, srec, r, L)
        assert torch.equal(q.replica_state(r), lat.state), r
        del lat
    del q
    torch.cuda.empty_cache()


def test_quad_hmc_steps_per_pass_bit_identical():
    """One step per pass over the state and passes of 2, 3 or 4 steps on grown
    32 x 32 tiles (step counts that leave a short last pass, odd and even pass
    counts) give the same trajectory bit for bit; settings outside 1 .. 4 are
    refused."""
    L = 96
    ref = None
    for steps in (1, 2, 3, 4):
        q = xy.Quad(L, SEEDS, BETAS)
        q.set_hmc_steps_per_pass(steps)
        assert q.hmc_steps_per_pass == steps
        q.sweep(1)
        rec = xy.hmc_records(q.hmc(2, 9, 0.15))
        q.hmc(1, 10, 0.15)
        got = (q.state.clone(), rec)
        if ref is None:
            ref = got
        else:
            assert torch.equal(got[0], ref[0]), steps
            assert np.array_equal(got[1]["accepted"], ref[1]["accepted"]), steps
            np.testing.assert_allclose(got[1]["dH"], ref[1]["dH"], rtol=0, atol=1e-9 * L * L)
        del q
    q = xy.Quad(32, SEEDS, BETAS)
    for bad in (0, 5):
        with pytest.raises(xy.XYError) as ei:
            q.set_hmc_steps_per_pass(bad)
        assert ei.value.code == xy.XY_EINVAL
    assert q.hmc_steps_per_pass == 4
