"""Pins of the parallel-tempering oracle (oracle/xy_pt_oracle.c).

* with every rung at the same temperature every exchange is accepted, so the
  lattices move along the ladder in the fixed even/odd pattern;
* a ladder of 4x4 lattices at beta = 0.5, 1.0, 2.0 samples each temperature's
  ensemble: the energies measured on each rung match the transfer-matrix values
  (tests/golden) -- a flipped sign or a wrong index in the exchange rule would
  send configurations to the wrong temperatures and bias them;
* the exchange uniforms are uniform and distinct per (round, ladder, rung).
"""
from __future__ import annotations

import json
import os

import numpy as np
import pytest

from mcstats import mean_err

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "exact_small_lattices.json")


def ladder(orc, L, M, seed0):
    phi = np.ascontiguousarray(np.stack([orc.hot_start(seed0 + i, L, "f32") for i in range(M)]))
    return phi, np.arange(M, dtype=np.int32)


def test_equal_temperatures_accept_every_exchange(orc):
    L, M = 8, 5
    phi, member = ladder(orc, L, M, 10)
    _, rung = orc.pt_run([10 + i for i in range(M)], phi, [1.0] * M, [1.0] * M, member, 7, 4, 1)
    # round 0 swaps (0,1),(2,3); round 1 swaps (1,2),(3,4); ...
    expect = list(range(M))
    for r in range(4):
        for i in range(M):
            assert rung[r, i] == expect.index(i)
        for t in range(r & 1, M - 1, 2):
            expect[t], expect[t + 1] = expect[t + 1], expect[t]
    assert list(member) == expect


def test_exchange_uniforms(orc):
    from scipy import stats
    u = np.array([orc.pt_uniform(3, r, g, t) for r in range(200) for g in range(3) for t in range(8)])
    assert len(set(u.tolist())) == u.size
    assert stats.kstest(u, "uniform").pvalue > 1e-3


def test_ladder_samples_each_temperature(orc):
    with open(GOLD) as f:
        exact = json.load(f)["xy_4x4_continuous_E"]
    betas = [0.5, 1.0, 2.0]
    L, M = 4, 3
    phi, member = ladder(orc, L, M, 20)
    rec, rung = orc.pt_run([20, 21, 22], phi, betas, [2.0] * M, member, 11, 40000, 1)
    e = -(rec[:, :, 3] + rec[:, :, 4]) / (L * L)          # (rounds, lattices)
    swaps = np.mean(rung[1:] != rung[:-1])
    assert swaps > 0.05                                     # the ladder does exchange
    for t, b in enumerate(betas):
        series = np.array([e[r, np.where(rung[r] == t)[0][0]] for r in range(e.shape[0])])
        mu, err = mean_err(series, discard=500)
        assert abs(mu - exact[repr(b)]["q14"]) < 3 * err, (b, mu, exact[repr(b)]["q14"], err)
