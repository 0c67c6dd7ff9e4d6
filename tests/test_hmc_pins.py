"""Pins of the HMC oracle (oracle/xy_hmc_oracle.c) against facts it does not compute itself.

* the momenta are independent standard normal numbers (Kolmogorov-Smirnov
  against the normal CDF, moments, no correlation between neighbours);
* the force is minus the derivative of beta E, checked against central
  differences of the Metropolis oracle's energy (a different code path);
* leap-frog is time reversible and symplectic (numerical Jacobian of a short
  trajectory on 4x4: det = 1), and its energy violation falls as eps^2;
* at equilibrium <exp(-dH)> = 1 (Creutz) and the accept rate equals
  <min(1, exp(-dH))>;
* HMC samples the same ensemble: <E>/N on 4x4 against the transfer matrix
  (tests/golden), and the high-temperature series at L = 16.

A dropped factor 2 pi in the drift, a flipped force sign or an asymmetric step
order each fail several of these.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np
import pytest

from mcstats import mean_err, observables

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "exact_small_lattices.json")


@pytest.fixture(scope="module")
def exact():
    with open(GOLD) as f:
        return json.load(f)


def _random_state(L, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(0, 1, (L, L)), rng.standard_normal((L, L))


def _turn_diff(a, b):
    d = np.asarray(a) - np.asarray(b)
    return d - np.round(d)


# ------------------------------------------------------------------ momenta

def test_momenta_standard_normal(orc):
    from scipy import stats
    L = 64
    p = np.concatenate([orc.hmc_momenta(5, L, t).ravel() for t in range(4)])
    assert abs(p.mean()) < 4 / math.sqrt(p.size)
    assert abs(p.var() - 1) < 4 * math.sqrt(2 / p.size)
    assert abs(stats.kurtosis(p)) < 4 * math.sqrt(24 / p.size)
    assert stats.kstest(p, "norm").pvalue > 1e-3
    one = orc.hmc_momenta(5, L, 0)
    c = np.corrcoef(one[:, :-1].ravel(), one[:, 1:].ravel())[0, 1]
    assert abs(c) < 4 / math.sqrt(one.size)
    assert not np.array_equal(one, orc.hmc_momenta(5, L, 1))
    assert not np.array_equal(one, orc.hmc_momenta(6, L, 0))
    assert orc.hmc_momentum(5, L, 7, 3, 0) == one[3, 7]


def test_accept_uniforms_uniform(orc):
    from scipy import stats
    u = np.array([orc.hmc_accept_uniform(9, t) for t in range(4000)])
    assert np.all((u > 0) & (u < 1))
    assert stats.kstest(u, "uniform").pvalue > 1e-3


# -------------------------------------------------------------------- force

@pytest.mark.parametrize("beta", [0.7, 1.3])
def test_force_is_minus_gradient_of_beta_E(orc, beta):
    L = 6
    phi, _ = _random_state(L, 1)
    F = orc.hmc_force(phi, beta)
    h = 1e-5                                   # radians
    for (y, x) in [(0, 0), (2, 3), (5, 5), (3, 0)]:
        a = phi.copy(); a[y, x] = (a[y, x] + h / (2 * math.pi)) % 1.0
        b = phi.copy(); b[y, x] = (b[y, x] - h / (2 * math.pi)) % 1.0
        dV = beta * (orc.energy(a) - orc.energy(b)) / (2 * h)
        assert abs(F[y, x] + dV) < 1e-7, (y, x, F[y, x], -dV)
    # the force sums to zero (rotation invariance of E)
    assert abs(F.sum()) < 1e-12


# ----------------------------------------------------------------- leap-frog

def test_leapfrog_reversible(orc):
    L = 8
    phi, p = _random_state(L, 2)
    a, q = phi.copy(), p.copy()
    orc.hmc_leapfrog(a, q, 1.1, 0.1, 20)
    assert np.max(np.abs(_turn_diff(a, phi))) > 1e-3          # it moved
    q = -q
    orc.hmc_leapfrog(a, q, 1.1, 0.1, 20)
    assert np.max(np.abs(_turn_diff(a, phi))) < 1e-12
    assert np.max(np.abs(q + p)) < 1e-11


def test_leapfrog_symplectic(orc):
    """Jacobian of (theta, p) -> leap-frog(theta, p) in canonical coordinates
    (theta in radians) on 4x4, by central differences: det = 1."""
    L, n, eps, beta = 4, 3, 0.2, 1.0
    phi, p = _random_state(L, 3)
    N = L * L
    z0 = np.concatenate([2 * math.pi * phi.ravel(), p.ravel()])

    def flow(z):
        a = np.ascontiguousarray((z[:N] / (2 * math.pi)).reshape(L, L) % 1.0)
        q = np.ascontiguousarray(z[N:].reshape(L, L).copy())
        orc.hmc_leapfrog(a, q, beta, eps, n)
        return a.ravel(), q.ravel()

    J = np.zeros((2 * N, 2 * N))
    h = 1e-6
    for k in range(2 * N):
        zp, zm = z0.copy(), z0.copy()
        zp[k] += h
        zm[k] -= h
        ap, qp = flow(zp)
        am, qm = flow(zm)
        J[:N, k] = 2 * math.pi * _turn_diff(ap, am) / (2 * h)
        J[N:, k] = (qp - qm) / (2 * h)
    assert abs(np.linalg.det(J) - 1) < 1e-5


def test_energy_violation_is_second_order(orc):
    """At fixed trajectory length, halving eps divides dH by ~4."""
    L, beta, tau = 8, 1.0, 1.0
    rms = []
    for eps in (0.1, 0.05, 0.025):
        dh = []
        for s in range(8):
            phi, p = _random_state(L, 10 + s)
            H0 = orc.hmc_hamiltonian(phi, p, beta)
            orc.hmc_leapfrog(phi, p, beta, eps, int(round(tau / eps)))
            dh.append(orc.hmc_hamiltonian(phi, p, beta) - H0)
        rms.append(math.sqrt(np.mean(np.square(dh))))
    for a, b in zip(rms, rms[1:]):
        assert 3.6 < a / b < 4.4, rms


# ----------------------------------------------------------------- ensemble

def test_creutz_identity_and_acceptance(orc):
    L, beta, eps, n = 8, 1.0, 0.25, 4
    phi = orc.hot_start(21, L)
    orc.hmc_run(21, phi, beta, eps, n, 300, 1)
    rec = orc.hmc_run(21, phi, beta, eps, n, 4000, 1, traj0=300)
    dH = rec[:, 2]
    mu, err = mean_err(np.exp(-dH))
    assert abs(mu - 1) < 3 * err + 1e-3, (mu, err)
    acc = rec[:, 1]
    a_mu, a_err = mean_err(acc - np.minimum(1.0, np.exp(-dH)))
    assert abs(a_mu) < 3 * a_err + 1e-3, (a_mu, a_err)
    assert 0.3 < acc.mean() < 0.999


def test_rejected_trajectory_restores_state(orc):
    L = 8
    phi = orc.hot_start(4, L)
    before = phi.copy()
    acc, dH, _ = orc.hmc_trajectory(4, phi, 1.0, 3.0, 10, 0)    # far too large a step
    assert not acc and dH > 50
    np.testing.assert_array_equal(phi, before)


@pytest.mark.parametrize("beta", [0.5, 1.0])
def test_hmc_4x4_against_transfer_matrix(orc, exact, beta):
    ref = exact["xy_4x4_continuous_E"][repr(beta)]
    L = 4
    phi = orc.hot_start(40, L)
    rec = orc.hmc_run(40, phi, beta, 0.3, 5, 40000, 1)
    e = -(rec[:, 3] + rec[:, 4]) / (L * L)
    mu, err = mean_err(e, discard=500)
    assert abs(mu - ref["q14"]) < 3 * err, (mu, ref["q14"], err)


def test_hmc_high_temperature_series(orc):
    L, beta = 16, 0.2
    phi = orc.hot_start(41, L)
    rec = orc.hmc_run(41, phi, beta, 0.5, 4, 6000, 1)
    e = -(rec[:, 3] + rec[:, 4]) / (L * L)
    mu, err = mean_err(e, discard=200)
    series = -beta - 3 * beta ** 3 / 8 - beta ** 5 / 48
    assert abs(mu - series) < 3 * err + 2e-4, (mu, series, err)
