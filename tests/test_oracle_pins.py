"""Pins of the FP64 CPU oracle against values fixed by the mathematics.

None of these re-type the oracle's formulas: they compare it with exact
enumeration of small lattices (the q = 6 clock restriction and the continuous
model, tests/golden/exact_small_lattices.json), with closed forms (ground
state, spin waves, the antiferromagnet, beta = 0), with the high-temperature
series of <E>, with library routines (numpy's IEEE binary16 and float32
arithmetic), and with structural properties of the checkerboard update.
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


# ---------------------------------------------------------------- random stream

def test_uniform_grid_is_exact_and_symmetric(orc):
    """u(w) = (2 (w>>9) + 1) 2^-24: never 0 or 1, exact in FP32, u(w) + u(~w) = 1."""
    assert orc.u01(0) == 2.0 ** -24
    assert orc.u01(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    rng = np.random.default_rng(7)
    for w in rng.integers(0, 2 ** 32, size=2000, dtype=np.uint64):
        w = int(w)
        u = orc.u01(w)
        assert 0.0 < u < 1.0
        assert float(np.float32(u)) == u
        assert u + orc.u01(w ^ 0xFFFFFFFF) == 1.0
        assert orc.u01(w) == orc.u01(w & ~0x1FF)          # only the top 23 bits matter


KAT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "philox4x32_10_kat.txt")


def test_philox_known_answers(orc):
    """Philox4x32-10 reproduces the published known-answer vectors (Salmon et al.,
    SC'11, the Random123 test file): zero counter and key, all-ones counter and key,
    and the pi-digit counter and key.  A wrong multiplier, Weyl increment, word
    order or round count changes every output word."""
    rows = []
    with open(KAT) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(t, 16) for t in line.split()])
    assert len(rows) == 3
    for v in rows:
        out = [int(x) for x in orc.philox4x32_10(v[:4], v[4:6])]
        assert out == v[6:], (["%08x" % x for x in out], ["%08x" % x for x in v[6:]])


def test_philox_statistics(orc):
    """Philox4x32-10 words over consecutive counters: uniform bytes (chi^2),
    uncorrelated words, and avalanche of a one-bit counter change."""
    words = []
    for i in range(20000):
        words.append(orc.philox4x32_10([i, 3, 1, 0], [1, 0]))
    w = np.array(words, dtype=np.uint64)
    bytes_ = np.concatenate([(w >> s) & 0xFF for s in (0, 8, 16, 24)]).ravel()
    counts = np.bincount(bytes_.astype(np.int64), minlength=256)
    expect = bytes_.size / 256
    chi2 = float(((counts - expect) ** 2 / expect).sum())
    assert chi2 < 255 + 6 * math.sqrt(2 * 255)                   # ~6 sigma of chi^2_255
    u = (w >> 9).astype(np.float64) / 2 ** 23
    for a in range(4):
        for b in range(a + 1, 4):
            r = np.corrcoef(u[:, a], u[:, b])[0, 1]
            assert abs(r) < 6 / math.sqrt(u.shape[0])
    flips = []
    for i in range(500):
        a = orc.philox4x32_10([i, 9, 0, 0], [5, 6])
        b = orc.philox4x32_10([i ^ (1 << (i % 32)), 9, 0, 0], [5, 6])
        flips.append(sum(bin(int(x) ^ int(y)).count("1") for x, y in zip(a, b)))
    assert abs(np.mean(flips) - 64) < 2.0


def test_site_words_distinct_and_keyed(orc):
    """Every (site, sweep, purpose, seed) gets its own draw; the pair of words a
    site takes never coincides with the other site of its Philox call."""
    L = 10                                 # L/2 odd: pairs never straddle a half-row
    seen = set()
    for y in range(L):
        for x in range(L):
            seen.add(orc.site_words(1, L, x, y, 4, 0))
    assert len(seen) == L * L
    assert orc.site_words(1, L, 3, 2, 4, 0) != orc.site_words(2, L, 3, 2, 4, 0)
    assert orc.site_words(1, L, 3, 2, 4, 0) != orc.site_words(1, L, 3, 2, 5, 0)
    assert orc.site_words(1, L, 3, 2, 4, 0) != orc.site_words(1, L, 3, 2, 4, 1)


# ------------------------------------------------------------ storage rounding

def test_round_f16_matches_ieee_binary16(orc):
    rng = np.random.default_rng(3)
    vals = np.concatenate([rng.uniform(0, 2 * np.pi, 20000), rng.uniform(0, 1e-4, 2000),
                           np.float16(rng.uniform(0, 7, 500)).astype(np.float64)])
    # exact midpoints between neighbouring binary16 values exercise ties-to-even
    h = np.float16(rng.uniform(0.1, 6.2, 500)).astype(np.float64)
    mids = h + 0.5 * (np.nextafter(np.float16(h), np.float16(10)).astype(np.float64) - h)
    for v in np.concatenate([vals, mids]):
        assert orc.round_f16(v) == float(np.float16(v)), v


BELOW_ONE_F32 = float(np.nextafter(np.float32(1), np.float32(0)))


def f32_wrap(t):
    """numpy float32 arithmetic: t - floor(t), one float32 rounding, kept below 1."""
    t = np.float32(t)
    v = np.float32(t - np.floor(t))
    return np.float32(BELOW_ONE_F32) if v >= 1 else v


@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_proposal_rounding_matches_ieee_float32_arithmetic(orc, prec):
    """In the rounded storage modes the proposal (in turns) is
    float32(phi + float32(Delta r)) with Delta = float32(delta / 2 pi), wrapped by
    float32(t - floor(t)) kept below 1, then stored; checked against numpy float32."""
    rng = np.random.default_rng(11)
    for _ in range(3000):
        ph = np.float32(rng.uniform(0, 1))
        if prec == "f16":
            ph = np.float32(np.float16(ph))
        delta = float(rng.choice([1.0, 1.2, np.pi, 0.3]))
        w = int(rng.integers(0, 2 ** 32))
        u1 = orc.u01(w)
        r = np.float32(2 * u1 - 1)
        t = np.float32(ph + np.float32(np.float32(delta / (2 * np.pi)) * r))
        t = f32_wrap(t)
        if prec == "f16":
            t = np.float32(np.float16(t))
        assert orc.propose(float(ph), delta, u1, prec) == float(t)


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_proposal_wrap_edges(orc, prec):
    """Wrapped proposals stay in [0, 1) turns at the edges of the angle range
    (binary16 storage may round a value just below 1 up to 1 itself)."""
    edge_u = [orc.u01(0), orc.u01(0xFFFFFFFF), 0.5 - 2 ** -24, 0.5 + 2 ** -24]
    edge_t = [0.0, 1e-30, 1e-7, float(np.float32(1 - 6e-8)), BELOW_ONE_F32, 0.5]
    for ph in edge_t:
        for u in edge_u:
            for d in [np.pi, 1.0, 1e-6]:
                v = orc.propose(ph, d, u, prec)
                assert 0.0 <= v < 1.0 or (prec == "f16" and v == 1.0), (ph, u, d, v)


@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_proposal_tiny_negative_step_wraps_below_one(orc, prec):
    """phi = 0 moved back by less than half a float32 ulp of 1: t - floor(t) = 1 - tiny
    rounds to 1 in float32 and is kept at the largest float32 below 1 instead
    (binary16 storage then rounds that to 1)."""
    u = orc.u01(0)                      # r = 2u - 1 = -1 + 2^-23
    v = orc.propose(0.0, 1e-9, u, prec)
    assert v == (BELOW_ONE_F32 if prec == "f32" else 1.0)
    # a step of more than one float32 ulp of 1 rounds to an ordinary value below 1
    v = orc.propose(0.0, 1e-5, u, prec)
    step = np.float32(np.float32(1e-5 / (2 * np.pi)) * np.float32(2 * u - 1))
    want = np.float32(np.float32(1) + step)
    assert v == (float(want) if prec == "f32" else float(np.float16(want)))


# ---------------------------------------------------------------- observables

def test_measure_ground_state_and_rotation(orc):
    """phi = const: E = -2N exactly (2N bonds), |m| = 1, helicity estimator 1;
    M = N (cos 2 pi phi, sin 2 pi phi)."""
    L = 8
    N = L * L
    for c in [0.0, 0.21, 0.25, 0.94]:
        m = orc.measure(np.full((L, L), c))
        assert m[0] == N and m[1] == N and m[2] == 0 and m[3] == 0
        assert math.isclose(m[4], N * math.cos(2 * math.pi * c), abs_tol=1e-12)
        assert math.isclose(m[5], N * math.sin(2 * math.pi * c), abs_tol=1e-12)
        assert orc.energy(np.full((L, L), c)) == -2.0 * N
    m = orc.measure(np.full((L, L), 0.25))      # a quarter turn: M along +y
    assert abs(m[4]) < 1e-12 and math.isclose(m[5], N, rel_tol=1e-15)


def test_measure_spin_wave_closed_form(orc):
    """theta(x, y) = 2 pi n x / L (phi = n x / L turns): Cx = N cos(2 pi n/L),
    Ix = -N sin(2 pi n/L), Cy = N, Iy = 0, M = 0; the transposed wave swaps the x
    and y sums."""
    L, n = 12, 1
    N = L * L
    x = np.arange(L)
    th = np.tile(n * x / L, (L, 1))
    m = orc.measure(th)
    k = 2 * np.pi * n / L
    np.testing.assert_allclose(m, [N * math.cos(k), N, -N * math.sin(k), 0, 0, 0], atol=1e-9)
    mt = orc.measure(np.ascontiguousarray(th.T))
    np.testing.assert_allclose(mt, [N, N * math.cos(k), 0, -N * math.sin(k), 0, 0], atol=1e-9)


def test_measure_antiferromagnet(orc):
    """theta = pi (x + y), half a turn on every other site: every bond
    anti-aligned, E = +2N, M = 0."""
    L = 6
    y, x = np.mgrid[0:L, 0:L]
    m = orc.measure(0.5 * ((x + y) % 2))
    np.testing.assert_allclose(m, [-L * L, -L * L, 0, 0, 0, 0], atol=1e-9)


def test_measure_single_rotated_site(orc):
    """One site turned by a from a uniform state changes exactly its 4 bonds:
    E rises by 4 (1 - cos a); its outgoing and incoming bond sines cancel (sin a and
    sin(-a)) in both directions."""
    L = 8
    th = np.zeros((L, L))
    a = 0.7
    th[3, 5] = a / (2 * math.pi)
    m = orc.measure(th)
    N = L * L
    assert math.isclose(-(m[0] + m[1]), -2 * N + 4 * (1 - math.cos(a)), abs_tol=1e-12)
    assert math.isclose(m[2], 0.0, abs_tol=1e-12) and math.isclose(m[3], 0.0, abs_tol=1e-12)


# --------------------------------------------------------- sweep structure

def test_hot_start_rounding_modes(orc):
    """The hot start phi = u lies on the 2^-24 odd grid, exact in FP32; FP16 storage
    rounds it once."""
    L = 16
    t64 = orc.hot_start(5, L, "f64")
    assert np.all((t64 > 0) & (t64 < 1))
    assert np.all(np.mod(t64 * 2 ** 24, 2) == 1)
    np.testing.assert_array_equal(orc.hot_start(5, L, "f32"), t64)
    np.testing.assert_array_equal(orc.hot_start(5, L, "f16"), t64.astype(np.float16).astype(np.float64))
    assert not np.array_equal(t64, orc.hot_start(6, L, "f64"))


def test_checkerboard_red_reads_only_black(orc):
    """Within a colour the updates are independent: the red half-sweep reads only
    black angles, so perturbing one red site before a sweep can change nothing but
    that site and, in the black half-sweep, its four black neighbours.  (A raster
    sweep over all sites would let the change cascade along the row.)"""
    L = 8
    for beta in [0.5, 1.0, 3.0]:
        for s in range(5):
            th0 = orc.hot_start(1 + s, L)
            a = th0.copy(); orc.sweep(1, a, beta, 1.0, s)
            b = th0.copy(); b[2, 4] = (b[2, 4] + 0.16) % 1.0
            orc.sweep(1, b, beta, 1.0, s)
            allowed = np.zeros((L, L), dtype=bool)
            for (yy, xx) in [(2, 4), (1, 4), (3, 4), (2, 3), (2, 5)]:
                allowed[yy, xx] = True
            assert not np.any((a != b) & ~allowed)


def test_beta_zero_accepts_everything(orc):
    L = 8
    th = orc.hot_start(2, L)
    rec = orc.run(2, th, 0.0, 1.0, 20, 1)
    assert np.all(rec[:, 1] == L * L)


def test_cold_start_frozen_at_huge_beta(orc):
    """From the ground state every proposal raises E, so at beta = 1e9 nothing is
    accepted and E stays exactly -2N."""
    L = 8
    th = np.zeros((L, L))
    rec = orc.run(3, th, 1e9, 0.5, 10, 1)
    assert np.all(rec[:, 1] == 0)
    assert np.all(-(rec[:, 2] + rec[:, 3]) == -2 * L * L)


def test_sweep_index_keys_the_stream(orc):
    """run(sweep0 = s) over k sweeps equals k single sweeps with indices s..s+k-1,
    and resuming a split run reproduces the unsplit run bit for bit."""
    L = 8
    a = orc.hot_start(4, L)
    orc.run(4, a, 1.1, 1.0, 7, 7, sweep0=3)
    b = orc.hot_start(4, L)
    for s in range(3, 10):
        orc.sweep(4, b, 1.1, 1.0, s)
    np.testing.assert_array_equal(a, b)
    c = orc.hot_start(4, L)
    orc.run(4, c, 1.1, 1.0, 3, 3, sweep0=3)
    orc.run(4, c, 1.1, 1.0, 4, 4, sweep0=6)
    np.testing.assert_array_equal(a, c)


def test_diagnostics_consistent(orc):
    """Per-site diagnostics: decision == (dE < T), T = -ln(u2)/beta, accepted sites
    hold the proposal; dE of the proposal agrees with a direct energy difference
    for the first red site (nothing before it has moved)."""
    L = 8
    th = orc.hot_start(9, L)
    th0 = th.copy()
    d = orc.sweep(9, th, 1.0, 1.0, 0, diagnostics=True)
    assert np.array_equal(d["dec"], d["dE"] < d["thr"])
    assert d["accepts"] == int(d["dec"].sum())
    np.testing.assert_array_equal(th[d["dec"]], d["prop"][d["dec"]])
    t1 = th0.copy(); t1[0, 0] = d["prop"][0, 0]
    assert math.isclose(d["dE"][0, 0], orc.energy(t1) - orc.energy(th0), abs_tol=1e-12)


# ------------------------------------------------ physics against exact values

def _clock_series(orc, L, q, beta, n, seed):
    rng = np.random.default_rng(seed)
    ks = rng.integers(0, q, size=(L, L)).astype(np.int32)
    rec = orc.clock_run(seed, ks, q, beta, n, 1)
    return observables(rec, L * L, beta)


@pytest.mark.parametrize("beta", [0.5, 1.0, 2.0])
def test_clock_3x3_q6_against_enumeration(orc, exact, beta):
    """3x3 periodic q = 6 clock model (odd L: sequential order): <E>/N, <|m|> and the
    helicity modulus within 3 sigma of the brute-force sums over all 6^9 states."""
    ex = exact["clock_3x3_q6_bruteforce"][repr(beta)]
    e, m, u = _clock_series(orc, 3, 6, beta, 200000, seed=21)
    for series, key in [(e, "E_per_site"), (m, "abs_m"), (u, "helicity")]:
        mu, err = mean_err(series, discard=1000)
        assert abs(mu - ex[key]) < 3 * err, (key, mu, ex[key], err)
    # the clock and continuous models differ here by many sigma: the test tells them apart
    if beta == 1.0:
        mu, err = mean_err(e, discard=1000)
        cont = exact["xy_3x3_continuous_E"]["1.0"]["q16"]
        assert abs(mu - cont) > 5 * err


@pytest.mark.parametrize("beta", [0.5, 1.0, 2.0])
def test_clock_4x4_q6_checkerboard_against_transfer_matrix(orc, exact, beta):
    ex = exact["clock_4x4_q6_transfer_E"][repr(beta)]
    e, _, _ = _clock_series(orc, 4, 6, beta, 100000, seed=22)
    mu, err = mean_err(e, discard=1000)
    assert abs(mu - ex) < 3 * err, (mu, ex, err)


@pytest.mark.parametrize("L,key,delta", [(3, "xy_3x3_continuous_E", 2.0),
                                         (4, "xy_4x4_continuous_E", 2.0)])
@pytest.mark.parametrize("beta", [0.5, 1.0, 2.0])
def test_continuous_small_lattices_against_transfer_matrix(orc, exact, L, key, delta, beta):
    """Continuous XY on 3x3 (sequential) and 4x4 (checkerboard, the smallest lattice
    the device path runs): <E>/N within 3 sigma of the q -> infinity transfer-matrix
    limit (two q values agree far below the error bar)."""
    ref = exact[key][repr(beta)]
    assert ref["diff"] < 1e-4
    exact_e = ref["q16"] if "q16" in ref else ref["q14"]
    th = orc.hot_start(30 + L, L)
    rec = orc.run(30 + L, th, beta, delta, 100000, 1)
    e, _, _ = observables(rec, L * L, beta)
    mu, err = mean_err(e, discard=1000)
    assert abs(mu - exact_e) < 3 * err, (mu, exact_e, err)


@pytest.mark.parametrize("beta", [0.1, 0.2, 0.3])
def test_high_temperature_series(orc, beta):
    """<E>/N = -beta - 3 beta^3/8 - beta^5/48 + O(beta^7) (character expansion; the
    leading closed currents are the unit plaquette and the 1x2 rectangle) on L = 16,
    where winding corrections O(t1^16) are negligible.  At beta = 0.3 the cubic term
    alone is ~15 error bars, so a dropped or mis-signed term fails."""
    L = 16
    th = orc.hot_start(40, L)
    rec = orc.run(40, th, beta, 2.0, 20000, 1)
    e, _, _ = observables(rec, L * L, beta)
    mu, err = mean_err(e, discard=200)
    series = -beta - 3 * beta ** 3 / 8 - beta ** 5 / 48
    assert abs(mu - series) < 3 * err + 2 * beta ** 7, (mu, series, err)


def test_low_temperature_spin_waves(orc):
    """beta = 20, cold start: <E>/N = -2 + (1 - 1/N)/(2 beta) + 1/(16 beta^2) + O(beta^-3)
    (equipartition over N - 1 harmonic modes plus the first quartic correction)."""
    L, beta = 16, 20.0
    N = L * L
    th = np.zeros((L, L))
    rec = orc.run(41, th, beta, 0.5, 10000, 1)
    e, _, _ = observables(rec, N, beta)
    mu, err = mean_err(e, discard=1000)
    pred = -2 + (1 - 1 / N) / (2 * beta) + 1 / (16 * beta ** 2)
    assert abs(mu - pred) < 3 * err + 1 / beta ** 3, (mu, pred, err)


def test_beta_zero_rayleigh(orc):
    """beta = 0: i.i.d. uniform angles in equilibrium, <E> = 0 and
    <|sum e^{i theta}|>/N -> sqrt(pi / (4N)) (Rayleigh)."""
    L = 16
    N = L * L
    th = orc.hot_start(42, L)
    rec = orc.run(42, th, 0.0, np.pi, 5000, 1)
    e, m, _ = observables(rec, N, 0.0)
    mu, err = mean_err(e)
    assert abs(mu) < 3 * err
    mu, err = mean_err(m)
    assert abs(mu - math.sqrt(math.pi / (4 * N))) < 3 * err + 1e-3 / math.sqrt(N)
