"""Four-replica lattices (xy_quad_* through the C ABI).

Replica r draws the numbers of a single lattice with seed_r, so its angles must
equal, bit for bit, those of the single-lattice path with (seed_r, beta_r,
delta_r), and through it the oracle's (up to the near-threshold decisions the
single-lattice parity tests exempt); this is checked directly against the oracle
too.  Records agree with an FP64 recomputation from the final state.
"""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch

from gpu_helpers import EXEMPT, exempt_mask, natural, obs_tol

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_0811_2111_amd import xy
else:  # collected on CPU-only machines; skipped by the marker filter
    xy = None

SEEDS = [3, 4, 5, 6]
BETAS = [0.7, 1.0, 1.2, 2.0]
DELTAS = [1.0, 1.2, 0.8, 0.5]
SHAPES = [(32, 16), (64, 8), (64, 16), (128, 4), (128, 8)]


def singles(L, n, measure_every=0):
    out = []
    for s, b, d in zip(SEEDS, BETAS, DELTAS):
        lat = xy.Lattice(L, seed=s, beta=b, delta=d)
        rec = lat.sweep(n, measure_every) if n else None
        out.append((lat, rec))
    return out


@pytest.mark.parametrize("L", [32, 96])
def test_quad_hot_start_matches_single_and_oracle(orc, L):
    q = xy.Quad(L, SEEDS, BETAS, DELTAS)
    for r, s in enumerate(SEEDS):
        lat = xy.Lattice(L, seed=s)
        assert torch.equal(q.replica_state(r), lat.state)
        np.testing.assert_array_equal(natural(q.replica_state(r)), orc.hot_start(s, L, "f32"))
    cold = xy.Quad(L, SEEDS, BETAS, DELTAS, start="cold")
    assert float(cold.state.abs().max()) == 0.0


@pytest.mark.parametrize("n", [1, 6, 7])
def test_quad_replicas_equal_single_lattices(n):
    L = 64
    q = xy.Quad(L, SEEDS, BETAS, DELTAS)
    qrec = q.sweep(n, 2)
    ref = singles(L, n, 2)
    for r, (lat, rec) in enumerate(ref):
        assert torch.equal(q.replica_state(r), lat.state), r
        if qrec is not None:
            a, b = xy.records(qrec[:, r]), xy.records(rec)
            np.testing.assert_array_equal(a["sweep"], b["sweep"])
            np.testing.assert_array_equal(a["n_accept"], b["n_accept"])
            for name in ("cx", "cy", "ix", "iy", "mx", "my"):
                np.testing.assert_allclose(a[name], b[name], rtol=0, atol=1e-7 * L * L)
    assert q.sweep_count == n


def test_quad_replica_against_oracle(orc):
    """Replica 1 sweep by sweep against the oracle (FP32 storage emulation): the
    angles agree bit for bit except at near-threshold decisions."""
    L, r = 32, 1
    q = xy.Quad(L, SEEDS, BETAS, DELTAS)
    th = orc.hot_start(SEEDS[r], L, "f32")
    for s in range(12):
        diag = orc.sweep(SEEDS[r], th, BETAS[r], DELTAS[r], s, prec="f32", diagnostics=True)
        q.sweep(1)
        dev = natural(q.replica_state(r))
        ex = exempt_mask(diag, L)
        if np.any(ex):
            np.testing.assert_array_equal(dev[~ex], th[~ex])
            return                                   # the trajectories may part after an exempt site
        np.testing.assert_array_equal(dev, th)


def test_quad_tile_invariance():
    L = 128
    states = []
    for tx, ty in SHAPES:
        q = xy.Quad(L, SEEDS, BETAS, DELTAS)
        q.set_tile(tx, ty)
        assert q.tile == (tx, ty)
        q.sweep(4)
        states.append(q.state.clone())
    for s in states[1:]:
        assert torch.equal(s, states[0])


def test_quad_records_match_fp64_recompute():
    L = 128
    q = xy.Quad(L, SEEDS, BETAS, DELTAS)
    rec = q.sweep(3, 3)
    tp = 2 * math.pi
    for r in range(4):
        nat = torch.tensor(natural(q.replica_state(r)), dtype=torch.float64, device="cuda")
        right = torch.roll(nat, -1, 1)
        down = torch.roll(nat, -1, 0)
        ref = [torch.cos(tp * (nat - right)).sum(), torch.cos(tp * (nat - down)).sum(),
               torch.sin(tp * (nat - right)).sum(), torch.sin(tp * (nat - down)).sum(),
               torch.cos(tp * nat).sum(), torch.sin(tp * nat).sum()]
        a = xy.records(rec[:, r])
        assert int(a["sweep"][0]) == 3 and 0 < int(a["n_accept"][0]) < L * L
        for name, v in zip(["cx", "cy", "ix", "iy", "mx", "my"], ref):
            assert abs(float(a[name][0]) - float(v)) <= obs_tol(float(v), L * L), (r, name)


def test_quad_full_size_equals_single_lattices():
    L = 4096
    q = xy.Quad(L, SEEDS, BETAS, DELTAS)
    q.sweep(3)
    for r, s in enumerate(SEEDS):
        lat = xy.Lattice(L, seed=s, beta=BETAS[r], delta=DELTAS[r])
        lat.sweep(3)
        assert torch.equal(q.replica_state(r), lat.state), r
        del lat


def test_quad_error_codes():
    L_ = xy.lib()
    s = torch.empty(1, device="cuda")
    sz = ctypes_size()
    for bad in (16, 48, 33, 0, -32):
        assert L_.xy_quad_state_bytes(bad, sz, None) == xy.XY_EINVAL
    q = xy.Quad(64, SEEDS, BETAS, DELTAS)
    assert L_.xy_quad_set_tile(q.h, 32, 8) == xy.XY_EINVAL        # not a quad shape
    assert L_.xy_quad_set_tile(q.h, 128, 4) == xy.XY_EINVAL       # does not divide L = 64
    assert L_.xy_quad_sweep(q.h, -1, 0, None) == xy.XY_EINVAL
    assert L_.xy_quad_sweep(None, 1, 0, None) == xy.XY_ESTATE
    q.set_sweep(0xFFFFFFFF - 2)
    assert L_.xy_quad_sweep(q.h, 5, 0, None) == xy.XY_ERANGE
    with pytest.raises(xy.XYError):
        xy.Quad(64, SEEDS, [1.0, 1.0, -1.0, 1.0], DELTAS)
    del s


def ctypes_size():
    import ctypes
    return ctypes.byref(ctypes.c_size_t())
