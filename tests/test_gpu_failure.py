"""Failure handling through the C ABI, forced from the host so that every kernel
still runs to its normal end.

* An injected launch failure (xy_test_inject_failure) makes a call return
  XY_EHIP part-way; the handle stays usable: its sweep counter counts exactly the
  sweeps enqueued, their angles are in the caller's buffer, and continuing gives
  the uninterrupted trajectory bit for bit, with the same records.
* A persistent batch whose barrier spin limit is a single poll gives up its
  waits; every later wait of the launch returns at once, the launch ends, and
  xy_batch_status reports XY_EBARRIER (sticky).  A fresh batch is unaffected.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

from gpu_helpers import obs_tol

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_0811_2111_amd import xy
else:
    xy = None

PLANS = {
    "stream": (64, (1, 0, 0, 1)),
    "fused": (256, (2, 128, 32, 1)),
    "fused2": (256, (2, 64, 32, 2)),
    "strip": (256, (3, 128, 32, 1)),
    "resident": (32, (4, 0, 0, 1)),
}


# (plan, launch point that fails); a resident call has a single launch point
CASES = [(name, after) for name in PLANS for after in ([0] if name == "resident" else [0, 1, 4, 7])]


@pytest.mark.parametrize("name,after", CASES)
def test_injected_failure_keeps_handle_consistent(name, after):
    L, plan = PLANS[name]
    n = 12
    ref = xy.Lattice(L, seed=77, beta=1.1, delta=1.0, plan=plan)
    ref_obs = xy.records(ref.sweep(n, 1))
    lat = xy.Lattice(L, seed=77, beta=1.1, delta=1.0, plan=plan)
    xy.xy_test_inject_failure(after)
    try:
        with pytest.raises(xy.XYError) as ei:
            lat.sweep(n, 1)
    finally:
        xy.xy_test_inject_failure(-1)
    assert ei.value.code == xy.XY_EHIP
    assert xy.lib().xy_last_hip_error().endswith(b"[injected]")
    s = lat.sweep_count
    assert 0 <= s <= n
    torch.cuda.synchronize()
    # the handle keeps working and continues the same trajectory
    if n - s > 0:
        rest = xy.records(lat.sweep(n - s, 1))
        for q in range(n - s):
            # counts exactly; the FP64 sums may be summed in another order (a call of
            # an odd number of sweeps ends on the streaming schedule), so 1e-6 relative
            assert int(rest[q]["sweep"]) == int(ref_obs[s + q]["sweep"]) == s + q + 1
            assert int(rest[q]["n_accept"]) == int(ref_obs[s + q]["n_accept"]), (name, after, s, q)
            for f in ("cx", "cy", "ix", "iy", "mx", "my"):
                r = float(ref_obs[s + q][f])
                assert abs(float(rest[q][f]) - r) <= obs_tol(r, L * L), (name, after, s, q, f)
    assert torch.equal(lat.state, ref.state)
    assert lat.sweep_count == n


def test_injected_failure_in_measure_and_batch():
    lat = xy.Lattice(64, seed=5)
    xy.xy_test_inject_failure(0)
    with pytest.raises(xy.XYError):
        lat.measure()
    out = lat.measure()
    assert xy.records(out)[0]["sweep"] == 0
    b = xy.Batch([64, 128], [1, 2], [1.0, 1.2], [1.0, 1.0])
    b.sweep(3)
    xy.xy_test_inject_failure(0)
    with pytest.raises(xy.XYError):
        b.sweep(4)
    assert b.sweep_count == 3
    b.sweep(4)
    ref = xy.Batch([64, 128], [1, 2], [1.0, 1.2], [1.0, 1.0])
    ref.sweep(7)
    torch.cuda.synchronize()
    assert torch.equal(b.state, ref.state)


def test_persistent_barrier_spin_limit_drains():
    Ls = [1024, 512, 256]
    b = xy.Batch(Ls, [1, 2, 3], [1.0, 1.1, 1.2], [1.0, 1.0, 1.0])
    b.set_schedule(xy.XY_BATCH_PERSISTENT)
    b.set_spin_limit(1)
    b.sweep(20, 5)
    torch.cuda.synchronize()
    with pytest.raises(xy.XYError) as ei:
        b.status()
    assert ei.value.code == xy.XY_EBARRIER
    with pytest.raises(xy.XYError):     # sticky
        b.status()
    fresh = xy.Batch(Ls, [1, 2, 3], [1.0, 1.1, 1.2], [1.0, 1.0, 1.0])
    fresh.set_schedule(xy.XY_BATCH_PERSISTENT)
    fresh.sweep(20, 5)
    fresh.status()
