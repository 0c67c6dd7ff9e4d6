"""The allocation-free entry point (xy_sweep_noalloc) against the existing one.

xy_sweep_noalloc runs the sweeps of xy_attach + xy_sweep with the library's
fixed per-device array as the workspace.  Both are called through the C ABI on
the same starting angles; the final angles and every record must agree bit for
bit.  Two calls in a row, the second on a smaller lattice, check that what the
first call left in the shared array does not leak into the second (counters are
cleared per call, partial records fully rewritten).
"""
from __future__ import annotations

import ctypes

import pytest
import torch

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_0811_2111_amd import xy
else:
    xy = None


def _pair(L, prec, seed, beta, delta, sweep0, n, me):
    base = xy.Lattice(L, seed=seed, beta=beta, delta=delta, precision=prec)
    a_state = base.state.clone()
    b_state = base.state.clone()
    ref = xy.Lattice(L, seed=seed, beta=beta, delta=delta, precision=prec, state=a_state, sweep=sweep0)
    ref_out = ref.sweep(n, me)
    nrec = n // me
    out = torch.full((nrec, 8), float("nan"), dtype=torch.float64, device=b_state.device)
    stream = torch.cuda.current_stream()
    rc = xy.lib().xy_sweep_noalloc(seed, L, beta, delta, xy._PREC[prec], sweep0, n, me,
                                   ctypes.c_void_p(b_state.data_ptr()), b_state.numel() * b_state.element_size(),
                                   ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream.cuda_stream))
    assert rc == 0, xy.lib().xy_strerror(rc)
    torch.cuda.synchronize()
    assert torch.equal(a_state, b_state)
    r_ref, r_new = xy.records(ref_out), xy.records(out)
    assert r_ref.tobytes() == r_new.tobytes()
    assert int(r_new[-1]["sweep"]) == sweep0 + nrec * me
    assert int(r_new[0]["n_accept"]) > 0


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_noalloc_two_calls_match_existing_entry_point(prec):
    big = 2432 if prec == "fp32" else 3342
    # first call: the largest lattice the array holds (L % 4 == 0: fused plan)
    _pair(2048, prec, 11, 1.05, 1.0, 7, 9, 3)
    # second call, smaller lattice, every sweep measured
    _pair(256, prec, 12, 0.9, 1.2, 0, 6, 1)
    # and the maximum size, then a tiny one on the streaming plan (L % 4 != 0)
    _pair(big, prec, 13, 1.1, 1.0, 2, 4, 2)
    _pair(6, prec, 14, 1.0, 1.0, 1, 5, 1)


def test_noalloc_rejects_sizes_beyond_the_array():
    st = torch.empty((2, 2436, 2436 // 2), dtype=torch.float32, device="cuda")
    rc = xy.lib().xy_sweep_noalloc(1, 2436, 1.0, 1.0, 0, 0, 1, 0, ctypes.c_void_p(st.data_ptr()),
                                   st.numel() * 4, None, None)
    assert rc == xy.XY_ESIZE
    rc = xy.lib().xy_sweep_noalloc(1, 2432, 1.0, 1.0, 0, 0, 1, 0, ctypes.c_void_p(st.data_ptr()), 100, None, None)
    assert rc == xy.XY_ESIZE
    rc = xy.lib().xy_sweep_noalloc(1, 64, 1.0, 1.0, 0, 0xFFFFFFF0, 100, 0, ctypes.c_void_p(st.data_ptr()),
                                   st.numel() * 4, None, None)
    assert rc == xy.XY_ERANGE
