"""Host-side checks of the C-ABI library that need no GPU: it loads, exports every
function include/xy.h declares, sizes buffers as documented, and rejects bad
arguments with the documented codes before touching the device."""
from __future__ import annotations

import ctypes
import json
import os
import subprocess

import pytest

from paper_0811_2111_amd import xy

L_ = xy.lib()
vp = ctypes.c_void_p


def test_every_declared_function_is_exported():
    declared = xy.header_functions()
    assert len(declared) >= 20
    out = subprocess.run(["nm", "-D", "--defined-only", xy.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [f for f in declared if f not in exported]
    assert not missing, missing


def test_library_carries_gfx950_code_object():
    with open(xy.LIB_PATH, "rb") as f:
        blob = f.read()
    assert b"amdgcn-amd-amdhsa--gfx950" in blob


@pytest.mark.parametrize("L,prec,elem", [(4, 0, 4), (32, 0, 4), (4096, 0, 4), (16384, 0, 4), (8192, 1, 2),
                                         (6, 0, 4), (130, 1, 2)])
def test_state_bytes(L, prec, elem):
    s, w = xy.xy_state_bytes(L, prec)
    assert s == L * L * elem
    assert w >= s + 256 + 4096 * 64          # ping-pong copy, counters, reduction partials


@pytest.mark.parametrize("L", [3, 5, 2, 0, -4, 46342 + 1, 1 << 16])
def test_state_bytes_rejects_bad_L(L):
    s = ctypes.c_size_t()
    assert L_.xy_state_bytes(L, 0, ctypes.byref(s), None) == xy.XY_EINVAL


def test_state_bytes_rejects_bad_precision():
    assert L_.xy_state_bytes(32, 7, None, None) == xy.XY_EINVAL


def _init(L=32, beta=1.0, delta=1.0, start=0, prec=0, state=1, slen=None, work=1, wlen=None):
    s, w = xy.xy_state_bytes(32, 0)
    slen = s if slen is None else slen
    wlen = w if wlen is None else wlen
    h = vp()
    rc = L_.xy_init(ctypes.byref(h), 1, L, beta, delta, start, prec, vp(state) if state else None, slen,
                    vp(work) if work else None, wlen, None)
    return rc, h


@pytest.mark.parametrize("kw,code", [
    (dict(L=31), xy.XY_EINVAL), (dict(L=2), xy.XY_EINVAL), (dict(beta=-0.1), xy.XY_EINVAL),
    (dict(beta=float("nan")), xy.XY_EINVAL), (dict(beta=float("inf")), xy.XY_EINVAL),
    (dict(delta=0.0), xy.XY_EINVAL), (dict(delta=3.2), xy.XY_EINVAL), (dict(delta=float("nan")), xy.XY_EINVAL),
    (dict(start=5), xy.XY_EINVAL), (dict(prec=3), xy.XY_EINVAL),
    (dict(slen=100), xy.XY_ESIZE), (dict(wlen=100), xy.XY_ESIZE),
    (dict(state=0), xy.XY_ESTATE), (dict(work=0), xy.XY_ESTATE),
])
def test_init_validation_codes(kw, code):
    rc, h = _init(**kw)
    assert rc == code
    assert not h.value


def test_null_handles():
    obs = vp(1)
    assert L_.xy_sweep(None, 1, 0, None) == xy.XY_ESTATE
    assert L_.xy_measure(None, obs) == xy.XY_ESTATE
    assert L_.xy_free(None) == xy.XY_ESTATE
    assert L_.xy_set_params(None, 1.0, 1.0) == xy.XY_ESTATE
    assert L_.xy_set_sweep(None, 3) == xy.XY_ESTATE
    assert L_.xy_debug_sweep(None, None, None) == xy.XY_ESTATE
    assert L_.xy_batch_sweep(None, 1, 0, None) == xy.XY_ESTATE
    assert L_.xy_batch_free(None) == xy.XY_ESTATE
    assert L_.xy_init(None, 1, 32, 1.0, 1.0, 0, 0, vp(1), 1 << 30, vp(1), 1 << 30, None) == xy.XY_ESTATE


def test_batch_validation_codes():
    Ls = (ctypes.c_int32 * 3)(64, 128, 66)                      # 66 % 4 != 0
    assert L_.xy_batch_state_bytes(3, Ls, 0, None, None) == xy.XY_EINVAL
    Ls = (ctypes.c_int32 * 2)(64, 128)
    assert L_.xy_batch_state_bytes(0, Ls, 0, None, None) == xy.XY_EINVAL
    assert L_.xy_batch_state_bytes(2, Ls, 9, None, None) == xy.XY_EINVAL
    s, w = ctypes.c_size_t(), ctypes.c_size_t()
    assert L_.xy_batch_state_bytes(2, Ls, 0, ctypes.byref(s), ctypes.byref(w)) == 0
    assert s.value == (64 * 64 + 128 * 128) * 4
    assert w.value >= s.value
    seeds = (ctypes.c_uint64 * 2)(1, 2)
    b = (ctypes.c_double * 2)(1.0, -1.0)
    d = (ctypes.c_double * 2)(1.0, 1.0)
    h = vp()
    assert L_.xy_batch_init(ctypes.byref(h), 2, seeds, Ls, b, d, 0, 0, vp(1), s.value, vp(1), w.value,
                            None) == xy.XY_EINVAL
    b = (ctypes.c_double * 2)(1.0, 1.0)
    assert L_.xy_batch_init(ctypes.byref(h), 2, seeds, Ls, b, d, 0, 0, vp(1), s.value - 4, vp(1), w.value,
                            None) == xy.XY_ESIZE


def test_strerror_covers_codes():
    for c in [0, -1, -2, -3, -4, -5, -6, -7, -8]:
        assert L_.xy_strerror(c)
    assert L_.xy_strerror(-99) == b"unknown error"


def test_tuned_plan_cache_parsing(tmp_path):
    p = tmp_path / "tune.json"
    p.write_text('{\n  "gfx950/4096/0": {"kind": 2, "tile_x": 128, "tile_y": 32, "sweeps_per_pass": 1, '
                 '"gupd_s": 300.0},\n  "gfx950/64/1": {"kind": 1, "tile_x": 0, "tile_y": 0, '
                 '"sweeps_per_pass": 1, "gupd_s": 1.0},\n  "gfx950/256/0": {"kind": 2, "tile_x": 96, '
                 '"tile_y": 32, "sweeps_per_pass": 1, "gupd_s": 1.0}\n}\n')
    json.loads(p.read_text())
    plan = xy.xy_plan()
    assert L_.xy_tuned_plan(str(p).encode(), 4096, 0, ctypes.byref(plan)) == 0
    assert plan.as_tuple() == (2, 128, 32, 1)
    assert L_.xy_tuned_plan(str(p).encode(), 64, 1, ctypes.byref(plan)) == 0
    assert plan.as_tuple() == (1, 0, 0, 1)
    # an entry naming an unsupported tile is refused
    assert L_.xy_tuned_plan(str(p).encode(), 256, 0, ctypes.byref(plan)) == xy.XY_EINVAL
    assert L_.xy_tuned_plan(str(p).encode(), 512, 0, ctypes.byref(plan)) == xy.XY_EINVAL
    assert L_.xy_tuned_plan(str(tmp_path / "missing.json").encode(), 64, 1, ctypes.byref(plan)) == xy.XY_EINVAL


def test_init_without_gpu_reports_hip_error():
    """On a machine without a GPU a valid xy_init returns XY_EHIP (no crash, no handle)."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    rc, h = _init()
    assert rc == xy.XY_EHIP
    assert not h.value
    assert L_.xy_last_hip_error()


@pytest.mark.parametrize("L", [4, 32, 130, 4096])
def test_hmc_work_bytes(L):
    b = xy.xy_hmc_work_bytes(L)
    assert b == 256 + 12 * L * L + 2 * (65536 + 256) * 64   # flag, 2 momenta + saved angles, records + chunk sums


def test_hmc_validation_without_gpu():
    L_ = xy.lib()
    s = ctypes.c_size_t()
    assert L_.xy_hmc_work_bytes(5, ctypes.byref(s)) == xy.XY_EINVAL
    assert L_.xy_hmc(None, 1, 1, 0.1, None, 0, None) == xy.XY_ESTATE


def test_injected_failure_reported_before_any_device_work():
    """An armed injected failure makes the next launch point fail with XY_EHIP and
    a message that names the injection; nothing reaches the HIP runtime, so this
    holds with or without a GPU.  The hook then disarms itself."""
    assert L_.xy_test_inject_failure(-2) == xy.XY_EINVAL
    assert L_.xy_test_inject_failure(0) == xy.XY_OK
    rc, h = _init()
    assert rc == xy.XY_EHIP
    assert not h.value
    assert L_.xy_last_hip_error().endswith(b"[injected]")
    assert L_.xy_test_inject_failure(-1) == xy.XY_OK


def test_strerror_io_code():
    assert L_.xy_strerror(xy.XY_EIO) == b"file could not be written"


def test_tuned_plan_cache_survives_malformed_files(tmp_path):
    """The tune-cache parser on hostile input: lines longer than its read buffer,
    truncated fields, binary junk, an empty file.  Lookups fail cleanly (run
    under the sanitizers too, tests/test_sanitizers.py)."""
    plan = xy.xy_plan()
    cases = {
        "long.json": '{\n  "gfx950/64/0": {"kind": 2' + " " * 5000 + ', "tile_x": 64}\n}\n',
        "trunc.json": '{\n  "gfx950/64/0": {"kind":',
        "junk.json": "\x00\xff\x01gfx950/64/0\"kind\":\n" * 50,
        "empty.json": "",
        "neg.json": '{"gfx950/64/0": {"kind": -7, "tile_x": -1, "tile_y": 99999999999, "sweeps_per_pass": 0}}\n',
    }
    for name, text in cases.items():
        p = tmp_path / name
        p.write_bytes(text.encode("latin-1"))
        rc = L_.xy_tuned_plan(str(p).encode(), 64, 0, ctypes.byref(plan))
        assert rc in (xy.XY_OK, xy.XY_EINVAL), name
        if rc == xy.XY_OK:   # whatever was parsed must be a plan the library accepts
            assert plan.kind in (1, 2, 3, 4), name


@pytest.mark.parametrize("L", [32, 96, 4096])
def test_quad_hmc_work_bytes_and_null_handles(L):
    """Workspace of the four-replica HMC: three float4 state-sized buffers (two
    momenta, saved angles; each rounded to 256 bytes), the flags, and per replica
    the partial records of H_old and H_new with their chunk sums; bad L and NULL
    handles are refused without device work."""
    L_ = xy.lib()
    s = ctypes.c_size_t()
    assert L_.xy_quad_hmc_work_bytes(L, ctypes.byref(s)) == xy.XY_OK
    st = (16 * L * L + 255) // 256 * 256
    cols = 2 * ((L // 2 + 255) // 256)
    rb = min(L, max(1, 4096 // cols))
    nrec = cols * rb * 4
    assert s.value == 3 * st + 256 + 2 * 4 * (nrec + (nrec + 255) // 256) * 64
    assert L_.xy_quad_hmc_work_bytes(L + 16, ctypes.byref(s)) == xy.XY_EINVAL   # L % 32 != 0
    assert L_.xy_quad_hmc_work_bytes(L, None) == xy.XY_ESTATE
    assert L_.xy_quad_hmc(None, 1, 1, 0.1, None, 0, None) == xy.XY_ESTATE
    assert L_.xy_quad_hmc_set_steps_per_pass(None, 2) == xy.XY_ESTATE
    v = ctypes.c_int32()
    assert L_.xy_quad_hmc_get_steps_per_pass(None, ctypes.byref(v)) == xy.XY_ESTATE
