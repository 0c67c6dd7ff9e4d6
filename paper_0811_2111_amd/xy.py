"""Python binding of the C ABI in include/xy.h (argument marshalling only).

Every function of the C ABI is exposed under the same name with ctypes; every
step of a sweep runs in the HIP library ``libxyhip.so``.  PyTorch supplies the
device memory (torch tensors) and the stream (the current torch stream).  There
is no CPU fallback: if the library is missing, importing this module raises.

    from paper_0811_2111_amd import xy
    lat = xy.Lattice(L=4096, seed=1, beta=1.12, delta=1.0)
    obs = lat.sweep(1000, measure_every=10)      # device tensor of xy_obs records
    rec = xy.records(obs)                          # host numpy structured array
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libxyhip.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "xy.h")

XY_OK, XY_EINVAL, XY_ESIZE, XY_ERANGE, XY_EHIP, XY_ESTATE, XY_ENOMEM, XY_EBARRIER, XY_EIO = \
    0, -1, -2, -3, -4, -5, -6, -7, -8
XY_FP32, XY_FP16 = 0, 1
XY_HOT, XY_COLD = 0, 1
XY_PLAN_AUTO, XY_PLAN_STREAM, XY_PLAN_FUSED, XY_PLAN_STRIP, XY_PLAN_RESIDENT = 0, 1, 2, 3, 4
XY_BATCH_PERSISTENT, XY_BATCH_PASSES, XY_BATCH_PASSES_WIDE = 0, 1, 2
_PREC = {"fp32": XY_FP32, "fp16": XY_FP16, XY_FP32: XY_FP32, XY_FP16: XY_FP16}
_START = {"hot": XY_HOT, "cold": XY_COLD, XY_HOT: XY_HOT, XY_COLD: XY_COLD}


class xy_obs(ctypes.Structure):
    _fields_ = [("sweep", ctypes.c_uint64), ("n_accept", ctypes.c_uint64),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double), ("ix", ctypes.c_double),
                ("iy", ctypes.c_double), ("mx", ctypes.c_double), ("my", ctypes.c_double)]


class xy_plan(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32),
                ("sweeps_per_pass", ctypes.c_int32)]

    def as_tuple(self):
        return (self.kind, self.tile_x, self.tile_y, self.sweeps_per_pass)


OBS_DTYPE = np.dtype([("sweep", "<u8"), ("n_accept", "<u8"), ("cx", "<f8"), ("cy", "<f8"),
                      ("ix", "<f8"), ("iy", "<f8"), ("mx", "<f8"), ("my", "<f8")])
HMC_DTYPE = np.dtype([("traj", "<u8"), ("accepted", "<u8"), ("dH", "<f8"), ("cx", "<f8"), ("cy", "<f8"),
                      ("ix", "<f8"), ("iy", "<f8"), ("mx", "<f8"), ("my", "<f8")])


class XYError(RuntimeError):
    def __init__(self, code: int, what: str):
        msg = "%s failed: %s (%d)" % (what, _lib.xy_strerror(code).decode(), code)
        if code == XY_EHIP:
            msg += " [%s]" % _lib.xy_last_hip_error().decode()
        super().__init__(msg)
        self.code = code


def _load():
    global LIB_PATH
    # XY_LIB names another build of the same sources (the sanitizer test's host-only build)
    LIB_PATH = os.environ.get("XY_LIB") or LIB_PATH
    if not os.path.exists(LIB_PATH):
        raise ImportError("libxyhip.so is not built (%s); run python -m paper_0811_2111_amd.build" % LIB_PATH)
    # torch first: its bundled HIP runtime carries the soname libamdhip64.so.7, so
    # the library's dependency then resolves to that same runtime.  Loaded the
    # other way round, torch would bring a second HIP runtime into the process,
    # and the library's one would see no device.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    vp, sz, i32, i64, u64, dbl = (ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64,
                                  ctypes.c_uint64, ctypes.c_double)
    P = ctypes.POINTER
    sig = {
        "xy_state_bytes": [i32, i32, P(sz), P(sz)],
        "xy_init": [P(vp), u64, i32, dbl, dbl, i32, i32, vp, sz, vp, sz, vp],
        "xy_attach": [P(vp), u64, i32, dbl, dbl, i32, u64, vp, sz, vp, sz, vp],
        "xy_sweep": [vp, i64, i32, vp],
        "xy_measure": [vp, vp],
        "xy_set_params": [vp, dbl, dbl],
        "xy_get_sweep": [vp, P(u64)],
        "xy_set_sweep": [vp, u64],
        "xy_set_stream": [vp, vp],
        "xy_set_plan": [vp, P(xy_plan)],
        "xy_get_plan": [vp, P(xy_plan)],
        "xy_free": [vp],
        "xy_debug_sweep": [vp, vp, vp],
        "xy_autotune": [vp, i32, ctypes.c_char_p, P(xy_plan)],
        "xy_tuned_plan": [ctypes.c_char_p, i32, i32, P(xy_plan)],
        "xy_batch_state_bytes": [i32, P(i32), i32, P(sz), P(sz)],
        "xy_batch_init": [P(vp), i32, P(u64), P(i32), P(dbl), P(dbl), i32, i32, vp, sz, vp, sz, vp],
        "xy_batch_sweep": [vp, i64, i32, vp],
        "xy_batch_get_sweep": [vp, P(u64)],
        "xy_batch_set_tile": [vp, i32, i32],
        "xy_batch_get_tile": [vp, P(i32), P(i32)],
        "xy_batch_autotune": [vp, i32, P(i32), P(i32)],
        "xy_batch_set_schedule": [vp, i32],
        "xy_hmc_set_steps_per_pass": [vp, i32],
        "xy_hmc_get_steps_per_pass": [vp, P(i32)],
        "xy_batch_get_schedule": [vp, P(i32)],
        "xy_batch_status": [vp],
        "xy_batch_free": [vp],
        "xy_hmc_work_bytes": [i32, P(sz)],
        "xy_batch_tempering": [vp, i64, i32, u64, vp, vp],
        "xy_batch_get_params": [vp, P(dbl), P(dbl)],
        "xy_quad_state_bytes": [i32, P(sz), P(sz)],
        "xy_quad_init": [P(vp), P(u64), i32, P(dbl), P(dbl), i32, vp, sz, vp, sz, vp],
        "xy_quad_sweep": [vp, i64, i32, vp],
        "xy_quad_set_params": [vp, P(dbl), P(dbl)],
        "xy_quad_get_sweep": [vp, P(u64)],
        "xy_quad_set_sweep": [vp, u64],
        "xy_quad_set_tile": [vp, i32, i32],
        "xy_quad_get_tile": [vp, P(i32), P(i32)],
        "xy_quad_free": [vp],
        "xy_hmc": [vp, i64, i32, dbl, vp, sz, vp],
        "xy_quad_hmc_work_bytes": [i32, P(sz)],
        "xy_quad_hmc": [vp, i64, i32, dbl, vp, sz, vp],
        "xy_quad_hmc_set_steps_per_pass": [vp, i32],
        "xy_quad_hmc_get_steps_per_pass": [vp, P(i32)],
        "xy_batch_set_spin_limit": [vp, ctypes.c_uint32],
        "xy_test_inject_failure": [i32],
        "xy_sweep_noalloc": [u64, i32, dbl, dbl, i32, u64, i64, i32, vp, sz, vp, vp],
        "xy_kernel_timer": [vp, i32],
        "xy_batch_hmc_work_bytes": [vp, P(sz)],
        "xy_batch_hmc": [vp, i64, i32, dbl, vp, sz, vp],
        "xy_batch_hmc_set_steps_per_pass": [vp, i32],
        "xy_kernel_timer_read": [vp, P(dbl), P(i64)],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.xy_strerror.argtypes = [ctypes.c_int]
    lib.xy_strerror.restype = ctypes.c_char_p
    lib.xy_last_hip_error.argtypes = []
    lib.xy_last_hip_error.restype = ctypes.c_char_p
    return lib


_lib = _load()


def lib():
    return _lib


def header_functions():
    """Names of the functions include/xy.h declares."""
    with open(HEADER) as f:
        text = f.read()
    return sorted(set(re.findall(r"^(?:int|const char\*)\s+(xy_\w+)\s*\(", text, flags=re.M)))


def xy_sweep_noalloc(seed: int, L: int, beta: float, delta: float, precision, sweep: int, n_sweeps: int,
                     measure_every: int, state, out=None, stream=None):
    """Allocation-free sweeps of the angles in `state` (a contiguous (2, L, L/2)
    device tensor), starting at sweep counter `sweep`; the library's fixed device
    array serves as the workspace.  `out`: None, or a float64 device tensor for the
    records (allocated here if None and records are asked for -- pass one to keep
    the call allocation-free)."""
    import torch
    prec = _PREC[precision]
    nrec = n_sweeps // measure_every if measure_every > 0 else 0
    if nrec and out is None:
        out = torch.empty((nrec, 8), dtype=torch.float64, device=state.device)
    if nrec:
        _check_out(out, nrec * 64, state.device, "xy_sweep_noalloc")
    if not state.is_contiguous():
        raise ValueError("xy_sweep_noalloc: state must be contiguous")
    check(_lib.xy_sweep_noalloc(int(seed), int(L), float(beta), float(delta), prec, int(sweep), int(n_sweeps),
                                int(measure_every), _ptr(state), _nbytes(state), _ptr(out) if nrec else None,
                                _stream_handle(stream)), "xy_sweep_noalloc")
    return out


def xy_test_inject_failure(after: int):
    """Test support: the (after + 1)-th launch point from now fails with XY_EHIP."""
    check(_lib.xy_test_inject_failure(int(after)), "xy_test_inject_failure")


def check(rc: int, what: str):
    if rc != XY_OK:
        raise XYError(rc, what)


# ------------------------------------------------------------- thin wrappers

def xy_state_bytes(L: int, precision=XY_FP32):
    s, w = ctypes.c_size_t(), ctypes.c_size_t()
    check(_lib.xy_state_bytes(L, _PREC[precision], ctypes.byref(s), ctypes.byref(w)), "xy_state_bytes")
    return s.value, w.value


def xy_batch_state_bytes(Ls, precision=XY_FP32):
    arr = (ctypes.c_int32 * len(Ls))(*Ls)
    s, w = ctypes.c_size_t(), ctypes.c_size_t()
    check(_lib.xy_batch_state_bytes(len(Ls), arr, _PREC[precision], ctypes.byref(s), ctypes.byref(w)),
          "xy_batch_state_bytes")
    return s.value, w.value


def records(obs) -> np.ndarray:
    """Copy a device tensor of xy_obs records to a host structured array."""
    import torch
    host = obs.detach().to("cpu").contiguous()
    return host.numpy().view(np.uint8).view(OBS_DTYPE).reshape(host.shape[:-1])


def hmc_records(obs) -> np.ndarray:
    """Copy a device tensor of xy_hmc_obs records (n, 9) to a host structured array."""
    host = obs.detach().to("cpu").contiguous()
    return host.numpy().view(np.uint8).view(HMC_DTYPE).reshape(host.shape[:-1])


def xy_hmc_work_bytes(L: int) -> int:
    b = ctypes.c_size_t()
    check(_lib.xy_hmc_work_bytes(L, ctypes.byref(b)), "xy_hmc_work_bytes")
    return b.value


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _nbytes(t):
    return t.numel() * t.element_size()


def _check_out(out, nbytes: int, device, what: str, dtype=None):
    """The C ABI writes `nbytes` of records through `out` with no length argument:
    refuse a tensor that is not a contiguous float64 device tensor of at least that
    size on the lattice's device, before any device write can run past its end."""
    import torch
    dtype = dtype or torch.float64
    if out.dtype != dtype or not out.is_contiguous() or out.device != torch.device(device):
        raise ValueError("%s: out must be a contiguous %s tensor on %s (got %s, %s, contiguous=%s)"
                         % (what, dtype, device, out.dtype, out.device, out.is_contiguous()))
    if _nbytes(out) < nbytes:
        raise ValueError("%s: out holds %d bytes, the call writes %d" % (what, _nbytes(out), nbytes))


class Lattice:
    """One L x L lattice: angles and workspace in torch device tensors, sweeps in HIP.

    ``state`` holds the angles in turns, phi = theta / (2 pi) in [0, 1], in the
    half-lattice layout (2, L, L/2); ``delta`` is the proposal width in radians."""

    def __init__(self, L: int, seed: int = 1, beta: float = 1.0, delta: float = 1.0, start="hot",
                 precision="fp32", device="cuda", stream=None, plan=None, state=None, sweep=None):
        import torch
        self.L, self.seed, self.beta, self.delta = int(L), int(seed), float(beta), float(delta)
        self.precision = _PREC[precision]
        sbytes, wbytes = xy_state_bytes(self.L, self.precision)
        dt = torch.float16 if self.precision == XY_FP16 else torch.float32
        if state is None:
            self.state = torch.empty((2, self.L, self.L // 2), dtype=dt, device=device)
        else:
            assert state.dtype == dt and state.is_contiguous() and _nbytes(state) >= sbytes
            self.state = state
        self.work = torch.empty((wbytes,), dtype=torch.uint8, device=device)
        self.stream = stream
        h = ctypes.c_void_p()
        if state is None:
            rc = _lib.xy_init(ctypes.byref(h), self.seed, self.L, self.beta, self.delta, _START[start],
                              self.precision, _ptr(self.state), _nbytes(self.state), _ptr(self.work),
                              _nbytes(self.work), _stream_handle(stream))
            check(rc, "xy_init")
        else:
            rc = _lib.xy_attach(ctypes.byref(h), self.seed, self.L, self.beta, self.delta, self.precision,
                                int(sweep or 0), _ptr(self.state), _nbytes(self.state), _ptr(self.work),
                                _nbytes(self.work), _stream_handle(stream))
            check(rc, "xy_attach")
        self.h = h
        if plan is not None:
            self.set_plan(*plan)

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value and _lib is not None:   # _lib is None at interpreter shutdown
            _lib.xy_free(h)
            self.h = None

    def sweep(self, n: int, measure_every: int = 0, out=None):
        import torch
        nrec = n // measure_every if measure_every > 0 else 0
        if nrec and out is None:
            out = torch.empty((nrec, 8), dtype=torch.float64, device=self.state.device)
        if nrec:
            _check_out(out, nrec * 64, self.state.device, "xy_sweep")
        rc = _lib.xy_sweep(self.h, int(n), int(measure_every), _ptr(out) if nrec else None)
        check(rc, "xy_sweep")
        return out

    @property
    def hmc_steps_per_pass(self) -> int:
        """Leap-frog steps per pass that xy_hmc runs (1 if L % 32 != 0)."""
        v = ctypes.c_int32()
        check(_lib.xy_hmc_get_steps_per_pass(self.h, ctypes.byref(v)), "xy_hmc_get_steps_per_pass")
        return v.value

    def set_hmc_steps_per_pass(self, steps: int):
        check(_lib.xy_hmc_set_steps_per_pass(self.h, int(steps)), "xy_hmc_set_steps_per_pass")

    def hmc(self, n_traj: int, n_md: int, eps: float, out=None):
        """n_traj HMC trajectories of n_md leap-frog steps of size eps; returns a
        device tensor (n_traj, 9) of xy_hmc_obs records (see hmc_records)."""
        import torch
        if getattr(self, "hmc_work", None) is None:
            self.hmc_work = torch.empty((xy_hmc_work_bytes(self.L),), dtype=torch.uint8, device=self.state.device)
        if out is None:
            out = torch.empty((max(int(n_traj), 1), 9), dtype=torch.float64, device=self.state.device)
        if n_traj > 0:
            _check_out(out, int(n_traj) * 72, self.state.device, "xy_hmc")
        rc = _lib.xy_hmc(self.h, int(n_traj), int(n_md), float(eps), _ptr(self.hmc_work), _nbytes(self.hmc_work),
                         _ptr(out) if n_traj > 0 else None)
        check(rc, "xy_hmc")
        return out[: int(n_traj)]

    def measure(self, out=None):
        import torch
        if out is None:
            out = torch.empty((1, 8), dtype=torch.float64, device=self.state.device)
        _check_out(out, 64, self.state.device, "xy_measure")
        check(_lib.xy_measure(self.h, _ptr(out)), "xy_measure")
        return out

    def debug_sweep(self):
        import torch
        acc = torch.empty((2, self.L, self.L // 2), dtype=torch.uint8, device=self.state.device)
        dE = torch.empty((2, self.L, self.L // 2), dtype=torch.float32, device=self.state.device)
        check(_lib.xy_debug_sweep(self.h, _ptr(acc), _ptr(dE)), "xy_debug_sweep")
        return acc, dE

    def set_params(self, beta: float, delta: float):
        check(_lib.xy_set_params(self.h, float(beta), float(delta)), "xy_set_params")
        self.beta, self.delta = float(beta), float(delta)

    @property
    def sweep_count(self) -> int:
        v = ctypes.c_uint64()
        check(_lib.xy_get_sweep(self.h, ctypes.byref(v)), "xy_get_sweep")
        return v.value

    def set_sweep(self, s: int):
        check(_lib.xy_set_sweep(self.h, int(s)), "xy_set_sweep")

    def set_plan(self, kind, tile_x=0, tile_y=0, sweeps_per_pass=1):
        p = xy_plan(kind, tile_x, tile_y, sweeps_per_pass)
        check(_lib.xy_set_plan(self.h, ctypes.byref(p)), "xy_set_plan")

    @property
    def plan(self):
        p = xy_plan()
        check(_lib.xy_get_plan(self.h, ctypes.byref(p)), "xy_get_plan")
        return p.as_tuple()

    def kernel_timer(self, capacity: int):
        """Time the next `capacity` tiled sweep launches with HIP events (0: off)."""
        check(_lib.xy_kernel_timer(self.h, int(capacity)), "xy_kernel_timer")

    def kernel_timer_read(self):
        """(total ms, launches) of the launches timed since the last read."""
        t, n = ctypes.c_double(), ctypes.c_int64()
        check(_lib.xy_kernel_timer_read(self.h, ctypes.byref(t), ctypes.byref(n)), "xy_kernel_timer_read")
        return t.value, n.value

    def autotune(self, sweeps_per_trial: int = 4, cache_path=None):
        p = xy_plan()
        cp = cache_path.encode() if cache_path else None
        check(_lib.xy_autotune(self.h, int(sweeps_per_trial), cp, ctypes.byref(p)), "xy_autotune")
        return p.as_tuple()


class Batch:
    """Many lattices (uneven L, own seed/beta/delta) advanced by one persistent launch per call."""

    def __init__(self, Ls, seeds, betas, deltas, start="hot", precision="fp32", device="cuda", stream=None):
        import torch
        n = len(Ls)
        assert len(seeds) == n and len(betas) == n and len(deltas) == n
        self.Ls = [int(v) for v in Ls]
        self.precision = _PREC[precision]
        sbytes, wbytes = xy_batch_state_bytes(self.Ls, self.precision)
        dt = torch.float16 if self.precision == XY_FP16 else torch.float32
        self.offsets = np.concatenate([[0], np.cumsum([L * L for L in self.Ls])]).astype(np.int64)
        self.state = torch.empty((int(self.offsets[-1]),), dtype=dt, device=device)
        self.work = torch.empty((wbytes,), dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        rc = _lib.xy_batch_init(ctypes.byref(h), n, (ctypes.c_uint64 * n)(*[int(s) for s in seeds]),
                                (ctypes.c_int32 * n)(*self.Ls), (ctypes.c_double * n)(*[float(b) for b in betas]),
                                (ctypes.c_double * n)(*[float(d) for d in deltas]), _START[start], self.precision,
                                _ptr(self.state), _nbytes(self.state), _ptr(self.work), _nbytes(self.work),
                                _stream_handle(stream))
        check(rc, "xy_batch_init")
        self.h = h

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value and _lib is not None:   # _lib is None at interpreter shutdown
            _lib.xy_batch_free(h)
            self.h = None

    def tempering(self, n_rounds: int, sweeps_per_round: int, pt_seed: int, out=None, rungs=None):
        """n_rounds parallel-tempering rounds; returns device tensors (records
        (n_rounds, n, 8) of xy_obs, rungs (n_rounds, n) int32)."""
        import torch
        n = len(self.Ls)
        if out is None:
            out = torch.empty((max(int(n_rounds), 1), n, 8), dtype=torch.float64, device=self.state.device)
        if rungs is None:
            rungs = torch.empty((max(int(n_rounds), 1), n), dtype=torch.int32, device=self.state.device)
        if n_rounds > 0:
            _check_out(out, int(n_rounds) * n * 64, self.state.device, "xy_batch_tempering")
            _check_out(rungs, int(n_rounds) * n * 4, self.state.device, "xy_batch_tempering", torch.int32)
        check(_lib.xy_batch_tempering(self.h, int(n_rounds), int(sweeps_per_round), int(pt_seed), _ptr(out),
                                      _ptr(rungs)), "xy_batch_tempering")
        return out[: int(n_rounds)], rungs[: int(n_rounds)]

    def hmc(self, n_traj: int, n_md: int, eps: float, out=None):
        """n_traj HMC trajectories of every lattice (one accept per lattice); returns
        a device tensor (n, n_traj, 9) of xy_hmc_obs records (see hmc_records)."""
        import torch
        n = len(self.Ls)
        if getattr(self, "hmc_work", None) is None:
            b = ctypes.c_size_t()
            check(_lib.xy_batch_hmc_work_bytes(self.h, ctypes.byref(b)), "xy_batch_hmc_work_bytes")
            self.hmc_work = torch.empty((b.value,), dtype=torch.uint8, device=self.state.device)
        if out is None:
            out = torch.empty((n, max(int(n_traj), 1), 9), dtype=torch.float64, device=self.state.device)
        if n_traj > 0:
            _check_out(out, n * int(n_traj) * 72, self.state.device, "xy_batch_hmc")
        check(_lib.xy_batch_hmc(self.h, int(n_traj), int(n_md), float(eps), _ptr(self.hmc_work),
                                _nbytes(self.hmc_work), _ptr(out) if n_traj > 0 else None), "xy_batch_hmc")
        return out[:, : int(n_traj)] if out.dim() == 3 else out

    def set_hmc_steps_per_pass(self, steps: int):
        check(_lib.xy_batch_hmc_set_steps_per_pass(self.h, int(steps)), "xy_batch_hmc_set_steps_per_pass")

    def params(self):
        n = len(self.Ls)
        b, d = (ctypes.c_double * n)(), (ctypes.c_double * n)()
        check(_lib.xy_batch_get_params(self.h, b, d), "xy_batch_get_params")
        return list(b), list(d)

    def lattice_state(self, i: int):
        L = self.Ls[i]
        return self.state[self.offsets[i]:self.offsets[i + 1]].view(2, L, L // 2)

    def sweep(self, n: int, measure_every: int = 0, out=None):
        import torch
        nrec = n // measure_every if measure_every > 0 else 0
        if nrec and out is None:
            out = torch.empty((len(self.Ls), nrec, 8), dtype=torch.float64, device=self.state.device)
        if nrec:
            _check_out(out, len(self.Ls) * nrec * 64, self.state.device, "xy_batch_sweep")
        check(_lib.xy_batch_sweep(self.h, int(n), int(measure_every), _ptr(out) if nrec else None),
              "xy_batch_sweep")
        return out

    @property
    def sweep_count(self) -> int:
        v = ctypes.c_uint64()
        check(_lib.xy_batch_get_sweep(self.h, ctypes.byref(v)), "xy_batch_get_sweep")
        return v.value

    def status(self):
        """Synchronise and raise if any persistent launch hit a barrier spin limit."""
        check(_lib.xy_batch_status(self.h), "xy_batch_status")

    def set_spin_limit(self, polls: int):
        """Test support: polls before a persistent barrier wait gives up."""
        check(_lib.xy_batch_set_spin_limit(self.h, int(polls)), "xy_batch_set_spin_limit")

    @property
    def tile(self):
        tx, ty = ctypes.c_int32(), ctypes.c_int32()
        check(_lib.xy_batch_get_tile(self.h, ctypes.byref(tx), ctypes.byref(ty)), "xy_batch_get_tile")
        return tx.value, ty.value

    def set_tile(self, tile_x: int, tile_y: int):
        check(_lib.xy_batch_set_tile(self.h, int(tile_x), int(tile_y)), "xy_batch_set_tile")

    def autotune(self, sweeps_per_trial: int = 4):
        """Pick the fastest tile shape and schedule; returns the shape."""
        tx, ty = ctypes.c_int32(), ctypes.c_int32()
        check(_lib.xy_batch_autotune(self.h, int(sweeps_per_trial), ctypes.byref(tx), ctypes.byref(ty)),
              "xy_batch_autotune")
        return tx.value, ty.value

    @property
    def schedule(self) -> int:
        v = ctypes.c_int32()
        check(_lib.xy_batch_get_schedule(self.h, ctypes.byref(v)), "xy_batch_get_schedule")
        return v.value

    def set_schedule(self, schedule: int):
        """XY_BATCH_PERSISTENT (one persistent kernel per call), XY_BATCH_PASSES (one launch per
        sweep) or XY_BATCH_PASSES_WIDE (the same with 256 x 16 tiles where L allows)."""
        check(_lib.xy_batch_set_schedule(self.h, int(schedule)), "xy_batch_set_schedule")


class Quad:
    """Four replicas of one L x L lattice in one float4 state (component r = replica r)."""

    def __init__(self, L: int, seeds, betas, deltas=(1.0, 1.0, 1.0, 1.0), start="hot", device="cuda", stream=None):
        import torch
        assert len(seeds) == 4 and len(betas) == 4 and len(deltas) == 4
        self.L = int(L)
        self.seeds, self.betas, self.deltas = [int(v) for v in seeds], [float(v) for v in betas], \
            [float(v) for v in deltas]
        s, w = ctypes.c_size_t(), ctypes.c_size_t()
        check(_lib.xy_quad_state_bytes(self.L, ctypes.byref(s), ctypes.byref(w)), "xy_quad_state_bytes")
        self.state = torch.empty((2, self.L, self.L // 2, 4), dtype=torch.float32, device=device)
        self.work = torch.empty((w.value,), dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        rc = _lib.xy_quad_init(ctypes.byref(h), (ctypes.c_uint64 * 4)(*self.seeds), self.L,
                               (ctypes.c_double * 4)(*self.betas), (ctypes.c_double * 4)(*self.deltas), _START[start],
                               _ptr(self.state), _nbytes(self.state), _ptr(self.work), _nbytes(self.work),
                               _stream_handle(stream))
        check(rc, "xy_quad_init")
        self.h = h

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value and _lib is not None:   # _lib is None at interpreter shutdown
            _lib.xy_quad_free(h)
            self.h = None

    def replica_state(self, r: int):
        """(2, L, L/2) view of replica r's angles (strided)."""
        return self.state[..., r]

    def sweep(self, n: int, measure_every: int = 0, out=None):
        """n sweeps; returns a device tensor (records, 4, 8) of xy_obs, or None."""
        import torch
        nrec = n // measure_every if measure_every > 0 else 0
        if nrec and out is None:
            out = torch.empty((nrec, 4, 8), dtype=torch.float64, device=self.state.device)
        if nrec:
            _check_out(out, nrec * 4 * 64, self.state.device, "xy_quad_sweep")
        check(_lib.xy_quad_sweep(self.h, int(n), int(measure_every), _ptr(out) if nrec else None), "xy_quad_sweep")
        return out

    @property
    def hmc_steps_per_pass(self) -> int:
        v = ctypes.c_int32()
        check(_lib.xy_quad_hmc_get_steps_per_pass(self.h, ctypes.byref(v)), "xy_quad_hmc_get_steps_per_pass")
        return v.value

    def set_hmc_steps_per_pass(self, steps: int):
        check(_lib.xy_quad_hmc_set_steps_per_pass(self.h, int(steps)), "xy_quad_hmc_set_steps_per_pass")

    def hmc(self, n_traj: int, n_md: int, eps: float, out=None):
        """n_traj HMC trajectories of all four replicas (n_md leap-frog steps of size
        eps, one accept decision per replica); returns a device tensor (n_traj, 4, 9)
        of xy_hmc_obs records (see hmc_records)."""
        import torch
        if getattr(self, "hmc_work", None) is None:
            b = ctypes.c_size_t()
            check(_lib.xy_quad_hmc_work_bytes(self.L, ctypes.byref(b)), "xy_quad_hmc_work_bytes")
            self.hmc_work = torch.empty((b.value,), dtype=torch.uint8, device=self.state.device)
        if out is None:
            out = torch.empty((max(int(n_traj), 1), 4, 9), dtype=torch.float64, device=self.state.device)
        if n_traj > 0:
            _check_out(out, int(n_traj) * 4 * 72, self.state.device, "xy_quad_hmc")
        rc = _lib.xy_quad_hmc(self.h, int(n_traj), int(n_md), float(eps), _ptr(self.hmc_work),
                              _nbytes(self.hmc_work), _ptr(out) if n_traj > 0 else None)
        check(rc, "xy_quad_hmc")
        return out[: int(n_traj)]

    def set_params(self, betas, deltas):
        check(_lib.xy_quad_set_params(self.h, (ctypes.c_double * 4)(*betas), (ctypes.c_double * 4)(*deltas)),
              "xy_quad_set_params")
        self.betas, self.deltas = [float(v) for v in betas], [float(v) for v in deltas]

    @property
    def sweep_count(self) -> int:
        v = ctypes.c_uint64()
        check(_lib.xy_quad_get_sweep(self.h, ctypes.byref(v)), "xy_quad_get_sweep")
        return v.value

    def set_sweep(self, s: int):
        check(_lib.xy_quad_set_sweep(self.h, int(s)), "xy_quad_set_sweep")

    def set_tile(self, tx: int, ty: int):
        check(_lib.xy_quad_set_tile(self.h, int(tx), int(ty)), "xy_quad_set_tile")

    @property
    def tile(self):
        a, b = ctypes.c_int32(), ctypes.c_int32()
        check(_lib.xy_quad_get_tile(self.h, ctypes.byref(a), ctypes.byref(b)), "xy_quad_get_tile")
        return a.value, b.value
