"""FP64 CPU oracle for checkerboard Metropolis sweeps of the 2-d XY model.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``; never by the product library.

The arithmetic lives in ``xy_oracle.c`` (plain C, FP64); this module builds it
with gcc when needed and marshals numpy arrays through ctypes.  Every function
follows the definitions stated in that file's header: the XY Hamiltonian of
section 1.2 (eq. 1) with J = 1 and Boltzmann weight exp(-beta H), single-site
Metropolis over the red then the black sublattice, Philox4x32-10 streams.

Angles use the natural layout ``theta[y, x]`` (an ``(L, L)`` float64 array).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "xy_oracle.c")
_SRC_HMC = os.path.join(_HERE, "xy_hmc_oracle.c")
_SRC_PT = os.path.join(_HERE, "xy_pt_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

PREC_F64, PREC_F32, PREC_F16 = 0, 1, 2
_PREC = {"f64": PREC_F64, "f32": PREC_F32, "f16": PREC_F16}


def build(force: bool = False) -> str:
    """Compile ``xy_oracle.c`` into ``liboracle.so`` with gcc (single-threaded)."""
    newest = max(os.path.getmtime(_SRC), os.path.getmtime(_SRC_HMC), os.path.getmtime(_SRC_PT))
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared", "-o", tmp,
                               _SRC, _SRC_HMC, _SRC_PT, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        # XY_ORACLE_LIB names another build of the same sources (the sanitizer test's)
        path = os.environ.get("XY_ORACLE_LIB") or build()
        L = ctypes.CDLL(path)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        dp = ctypes.POINTER(ctypes.c_double)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        i32p = ctypes.POINTER(ctypes.c_int32)
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_philox4x32_10.restype = None
        L.orc_u01.argtypes = [ctypes.c_uint32]
        L.orc_u01.restype = ctypes.c_double
        L.orc_site_words.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_uint32, ctypes.c_uint32, u32p]
        L.orc_site_words.restype = None
        L.orc_round_f16.argtypes = [ctypes.c_double]
        L.orc_round_f16.restype = ctypes.c_double
        L.orc_propose.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int]
        L.orc_propose.restype = ctypes.c_double
        L.orc_hot_start.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int, dp]
        L.orc_hot_start.restype = None
        L.orc_measure.argtypes = [ctypes.c_int, dp, dp]
        L.orc_measure.restype = None
        L.orc_energy.argtypes = [ctypes.c_int, dp]
        L.orc_energy.restype = ctypes.c_double
        L.orc_sweep.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                ctypes.c_uint32, ctypes.c_int, dp, dp, dp, u8p, dp]
        L.orc_sweep.restype = ctypes.c_int64
        L.orc_run.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                              ctypes.c_uint32, ctypes.c_int64, ctypes.c_int64, ctypes.c_int, dp, dp]
        L.orc_run.restype = ctypes.c_int64
        L.orc_clock_sweep.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                      ctypes.c_uint32, i32p]
        L.orc_clock_sweep.restype = ctypes.c_int64
        L.orc_clock_run.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_uint32, ctypes.c_int64, ctypes.c_int64, i32p, dp]
        L.orc_clock_run.restype = ctypes.c_int64
        L.orc_site_update_explicit.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                               ctypes.c_uint32, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                               ctypes.c_double, dp, dp, dp, dp, dp]
        L.orc_site_update_explicit.restype = ctypes.c_int
        L.orc_hot_start_site.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.orc_hot_start_site.restype = ctypes.c_double
        L.orc_hmc_momentum.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint32]
        L.orc_hmc_momentum.restype = ctypes.c_double
        L.orc_hmc_momenta.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32, dp]
        L.orc_hmc_momenta.restype = None
        L.orc_hmc_accept_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint32]
        L.orc_hmc_accept_uniform.restype = ctypes.c_double
        L.orc_hmc_force.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp]
        L.orc_hmc_force.restype = None
        L.orc_hmc_hamiltonian.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp]
        L.orc_hmc_hamiltonian.restype = ctypes.c_double
        L.orc_hmc_leapfrog.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int, dp, dp]
        L.orc_hmc_leapfrog.restype = ctypes.c_int
        L.orc_hmc_trajectory.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_int, ctypes.c_uint32, dp, dp, dp]
        L.orc_hmc_trajectory.restype = ctypes.c_int
        L.orc_hmc_run.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                  ctypes.c_uint32, ctypes.c_int64, ctypes.c_int64, dp, dp]
        L.orc_hmc_run.restype = ctypes.c_int64
        i32p = ctypes.POINTER(ctypes.c_int32)
        L.orc_pt_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32]
        L.orc_pt_uniform.restype = ctypes.c_double
        L.orc_pt_run.argtypes = [ctypes.POINTER(ctypes.c_uint64), ctypes.c_int, ctypes.c_int, dp, dp, i32p,
                                 ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int64,
                                 ctypes.c_int, ctypes.c_int, dp, dp, i32p]
        L.orc_pt_run.restype = ctypes.c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _prec(p) -> int:
    return _PREC[p] if isinstance(p, str) else int(p)


def philox4x32_10(ctr, key) -> np.ndarray:
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def u01(w: int) -> float:
    return lib().orc_u01(int(w) & 0xFFFFFFFF)


def site_words(seed: int, L: int, x: int, y: int, sweep: int, purpose: int):
    w = (ctypes.c_uint32 * 2)()
    lib().orc_site_words(seed, L, x, y, sweep, purpose, w)
    return int(w[0]), int(w[1])


def round_f16(v: float) -> float:
    return lib().orc_round_f16(float(v))


def propose(theta: float, delta: float, u1: float, prec="f64") -> float:
    return lib().orc_propose(float(theta), float(delta), float(u1), _prec(prec))


def hot_start(seed: int, L: int, prec="f64") -> np.ndarray:
    th = np.zeros((L, L), dtype=np.float64)
    lib().orc_hot_start(seed, L, _prec(prec), _dp(th))
    return th


def measure(theta: np.ndarray) -> np.ndarray:
    """FP64 [Cx, Cy, Ix, Iy, Mx, My] of a natural-layout (L, L) state."""
    th = np.ascontiguousarray(theta, dtype=np.float64)
    out = np.zeros(6, dtype=np.float64)
    lib().orc_measure(th.shape[0], _dp(th), _dp(out))
    return out


def energy(theta: np.ndarray) -> float:
    th = np.ascontiguousarray(theta, dtype=np.float64)
    return lib().orc_energy(th.shape[0], _dp(th))


def sweep(seed: int, theta: np.ndarray, beta: float, delta: float, sweep_index: int,
          prec="f64", diagnostics: bool = False):
    """One sweep in place.  Returns the accept count, or with ``diagnostics``
    a dict of per-site dE, threshold T (decision is dE < T), decision and
    proposed angle, all in the natural layout."""
    L = theta.shape[0]
    assert theta.dtype == np.float64 and theta.flags.c_contiguous
    if not diagnostics:
        return lib().orc_sweep(seed, L, beta, delta, sweep_index, _prec(prec), _dp(theta),
                               None, None, None, None)
    dE = np.zeros((L, L)); thr = np.zeros((L, L)); prop = np.zeros((L, L))
    dec = np.zeros((L, L), dtype=np.uint8)
    acc = lib().orc_sweep(seed, L, beta, delta, sweep_index, _prec(prec), _dp(theta),
                          _dp(dE), _dp(thr), dec.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                          _dp(prop))
    return {"accepts": acc, "dE": dE, "thr": thr, "dec": dec.astype(bool), "prop": prop}


def run(seed: int, theta: np.ndarray, beta: float, delta: float, n_sweeps: int,
        measure_every: int = 1, sweep0: int = 0, prec="f64") -> np.ndarray:
    """n_sweeps sweeps in place; returns records (n_rec, 8):
    [sweep count after, accepts, Cx, Cy, Ix, Iy, Mx, My]."""
    L = theta.shape[0]
    assert theta.dtype == np.float64 and theta.flags.c_contiguous
    nrec = n_sweeps // measure_every if measure_every > 0 else 0
    rec = np.zeros((max(nrec, 1), 8), dtype=np.float64)
    got = lib().orc_run(seed, L, beta, delta, sweep0, n_sweeps, measure_every, _prec(prec),
                        _dp(theta), _dp(rec))
    return rec[:got]


def clock_run(seed: int, ks: np.ndarray, q: int, beta: float, n_sweeps: int,
              measure_every: int = 1, sweep0: int = 0) -> np.ndarray:
    L = ks.shape[0]
    assert ks.dtype == np.int32 and ks.flags.c_contiguous
    nrec = n_sweeps // measure_every
    rec = np.zeros((max(nrec, 1), 8), dtype=np.float64)
    got = lib().orc_clock_run(seed, L, q, beta, sweep0, n_sweeps, measure_every,
                              ks.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(rec))
    return rec[:got]


def clock_sweep(seed: int, ks: np.ndarray, q: int, beta: float, sweep_index: int) -> int:
    L = ks.shape[0]
    return lib().orc_clock_sweep(seed, L, q, beta, sweep_index,
                                 ks.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))


def hot_start_site(seed: int, L: int, x: int, y: int, prec="f64") -> float:
    """Hot-start angle of site (x, y), without building the whole lattice."""
    return lib().orc_hot_start_site(seed, L, x, y, _prec(prec))


def site_update(seed: int, L: int, x: int, y: int, sweep_index: int, beta: float, delta: float,
                theta: float, neighbours, prec="f64"):
    """One Metropolis update of site (x, y) from explicit inputs (its angle and its
    four neighbours).  Returns (new angle, accepted, dE, threshold T, proposal)."""
    nb = np.ascontiguousarray(np.asarray(neighbours, dtype=np.float64).reshape(4))
    out = np.zeros(4, dtype=np.float64)
    acc = lib().orc_site_update_explicit(seed, L, x, y, sweep_index, _prec(prec), float(beta), float(delta),
                                         float(theta), _dp(nb), _dp(out[0:]), _dp(out[1:]), _dp(out[2:]),
                                         _dp(out[3:]))
    return float(out[0]), bool(acc), float(out[1]), float(out[2]), float(out[3])


# ------------------------------------------------------------------ HMC
# Hybrid Monte Carlo trajectories (xy_hmc_oracle.c): angles in turns, momenta
# in the natural layout, everything FP64.

def hmc_momenta(seed: int, L: int, traj: int) -> np.ndarray:
    p = np.zeros((L, L), dtype=np.float64)
    lib().orc_hmc_momenta(seed, L, traj, _dp(p))
    return p


def hmc_momentum(seed: int, L: int, x: int, y: int, traj: int) -> float:
    return lib().orc_hmc_momentum(seed, L, x, y, traj)


def hmc_accept_uniform(seed: int, traj: int) -> float:
    return lib().orc_hmc_accept_uniform(seed, traj)


def hmc_force(phi: np.ndarray, beta: float) -> np.ndarray:
    ph = np.ascontiguousarray(phi, dtype=np.float64)
    F = np.zeros_like(ph)
    lib().orc_hmc_force(ph.shape[0], beta, _dp(ph), _dp(F))
    return F


def hmc_hamiltonian(phi: np.ndarray, p: np.ndarray, beta: float) -> float:
    ph = np.ascontiguousarray(phi, dtype=np.float64)
    pp = np.ascontiguousarray(p, dtype=np.float64)
    return lib().orc_hmc_hamiltonian(ph.shape[0], beta, _dp(ph), _dp(pp))


def hmc_leapfrog(phi: np.ndarray, p: np.ndarray, beta: float, eps: float, n: int) -> None:
    """n leap-frog steps in place (both arrays float64, C-contiguous)."""
    assert phi.dtype == np.float64 and p.dtype == np.float64 and phi.flags.c_contiguous and p.flags.c_contiguous
    if lib().orc_hmc_leapfrog(phi.shape[0], beta, eps, n, _dp(phi), _dp(p)) != 0:
        raise MemoryError("orc_hmc_leapfrog")


def hmc_trajectory(seed: int, phi: np.ndarray, beta: float, eps: float, n: int, traj: int):
    """One trajectory in place; returns (accepted, dH, H_old)."""
    assert phi.dtype == np.float64 and phi.flags.c_contiguous
    out = np.zeros(2)
    acc = lib().orc_hmc_trajectory(seed, phi.shape[0], beta, eps, n, traj, _dp(phi), _dp(out[0:]), _dp(out[1:]))
    if acc < 0:
        raise MemoryError("orc_hmc_trajectory")
    return bool(acc), float(out[0]), float(out[1])


def hmc_run(seed: int, phi: np.ndarray, beta: float, eps: float, n: int, n_traj: int,
            measure_every: int = 1, traj0: int = 0) -> np.ndarray:
    """n_traj trajectories in place; records (n_rec, 9):
    [trajectory count after, accepted, dH, Cx, Cy, Ix, Iy, Mx, My]."""
    assert phi.dtype == np.float64 and phi.flags.c_contiguous
    nrec = n_traj // measure_every if measure_every > 0 else 0
    rec = np.zeros((max(nrec, 1), 9), dtype=np.float64)
    got = lib().orc_hmc_run(seed, phi.shape[0], beta, eps, n, traj0, n_traj, measure_every, _dp(phi), _dp(rec))
    if got < 0:
        raise MemoryError("orc_hmc_run")
    return rec[:got]


# ------------------------------------------------------- parallel tempering
# One ladder of M lattices of the same L (xy_pt_oracle.c).

def pt_uniform(pt_seed: int, rnd: int, ladder: int, rung: int) -> float:
    return lib().orc_pt_uniform(pt_seed, rnd, ladder, rung)


def pt_run(seeds, phi: np.ndarray, betas, deltas, member: np.ndarray, pt_seed: int, n_rounds: int, K: int,
           ladder: int = 0, round0: int = 0, sweep0: int = 0, prec="f32"):
    """n_rounds tempering rounds in place.  phi: (M, L, L) float64 (C-contiguous);
    member: int32 (M,) lattice on each rung, updated.  Returns (rec, rung):
    rec (n_rounds, M, 9) = [round, sweep count after, accepts, Cx, Cy, Ix, Iy, Mx, My]
    of each lattice, rung (n_rounds, M) = its rung during the round."""
    M, L = phi.shape[0], phi.shape[1]
    assert phi.dtype == np.float64 and phi.flags.c_contiguous
    assert member.dtype == np.int32 and member.flags.c_contiguous and member.shape == (M,)
    sd = (ctypes.c_uint64 * M)(*[int(v) for v in seeds])
    b = np.ascontiguousarray(betas, dtype=np.float64)
    d = np.ascontiguousarray(deltas, dtype=np.float64)
    rec = np.zeros((n_rounds, M, 9), dtype=np.float64)
    rung = np.zeros((n_rounds, M), dtype=np.int32)
    i32 = ctypes.POINTER(ctypes.c_int32)
    rc = lib().orc_pt_run(sd, M, L, _dp(b), _dp(d), member.ctypes.data_as(i32), pt_seed, ladder, round0, sweep0,
                          n_rounds, K, _prec(prec), _dp(phi), _dp(rec), rung.ctypes.data_as(i32))
    if rc != 0:
        raise MemoryError("orc_pt_run")
    return rec, rung
