"""Exact finite-lattice values of the 2-d XY model and its q-state clock restriction.

Writes ``exact_small_lattices.json`` next to this file.  The values pin the FP64
oracle's Markov chain (the tests compare long oracle runs against them); they
are computed here from the definition of the ensemble only and import nothing
from the oracle or from the product library.

Model: H = -J sum_<ij> cos(theta_i - theta_j) on a periodic W x Ly lattice,
J = 1, every nearest-neighbour pair counted once (section 1.2, eq. 1), weight
exp(-beta H).  Clock restriction: theta = 2 pi k / q.

Methods
  * brute force: every one of the q^N configurations (3x3, q = 6);
  * row transfer matrix: Z = Tr T^Ly with
    T(s, s') = exp(beta [h(s)/2 + h(s')/2 + v(s, s')]), h the horizontal bonds
    of one periodic row and v the vertical bonds between two rows.  For 4x4 the
    global-rotation symmetry k -> k+1 block-diagonalises T into q sectors
    T_m(s, s') = sum_d omega^(-m d) T(s, R^d s'), s, s' restricted to k_0 = 0,
    and Z = sum_m Tr T_m^Ly.
  * <E> = -d ln Z / d beta, differentiated analytically:
    dZ/dbeta = Ly Tr(T^(Ly-1) dT/dbeta), dT/dbeta = X * T elementwise.
  * The continuous model is the q -> infinity limit of the clock model; the
    error decays faster than any power of 1/q, and agreement between two q
    values is recorded as evidence of convergence.

Run:  python tests/golden/exact_xy.py     (about a minute on 8 cores)
"""
from __future__ import annotations

import itertools
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "exact_small_lattices.json")


def brute_force_clock(L: int, q: int, betas):
    """All q^(L*L) states of the periodic L x L q-clock model.

    Returns {beta: {"E_per_site", "abs_m", "helicity", "C"}} where
    abs_m = <|sum_i (cos, sin)|>/N, helicity = (<Cx+Cy> - beta <Ix^2+Iy^2>)/(2N),
    C = beta^2 Var(E)/N.
    """
    N = L * L
    ang = 2.0 * np.pi * np.arange(q) / q
    cos_d = np.cos(2.0 * np.pi * np.arange(q) / q)      # cos of angle difference (k_i - k_j) mod q
    sin_d = np.sin(2.0 * np.pi * np.arange(q) / q)
    # split the N sites into a leading block (outer loop) and a trailing block (vectorised)
    n_tail = min(N, 6)
    n_head = N - n_tail
    tail = np.array(list(itertools.product(range(q), repeat=n_tail)), dtype=np.int64)  # (q^t, t)
    betas = list(betas)
    E0 = -2.0 * N
    acc = {b: np.zeros(6) for b in betas}   # sum w, wE, wE^2, w|m|, w(Cx+Cy), w(Ix^2+Iy^2)
    for head in itertools.product(range(q), repeat=n_head):
        k = np.empty((tail.shape[0], N), dtype=np.int64)
        k[:, :n_head] = np.array(head, dtype=np.int64)[None, :]
        k[:, n_head:] = tail
        cxy = np.zeros(tail.shape[0])
        ix = np.zeros(tail.shape[0])
        iy = np.zeros(tail.shape[0])
        for y in range(L):
            for x in range(L):
                i = y * L + x
                r = y * L + (x + 1) % L
                d = ((y + 1) % L) * L + x
                dr = (k[:, i] - k[:, r]) % q
                dd = (k[:, i] - k[:, d]) % q
                cxy += cos_d[dr] + cos_d[dd]
                ix += sin_d[dr]
                iy += sin_d[dd]
        mx = np.cos(ang[k]).sum(axis=1)
        my = np.sin(ang[k]).sum(axis=1)
        E = -cxy
        am = np.hypot(mx, my)
        I2 = ix * ix + iy * iy
        for b in betas:
            w = np.exp(-b * (E - E0))
            a = acc[b]
            a[0] += w.sum(); a[1] += (w * E).sum(); a[2] += (w * E * E).sum()
            a[3] += (w * am).sum(); a[4] += (w * cxy).sum(); a[5] += (w * I2).sum()
    res = {}
    for b in betas:
        a = acc[b]
        Z = a[0]
        e = a[1] / Z
        var = a[2] / Z - e * e
        res[b] = {
            "E_per_site": e / N,
            "abs_m": a[3] / Z / N,
            "helicity": (a[4] / Z - b * a[5] / Z) / (2.0 * N),
            "C": b * b * var / N,
        }
    return res


def _row_parts(W: int, q: int):
    """Row states (all q^W), horizontal-bond sum h(s) of a periodic row."""
    states = np.array(list(itertools.product(range(q), repeat=W)), dtype=np.int64)
    th = 2.0 * np.pi * states / q
    h = np.zeros(states.shape[0])
    for i in range(W):
        h += np.cos(th[:, i] - th[:, (i + 1) % W])
    return states, th, h


def _dlnZ_from_blocks(blocks, Ly: int) -> float:
    """d ln Z / d beta for Z = sum_b Tr A_b^Ly given pairs (A_b, dA_b/dbeta):
    dZ = Ly sum_b Tr(A_b^(Ly-1) dA_b)."""
    Z = 0.0
    dZ = 0.0
    for A, dA in blocks:
        P = np.linalg.matrix_power(A, Ly - 1)
        Z += np.real(np.trace(P @ A))
        dZ += Ly * np.real(np.sum(P * dA.T))      # Tr(P dA)
    return dZ / Z


def dlnZ_transfer(W: int, Ly: int, q: int, beta: float) -> float:
    """d ln Z / d beta of the periodic W x Ly q-clock model, full row transfer matrix."""
    states, th, h = _row_parts(W, q)
    v = np.zeros((states.shape[0], states.shape[0]))
    for i in range(W):
        v += np.cos(th[:, i][:, None] - th[:, i][None, :])
    shift = 2.0 * W            # largest possible h/2 + h/2 + v, keeps entries O(1)
    X = 0.5 * h[:, None] + 0.5 * h[None, :] + v - shift
    T = np.exp(beta * X)
    return _dlnZ_from_blocks([(T, X * T)], Ly) + shift * Ly


def dlnZ_transfer_sectors(W: int, Ly: int, q: int, beta: float) -> float:
    """d ln Z / d beta of the periodic W x Ly q-clock model, rotation-symmetry sectors."""
    reps = np.array([(0,) + t for t in itertools.product(range(q), repeat=W - 1)], dtype=np.int64)
    th = 2.0 * np.pi * reps / q
    h = np.zeros(reps.shape[0])
    for i in range(W):
        h += np.cos(th[:, i] - th[:, (i + 1) % W])
    shift = 2.0 * W
    base = 0.5 * h[:, None] + 0.5 * h[None, :] - shift
    Td, Xd = [], []            # T(s, R^d s') and its exponent, for every rotation d
    for d in range(q):
        v = np.zeros((reps.shape[0], reps.shape[0]))
        rot = th + 2.0 * np.pi * d / q
        for i in range(W):
            v += np.cos(th[:, i][:, None] - rot[:, i][None, :])
        X = base + v
        Td.append(np.exp(beta * X))
        Xd.append(X)
    blocks = []
    for m in range(q):
        Tm = np.zeros_like(Td[0], dtype=np.complex128)
        dTm = np.zeros_like(Td[0], dtype=np.complex128)
        for d in range(q):
            ph = np.exp(-2j * np.pi * m * d / q)
            Tm += ph * Td[d]
            dTm += ph * (Xd[d] * Td[d])
        blocks.append((Tm, dTm))
    return _dlnZ_from_blocks(blocks, Ly) + shift * Ly


def energy_per_site(dlnZ, W: int, Ly: int, q: int, beta: float) -> float:
    return -dlnZ(W, Ly, q, beta) / (W * Ly)


def main():
    betas = [0.1, 0.5, 1.0, 1.12, 1.5, 2.0]
    out = {
        "citation": ("XY Hamiltonian H = -sum_<ij> cos(theta_i - theta_j), section 1.2 eq. 1, "
                     "J = 1, periodic boundaries, weight exp(-beta H); values computed by "
                     "tests/golden/exact_xy.py (brute force / row transfer matrix)"),
        "clock_3x3_q6_bruteforce": {},
        "clock_3x3_q6_transfer_E": {},
        "clock_4x4_q6_transfer_E": {},
        "xy_3x3_continuous_E": {},
        "xy_4x4_continuous_E": {},
    }
    bf = brute_force_clock(3, 6, betas)
    for b in betas:
        out["clock_3x3_q6_bruteforce"][repr(b)] = bf[b]
        out["clock_3x3_q6_transfer_E"][repr(b)] = energy_per_site(dlnZ_transfer, 3, 3, 6, b)
    for b in [0.5, 1.0, 2.0]:
        out["clock_4x4_q6_transfer_E"][repr(b)] = energy_per_site(dlnZ_transfer, 4, 4, 6, b)
        e12 = energy_per_site(dlnZ_transfer, 3, 3, 12, b)
        e16 = energy_per_site(dlnZ_transfer, 3, 3, 16, b)
        out["xy_3x3_continuous_E"][repr(b)] = {"q16": e16, "q12": e12, "diff": abs(e16 - e12)}
        f12 = energy_per_site(dlnZ_transfer_sectors, 4, 4, 12, b)
        f14 = energy_per_site(dlnZ_transfer_sectors, 4, 4, 14, b)
        out["xy_4x4_continuous_E"][repr(b)] = {"q14": f14, "q12": f12, "diff": abs(f14 - f12)}
        print("beta", b, "3x3", e12, e16, "4x4", f12, f14, flush=True)
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
