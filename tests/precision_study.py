"""Precision study: FP16 vs FP32 angle storage against the FP64 oracle.

Not collected by pytest (a long measurement, run by hand on an MI355X):

    python tests/precision_study.py [--sweeps 20000 --discard 2000]   # writes tests/results/precision_study_L8192.json

* device, L = 8192, beta in {0.9, 1.0, 1.1}: FP32 and FP16 storage from the same
  seed and Philox stream, records every 10 sweeps after `discard` sweeps;
* bias run, L = 256, same betas: device FP32, device FP16 and the FP64 oracle
  (FP64 storage), same seed; the oracle runs in one process per beta.

Reports <e>, <|m|> and the helicity modulus with binned errors, and the FP16 and
FP32 biases against the oracle in units of the combined error.
"""
from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)

from mcstats import mean_err  # noqa: E402


def series(cx, cy, ix, iy, mx, my, N, beta):
    e = -(cx + cy) / N
    m = np.hypot(mx, my) / N
    u = (cx + cy - beta * (ix * ix + iy * iy)) / (2.0 * N)
    return e, m, u


def summarize(e, m, u):
    out = {}
    for name, s in (("e", e), ("abs_m", m), ("helicity", u)):
        mu, err = mean_err(s)
        out[name] = [float(mu), float(err)]
    return out


def device_run(L, beta, prec, seed, sweeps, discard, every):
    import torch

    from paper_0811_2111_amd import xy
    lat = xy.Lattice(L, seed=seed, beta=beta, delta=1.0, precision=prec)
    lat.sweep(discard)
    t0 = time.perf_counter()
    obs = lat.sweep(sweeps, every)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    r = xy.records(obs)
    s = summarize(*series(r["cx"], r["cy"], r["ix"], r["iy"], r["mx"], r["my"], L * L, beta))
    s["seconds"] = dt
    return s


def oracle_run(args):
    L, beta, seed, sweeps, discard, every = args
    import oracle
    th = oracle.hot_start(seed, L, "f64")
    oracle.run(seed, th, beta, 1.0, discard, 0, prec="f64")
    recs, done, chunk = [], 0, 1000
    while done < sweeps:                   # chunks, so a long run reports progress
        n = min(chunk, sweeps - done)
        recs.append(oracle.run(seed, th, beta, 1.0, n, every, sweep0=discard + done, prec="f64"))
        done += n
        print("oracle L=%d beta=%s: %d/%d sweeps" % (L, beta, done, sweeps), flush=True)
    rec = np.concatenate(recs)
    return summarize(*series(rec[:, 2], rec[:, 3], rec[:, 4], rec[:, 5], rec[:, 6], rec[:, 7], L * L, beta))


def bias(a, b):
    return {k: [a[k][0] - b[k][0], math.hypot(a[k][1], b[k][1])] for k in ("e", "abs_m", "helicity")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "results", "precision_study_L8192.json"))
    ap.add_argument("--sweeps", type=int, default=20000)
    ap.add_argument("--discard", type=int, default=2000)
    ap.add_argument("--oracle-sweeps", type=int, default=20000)
    ap.add_argument("--large-L", type=int, default=8192)
    ap.add_argument("--bias-L", type=int, default=256)
    ap.add_argument("--seed", type=int, default=1)
    a = ap.parse_args()
    betas = (0.9, 1.0, 1.1)
    res = {"config": vars(a), "betas": betas, "large": {}, "bias": {}}

    pool = mp.get_context("spawn").Pool(len(betas))
    jobs = pool.map_async(oracle_run, [(a.bias_L, b, a.seed, a.oracle_sweeps, a.discard, 10) for b in betas])

    for b in betas:
        for prec in ("fp32", "fp16"):
            r = device_run(a.large_L, b, prec, a.seed, a.sweeps, a.discard, 10)
            res["large"]["%s/%s" % (b, prec)] = r
            print("L=%d beta=%s %s: %s" % (a.large_L, b, prec, r), flush=True)
    dev = {}
    for b in betas:
        for prec in ("fp32", "fp16"):
            dev[(b, prec)] = device_run(a.bias_L, b, prec, a.seed, a.oracle_sweeps, a.discard, 10)
    orc = jobs.get()
    pool.close()
    for b, o in zip(betas, orc):
        entry = {"oracle_f64": o, "fp32": dev[(b, "fp32")], "fp16": dev[(b, "fp16")],
                 "bias_fp32": bias(dev[(b, "fp32")], o), "bias_fp16": bias(dev[(b, "fp16")], o)}
        res["bias"][str(b)] = entry
        print("L=%d beta=%s bias fp32 %s fp16 %s" % (a.bias_L, b, entry["bias_fp32"], entry["bias_fp16"]), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
