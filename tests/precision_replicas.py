"""Storage-precision bias from independent replicas (FP32 and FP16 storage on the
device against FP64 storage in the oracle).

Not collected by pytest (a long measurement, run by hand on an MI355X):

    python tests/precision_replicas.py [--replicas 16 --sweeps 4000 --discard 1000]   # writes tests/results/precision_replicas_L256.json

For each beta, R replicas of an L x L lattice (seeds seed0 .. seed0 + R - 1, hot
start) run `sweeps` sweeps; each replica's means of e, |m| and the helicity
estimator over the records after `discard` sweeps are one sample.  The device
runs the R replicas of one storage format as one batch launch; the oracle runs
each replica in its own process.  The bias of a format is the difference of the
replica averages, its error the standard error from the replica-to-replica
spread (replicas are independent, so no autocorrelation analysis is needed;
replica r draws the same Philox numbers on both sides, which only correlates
the two samples and makes the quoted error conservative).
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


def replica_means(cx, cy, ix, iy, mx, my, N, beta):
    e = -(cx + cy) / N
    m = np.hypot(mx, my) / N
    u = (cx + cy - beta * (ix * ix + iy * iy)) / (2.0 * N)
    return [float(e.mean()), float(m.mean()), float(u.mean())]


def oracle_replica(args):
    L, beta, seed, sweeps, discard, every = args
    import oracle
    th = oracle.hot_start(seed, L, "f64")
    oracle.run(seed, th, beta, 1.0, discard, 0, prec="f64")
    rec = oracle.run(seed, th, beta, 1.0, sweeps - discard, every, sweep0=discard, prec="f64")
    return replica_means(rec[:, 2], rec[:, 3], rec[:, 4], rec[:, 5], rec[:, 6], rec[:, 7], L * L, beta)


def device_replicas(L, beta, seeds, sweeps, discard, every, prec):
    import torch

    from paper_0811_2111_amd import xy
    R = len(seeds)
    b = xy.Batch([L] * R, seeds, [beta] * R, [1.0] * R, precision=prec)
    b.sweep(discard)
    out = b.sweep(sweeps - discard, every)
    torch.cuda.synchronize()
    res = []
    for r in range(R):
        rec = xy.records(out[r])
        res.append(replica_means(rec["cx"], rec["cy"], rec["ix"], rec["iy"], rec["mx"], rec["my"], L * L, beta))
    return res


def summary(samples):
    a = np.asarray(samples)
    return a.mean(axis=0), a.std(axis=0, ddof=1) / math.sqrt(a.shape[0])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "results", "precision_replicas_L256.json"))
    ap.add_argument("--L", type=int, default=256)
    ap.add_argument("--replicas", type=int, default=16)
    ap.add_argument("--sweeps", type=int, default=4000)
    ap.add_argument("--discard", type=int, default=1000)
    ap.add_argument("--every", type=int, default=10)
    ap.add_argument("--seed0", type=int, default=1000)
    ap.add_argument("--procs", type=int, default=16)
    a = ap.parse_args()
    betas = (0.9, 1.0, 1.1)
    seeds = [a.seed0 + r for r in range(a.replicas)]
    jobs = [(a.L, b, s, a.sweeps, a.discard, a.every) for b in betas for s in seeds]
    pool = mp.get_context("spawn").Pool(a.procs)
    pending = pool.map_async(oracle_replica, jobs, chunksize=1)
    t0 = time.time()
    dev = {}
    for b in betas:
        for prec in ("fp32", "fp16"):
            dev[(b, prec)] = device_replicas(a.L, b, seeds, a.sweeps, a.discard, a.every, prec)
            print("device beta=%s %s done (%.0f s)" % (b, prec, time.time() - t0), flush=True)
    while not pending.ready():
        pending.wait(30)
        print("oracle replicas running (%.0f s)" % (time.time() - t0), flush=True)
    orc = pending.get()
    pool.close()
    names = ("e", "abs_m", "helicity")
    res = {"config": vars(a), "betas": betas, "results": {}}
    for i, b in enumerate(betas):
        o = orc[i * a.replicas:(i + 1) * a.replicas]
        om, oe = summary(o)
        entry = {"oracle_f64": {n: [float(om[k]), float(oe[k])] for k, n in enumerate(names)}}
        for prec in ("fp32", "fp16"):
            dm, de = summary(dev[(b, prec)])
            entry[prec] = {n: [float(dm[k]), float(de[k])] for k, n in enumerate(names)}
            entry["bias_" + prec] = {n: [float(dm[k] - om[k]), float(math.hypot(de[k], oe[k]))]
                                     for k, n in enumerate(names)}
        res["results"][str(b)] = entry
        print("beta=%s bias fp32 %s" % (b, {n: "%+.5f(%.5f)" % tuple(v) for n, v in entry["bias_fp32"].items()}),
              flush=True)
        print("beta=%s bias fp16 %s" % (b, {n: "%+.5f(%.5f)" % tuple(v) for n, v in entry["bias_fp16"].items()}),
              flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
