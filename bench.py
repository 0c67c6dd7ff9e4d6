#!/usr/bin/env python
"""Benchmark: checkerboard Metropolis sweeps of the 2-d XY model on one MI355X.

Workload (default): the HBM-streaming lattice, L = 16384 (268 M sites, 1 GiB of
FP32 angles), beta = 1.0, delta = 1.2, hot start from seed 1, every observable
(FP64 energy, helicity and magnetisation sums) recorded after every sweep.  One
step = 25 sweeps with their 25 records; W warm-up steps, then K timed steps
(defaults W = 4, K = 20: the configuration's 500 sweeps), the plan picked by the
library's autotuner on a scratch lattice of the same size.

Prints one JSON line.  `value` is site-updates per second (Gupd/s) of the timed
region, inputs resident in HBM.  `roofline` covers the dominant kernel (the
sweep kernel of the chosen plan, measured sweeps): its launches in the timed
region are bracketed by HIP events on the stream they run on (the library's
kernel timer), and achieved = 8 algorithmic bytes per site-update (read and
write each FP32 angle once) x L^2 / average launch duration, against the 8 TB/s
HBM3E peak; the device-to-device copy rate measured in the same run is given
beside it.  `traffic` is the counter-measured HBM bytes per launch from the
committed profile, while the kernel sources still hash as profiled.
`cpu_baseline` is the FP64 C oracle on one sweep of the same lattice on one host
core.  `extra` holds the other configurations of the metric: the MALL-resident
L = 4096 lattice with its ALU roofline, the batched 96-lattice temperature scan
against per-lattice launches, tempering, FP16 storage, four replicas per texel
and HMC.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0                    # MI355X HBM3E
# VALU issue slots: one slot = the issue cost of one wave64 v_add_f32.  Peak:
# 256 CUs x 128 FP32 lanes x 2.4 GHz = 78.6 T slots/s (the non-packed FP32 rate,
# half of the 157.3 TFLOP/s vector FMA peak).
VALU_PEAK_TSLOTS = 256 * 128 * 2.4e9 / 1e12
# Algorithmic VALU slots of one site update of a sweep that reads the angles once,
# with the issue costs measured on MI355X relative to v_add_f32
# (throughput microbenchmark, profiles/valu_issue_costs.md: v_mad_u64_u32 2.76, v_sin/v_cos 3.42,
# v_exp 3.50, v_bitop3_b32 1.72, v_fma/v_fmaak 1.14, v_fract 1.06, others 1) and the
# instruction counts of the compiled update:
#   half a Philox4x32-10 call (16.5 v_mad_u64_u32, 13 v_bitop3, 3 v_xor per call)   35.5
#   two uniforms (2 alignbit, fmaak, 2 add)                                         5.1
#   proposal: multiply, add, fract                                                  3.1
#   sin and cos of the proposal                                                     6.8
#   sin and cos of the site's loaded angle (the (cos, sin) shared with neighbours)  6.8
#   two neighbour sums of four terms                                                6
#   dE (2 sub, mul, fma)                                                            4.1
#   acceptance (mul, exp2, compare)                                                 5.5
#   three selects                                                                   3
ALG_SLOTS_PER_UPDATE = 76.0
# A measured sweep adds the bond and magnetisation sums at every black site (half
# the updates): 8 fma for the four bond cosines and sines (the left + right and
# up + down sums are the update's own), 4 subtractions, 4 additions for Mx, My:
# 8 x 1.14 + 8 = 17.1 slots per black site, 8.56 per update.
ALG_SLOTS_MEAS_PER_UPDATE = 8.56
ALG_BYTES_FUSED = 8.0                    # bytes per site-update of one fused sweep: read 4 + write 4 (FP32)
ALG_BYTES_STREAM = 12.0                  # two half-sweep passes: read both colours, write one, per half
ALG_BYTES_HMC_STEP = 16.0                # one leap-frog step: read and write the angle and the momentum
PLAN_NAMES = {1: "stream", 2: "fused", 3: "strip", 4: "resident"}
BATCH_SCHEDULES = {0: "persistent", 1: "per-sweep launches", 2: "per-sweep launches, 256x16 tiles where L allows"}
KERNEL_NAMES = {1: "k_half_sweep", 2: "k_fused (LDS-tiled fused red+black sweep)",
                3: "k_strip (strip segment, rows streamed through LDS rings)"}
# Counter profiles (FETCH_SIZE / WRITE_SIZE per launch) of the tiled sweep kernels,
# valid while the kernel's sources hash as they did when the counters were taken.
TRAFFIC_FILES = {2: os.path.join(ROOT, "profiles", "k_fused_traffic.json"),
                 3: os.path.join(ROOT, "profiles", "k_strip_traffic.json")}
KERNEL_SOURCES = {2: ["xy_device.hpp", "xy_tile1.hpp", "xy_fused.hip"],
                  3: ["xy_device.hpp", "xy_tile1.hpp", "xy_strip.hpp", "xy_strip.hip"]}
TRAFFIC_FILE = TRAFFIC_FILES[2]           # the fused kernel's file (kept for its CPU test)


def kernel_sources_hash(kind: int = 2) -> str:
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[kind]:
        with open(os.path.join(ROOT, "paper_0811_2111_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(L, plan, measured=False):
    """HBM bytes per launch of the plan's sweep kernel (measured or unmeasured
    sweep) from the committed counter profile, if it was taken on the current
    kernel sources for this lattice and tile; else None."""
    e = counter_entry(L, plan, measured)
    return None if e is None else e.get("bytes_per_launch")


def counter_entry(L, plan, measured=False):
    """The committed counter record of the plan's sweep kernel (HBM bytes, and
    for the headline kernel its VALU counters) if it was taken on the current
    kernel sources for this lattice and tile; else None."""
    kind = plan[0]
    path = TRAFFIC_FILE if kind == 2 else TRAFFIC_FILES.get(kind)
    if path is None:
        return None
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sources_sha256") != kernel_sources_hash(kind):
        return None
    key = "%d/%d,%d,%d" % (L, plan[1], plan[2], plan[3]) + ("/meas" if measured else "")
    e = t.get("entries", {}).get(key)
    if e is None and not measured and kind == 2:
        e = t.get("entries", {}).get("%d/%d,%d,%d" % (L, plan[1], plan[2], plan[3]))
    return e


def host_cpu():
    """Host CPU of this run: logical CPUs usable by this process and the model name."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count()
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return n, model


def copy_rate_gbs(stream, nbytes=1 << 30, reps=10):
    """Device-to-device copy of nbytes (read + write bytes per second): the HBM
    rate a plain streaming kernel reaches on this device."""
    import torch
    a = torch.ones((nbytes // 4,), dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    ms = timed(lambda: [b.copy_(a) for _ in range(reps)], stream)
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * nbytes * reps / (ms * 1e-3) / 1e9


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed steps of 25 sweeps (default: 500 sweeps)")
    ap.add_argument("--warmup", type=int, default=4, help="untimed steps of 25 sweeps before the timed ones")
    ap.add_argument("--no-extra", action="store_true", help="skip the L=4096, batched, FP16, quad and HMC legs")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-sweeps", type=int, default=1, help="oracle sweeps of the L=16384 sample")
    ap.add_argument("--kernel-only", action="store_true",
                    help="only the main workload's sweeps (for profiler runs)")
    ap.add_argument("--plan", type=str, default=None,
                    help="fixed plan 'kind,tile_x,tile_y,sweeps_per_pass' instead of autotuning")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one 256 MiB device-to-device copy (calibrates HBM byte counters)")
    ap.add_argument("--workload", choices=["l4096", "l4096_tuned", "l16384", "batch", "hmc", "hmc_batch", "quad",
                                           "quad_hmc", "fp16", "l8192",
                                           "tempering", "small"],
                    default="l16384",
                    help="with --kernel-only: which configuration's sweeps to run (for profiler runs)")
    ap.add_argument("--schedule", type=int, default=None,
                    help="with --kernel-only --workload batch, tempering or small: batch schedule (0 persistent, 1 per-sweep, "
                         "2 per-sweep with wide tiles; default: the library's)")
    return ap.parse_args()


def timed(fn, stream):
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)            # ms


SWEEPS_PER_STEP = 25


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (got --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_0811_2111_amd import workloads, xy

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.kernel_only and args.workload != "l16384":
        profile_leg(args, stream)
        return
    cfg = workloads.SINGLE_16384
    L, me, sps = cfg["L"], cfg["measure_every"], SWEEPS_PER_STEP
    N = L * L
    # the plan (schedule and tile shape) is picked by the library's autotuner on a
    # scratch lattice of the same size; it does not change the trajectory
    if args.plan:
        tuned = tuple(int(v) for v in args.plan.split(","))
    else:
        scratch = xy.Lattice(L, seed=cfg["seed"] + 1000, beta=cfg["beta"], delta=cfg["delta"])
        tuned = scratch.autotune(8)
        del scratch
        torch.cuda.empty_cache()
    lat = xy.Lattice(L, seed=cfg["seed"], beta=cfg["beta"], delta=cfg["delta"], plan=tuned)
    plan = lat.plan
    tiled = plan[0] in (xy.XY_PLAN_FUSED, xy.XY_PLAN_STRIP)
    if args.calib_copy:
        a = torch.ones((64 << 20,), dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    copy_gbs = None if args.kernel_only else copy_rate_gbs(stream)
    obs_w = torch.empty((max(args.warmup * sps, 1), 8), dtype=torch.float64, device="cuda")
    obs_t = torch.empty((max(args.steps * sps, 1), 8), dtype=torch.float64, device="cuda")
    # warm-up steps right before the timed ones bring the clocks up after the host
    # work above; the library's kernel timer brackets every sweep launch of the
    # timed region with HIP events on the lattice's stream
    torch.cuda.synchronize()
    if args.warmup:
        lat.sweep(sps * args.warmup, me, out=obs_w)
    torch.cuda.synchronize()
    if tiled:
        lat.kernel_timer(args.steps * sps)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    lat.sweep(sps * args.steps, me, out=obs_t)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    k_ms, k_n = lat.kernel_timer_read() if tiled else (0.0, 0)
    lat.kernel_timer(0)
    updates = float(N) * sps * args.steps
    gupd = updates / (ms * 1e-3) / 1e9
    rec = xy.records(obs_t[: args.steps * sps])
    e_mean = float(-(rec["cx"] + rec["cy"]).mean() / N)
    acc_rate = float(rec["n_accept"].mean() / N)
    ups = float(rec["cx"].size)

    # dominant kernel: the measured sweep launch of the chosen plan
    if k_n:
        per_launch_ms = k_ms / k_n
        upd_per_launch = N * plan[3]
        alg_bytes = ALG_BYTES_FUSED * N          # one read and one write of every angle per launch
    else:                                        # streaming plan: no timer; whole sweeps
        per_launch_ms = ms / (sps * args.steps)
        upd_per_launch = N
        alg_bytes = ALG_BYTES_STREAM * N
    achieved_gbs = alg_bytes / (per_launch_ms * 1e-3) / 1e9
    roofline = {
        "kernel": KERNEL_NAMES.get(plan[0], "sweep") + ", measured sweep",
        "bound": "hbm",
        "achieved": round(achieved_gbs, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved_gbs / HBM_PEAK_GBS, 4),
        "traffic": measured_traffic(L, plan, measured=True),
        "alg_bytes_per_update": ALG_BYTES_FUSED if k_n else ALG_BYTES_STREAM,
        "alg_bytes_per_launch": alg_bytes,
        "avg_launch_ms": round(per_launch_ms, 5),
        "launches_timed": k_n,
        "kernel_gupd_s": round(upd_per_launch / (per_launch_ms * 1e-3) / 1e9, 2),
    }
    if copy_gbs is not None:
        roofline["device_copy_GBs"] = round(copy_gbs, 1)
        roofline["frac_of_device_copy"] = round(achieved_gbs / copy_gbs, 4)
    # the same launch against the VALU issue rate (the measured sweep's update and
    # record arithmetic; peak 78.6 T slots/s)
    slots = (ALG_SLOTS_PER_UPDATE + ALG_SLOTS_MEAS_PER_UPDATE) * upd_per_launch / (per_launch_ms * 1e-3) / 1e12
    roofline["alu"] = {"achieved": round(slots, 2), "peak": round(VALU_PEAK_TSLOTS, 2), "unit": "T VALU-slot/s",
                       "frac": round(slots / VALU_PEAK_TSLOTS, 4),
                       "alg_slots_per_update": ALG_SLOTS_PER_UPDATE + ALG_SLOTS_MEAS_PER_UPDATE}
    # the committed counter record of this kernel (same sources): vector
    # instructions per update and rocprof's VALU-busy measure
    # (100 SQ_ACTIVE_INST_VALU / 256 CUs / (GRBM_GUI_ACTIVE / 8 XCDs)); None if stale
    ce = counter_entry(L, plan, measured=True)
    roofline["alu"]["valu_insts_per_update"] = None if ce is None else ce.get("valu_insts_per_update")
    roofline["alu"]["valu_busy_pct"] = None if ce is None else ce.get("valu_busy_pct")
    out = {
        "metric": "site-updates/sec (Gupd/s) at 1 MI355X; % HBM roofline; batched vs per-lattice speedup",
        "value": round(gupd, 3),
        "unit": "Gupd/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / max(args.steps, 1), 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (hot start from Philox seed 1)",
        "config": {"workload": "XY checkerboard Metropolis, L=16384 single lattice (HBM-streaming), beta=1.0, "
                               "delta=1.2, FP64 E/helicity/M record every sweep; step = 25 sweeps",
                   "L": L, "beta": cfg["beta"], "delta": cfg["delta"], "sweeps_per_step": sps,
                   "measure_every": me,
                   "plan": {"kind": PLAN_NAMES[plan[0]], "tile_x": plan[1], "tile_y": plan[2],
                            "sweeps_per_pass": plan[3]},
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "observables": {"E_per_site": round(e_mean, 6), "accept_rate": round(acc_rate, 4),
                        "records": int(ups)},
    }

    if not args.kernel_only and not args.no_extra:
        del lat, obs_w, obs_t
        torch.cuda.empty_cache()
        out["extra"] = extra_legs(stream, args)

    if not args.kernel_only and not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_sweeps)

    print(json.dumps(out), flush=True)


def l4096_leg(stream, steps=1000, warmup=100):
    """The MALL-resident L = 4096 lattice (beta = 1.12, delta = 1.0, a record every
    10 sweeps): Gupd/s, and the dominant (unmeasured fused) launch against the ALU
    and HBM peaks."""
    import torch

    from paper_0811_2111_amd import workloads, xy
    cfg = workloads.SINGLE_4096
    L, me = cfg["L"], cfg["measure_every"]
    N = L * L
    scratch = xy.Lattice(L, seed=cfg["seed"] + 1000, beta=cfg["beta"], delta=cfg["delta"])
    tuned = scratch.autotune(20)
    del scratch
    lat = xy.Lattice(L, seed=cfg["seed"], beta=cfg["beta"], delta=cfg["delta"], plan=tuned)
    plan = lat.plan
    obs_w = torch.empty((warmup, 8), dtype=torch.float64, device="cuda")
    obs_t = torch.empty((steps, 8), dtype=torch.float64, device="cuda")
    lat.sweep(me * warmup, me, out=obs_w)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    lat.sweep(me * steps, me, out=obs_t)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    gupd = float(N) * me * steps / (ms * 1e-3) / 1e9
    res = {"gupd_s": round(gupd, 2), "sweeps": me * steps, "ms": round(ms, 2), "plan": list(plan),
           "thermalisation_sweeps": me * warmup}
    tiled = plan[0] in (xy.XY_PLAN_FUSED, xy.XY_PLAN_STRIP)
    if tiled:
        # unmeasured launches (9 of every 10 sweeps) timed by the library's kernel
        # timer, after 200 untimed sweeps queued right before
        lat.sweep(plan[3] * 200)
        lat.kernel_timer(600)
        lat.sweep(plan[3] * 600)
        k_ms, k_n = lat.kernel_timer_read()
        lat.kernel_timer(0)
        per_launch_ms = k_ms / k_n
        upd = N * plan[3]
        slots = ALG_SLOTS_PER_UPDATE * upd / (per_launch_ms * 1e-3) / 1e12
        gbs = ALG_BYTES_FUSED * N / (per_launch_ms * 1e-3) / 1e9
        res["roofline_alu"] = {"kernel": KERNEL_NAMES[plan[0]] + ", unmeasured sweep", "bound": "alu",
                               "achieved": round(slots, 2), "peak": round(VALU_PEAK_TSLOTS, 2),
                               "unit": "T VALU-slot/s", "frac": round(slots / VALU_PEAK_TSLOTS, 4),
                               "alg_slots_per_update": ALG_SLOTS_PER_UPDATE,
                               "avg_launch_ms": round(per_launch_ms, 5), "launches_timed": k_n,
                               "kernel_gupd_s": round(upd / (per_launch_ms * 1e-3) / 1e9, 2),
                               "traffic": measured_traffic(L, plan),
                               "hbm": {"achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                       "frac": round(gbs / HBM_PEAK_GBS, 4),
                                       "alg_bytes_per_update": ALG_BYTES_FUSED}}
    del lat, obs_w, obs_t
    torch.cuda.empty_cache()
    return res


def profile_leg(args, stream):
    """Only the sweeps of one non-default configuration (profiler runs)."""
    import torch

    from paper_0811_2111_amd import workloads, xy
    if args.calib_copy:
        a = torch.ones((64 << 20,), dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.workload == "l4096_tuned":
        # the benchmark's L = 4096 leg itself: the autotuner's trials, then the sweeps
        print(json.dumps({"workload": "L4096 tuned", **l4096_leg(stream, steps=args.steps, warmup=args.warmup)}))
    elif args.workload == "l4096":
        c2 = workloads.SINGLE_4096
        plan = tuple(int(v) for v in args.plan.split(",")) if args.plan else None
        lat = xy.Lattice(c2["L"], seed=c2["seed"], beta=c2["beta"], delta=c2["delta"], plan=plan)
        me = c2["measure_every"]
        obs = torch.empty((max(args.steps, 1), 8), dtype=torch.float64, device="cuda")
        lat.sweep(me * args.warmup, me, out=obs[: max(args.warmup, 1)])
        ms = timed(lambda: lat.sweep(me * args.steps, me, out=obs[: args.steps]), stream)
        print(json.dumps({"workload": "L4096", "sweeps": me * args.steps, "ms": ms, "plan": list(lat.plan),
                          "gupd_s": float(c2["L"]) ** 2 * me * args.steps / (ms * 1e-3) / 1e9}))
    elif args.workload == "hmc":
        hc = workloads.HMC_16384
        lat = xy.Lattice(hc["L"], seed=hc["seed"], beta=hc["beta"])
        lat.sweep(args.warmup)
        ms = timed(lambda: lat.hmc(args.steps, hc["n_md"], hc["eps"]), stream)
        print(json.dumps({"workload": "HMC L16384", "trajectories": args.steps, "ms": ms,
                          "g_site_steps_s": float(hc["L"]) ** 2 * hc["n_md"] * args.steps / (ms * 1e-3) / 1e9}))
    elif args.workload == "hmc_batch":
        hb = workloads.HMC_SCAN
        sc = workloads.temperature_scan()
        bh = xy.Batch(sc["Ls"], sc["seeds"], sc["betas"], sc["deltas"])
        bh.sweep(args.warmup)
        bh.hmc(1, hb["n_md"], hb["eps"])
        ms = timed(lambda: bh.hmc(args.steps, hb["n_md"], hb["eps"]), stream)
        sites = sum(L * L for L in sc["Ls"])
        print(json.dumps({"workload": "batched HMC scan", "trajectories": args.steps, "ms": ms,
                          "g_site_steps_s": float(sites) * hb["n_md"] * args.steps / (ms * 1e-3) / 1e9}))
    elif args.workload == "quad":
        qc = workloads.QUAD_4096
        qd = xy.Quad(qc["L"], qc["seeds"], qc["betas"], [qc["delta"]] * 4)
        nrec = max(args.steps // qc["measure_every"], 1)
        qobs = torch.empty((nrec, 4, 8), dtype=torch.float64, device="cuda")
        qd.sweep(args.warmup)
        ms = timed(lambda: qd.sweep(args.steps, qc["measure_every"], out=qobs), stream)
        print(json.dumps({"workload": "quad L4096", "sweeps": args.steps, "ms": ms,
                          "gupd_s": 4.0 * float(qc["L"]) ** 2 * args.steps / (ms * 1e-3) / 1e9}))
    elif args.workload in ("fp16", "l8192"):
        # the L = 8192 storage comparison, FP16 or FP32 angles
        pc = workloads.PRECISION
        prec = "fp16" if args.workload == "fp16" else "fp32"
        plan = tuple(int(v) for v in args.plan.split(",")) if args.plan else None
        lat = xy.Lattice(pc["L"], seed=pc["seed"], beta=1.0, delta=pc["delta"], precision=prec, plan=plan)
        lat.sweep(args.warmup)
        ms = timed(lambda: lat.sweep(args.steps, 10), stream)
        print(json.dumps({"workload": "%s L8192" % prec.upper(), "sweeps": args.steps, "ms": ms,
                          "plan": list(lat.plan), "gupd_s": float(pc["L"]) ** 2 * args.steps / (ms * 1e-3) / 1e9}))
    elif args.workload == "small":
        # the parity configuration (L = 32, a record every sweep) on the LDS-resident
        # plan and on the streaming plan, then a batch of 2048 such lattices
        pc = workloads.PARITY_32
        res = {}
        for name, plan in (("resident", (xy.XY_PLAN_RESIDENT, 0, 0, 1)), ("stream", (xy.XY_PLAN_STREAM, 0, 0, 1))):
            lat = xy.Lattice(pc["L"], seed=pc["seed"], beta=pc["beta"], delta=pc["delta"], plan=plan)
            lat.sweep(args.warmup, 1)
            ms = timed(lambda: lat.sweep(args.steps, 1), stream)
            res[name] = {"us_per_sweep": ms * 1e3 / args.steps,
                         "gupd_s": float(pc["L"]) ** 2 * args.steps / (ms * 1e-3) / 1e9}
            del lat
        n = 2048
        b = xy.Batch([pc["L"]] * n, [pc["seed"] + i for i in range(n)], [pc["beta"]] * n, [pc["delta"]] * n)
        if args.schedule is not None:
            b.set_schedule(args.schedule)
        b.sweep(args.warmup)
        ms = timed(lambda: b.sweep(args.steps, 10), stream)
        res["batch_2048"] = {"gupd_s": float(pc["L"]) ** 2 * n * args.steps / (ms * 1e-3) / 1e9}
        print(json.dumps({"workload": "L32", "sweeps": args.steps, **res}))
    elif args.workload == "quad_hmc":
        print(json.dumps({"workload": "quad HMC L4096", **quad_hmc_leg(stream, singles=False)}))
    elif args.workload == "tempering":
        sc = workloads.temperature_scan()
        tb = xy.Batch(sc["Ls"], sc["seeds"], sc["betas"], sc["deltas"])
        if args.schedule is not None:
            tb.set_schedule(args.schedule)
        K = sc["measure_every"]
        rounds = max(args.steps // K, 1)
        tb.tempering(max(args.warmup // K, 1), K, 1)
        ms = timed(lambda: tb.tempering(rounds, K, 1), stream)
        sites = sum(L * L for L in sc["Ls"])
        print(json.dumps({"workload": "tempering scan", "rounds": rounds, "ms": ms,
                          "gupd_s": float(sites) * rounds * K / (ms * 1e-3) / 1e9}))
    else:
        sc = workloads.temperature_scan()
        b = xy.Batch(sc["Ls"], sc["seeds"], sc["betas"], sc["deltas"])
        if args.schedule is not None:
            b.set_schedule(args.schedule)
        nrec = max(args.steps // sc["measure_every"], 1)
        bobs = torch.empty((len(sc["Ls"]), nrec, 8), dtype=torch.float64, device="cuda")
        b.sweep(args.warmup)
        ms = timed(lambda: b.sweep(args.steps, sc["measure_every"], out=bobs), stream)
        sites = sum(L * L for L in sc["Ls"])
        print(json.dumps({"workload": "batched scan", "sweeps": args.steps, "ms": ms,
                          "gupd_s": float(sites) * args.steps / (ms * 1e-3) / 1e9}))


def extra_legs(stream, args=None):
    import torch

    from paper_0811_2111_amd import workloads, xy
    ex = {}
    # the MALL-resident single lattice (ALU-bound) with its roofline
    ex["L4096_mall_resident"] = l4096_leg(stream)
    main_plan = tuple(ex["L4096_mall_resident"]["plan"])

    # batched temperature scan vs per-lattice launches
    sc = workloads.temperature_scan()
    n = len(sc["Ls"])
    sites = sum(L * L for L in sc["Ls"])
    tune = xy.Batch(sc["Ls"], sc["seeds"], sc["betas"], sc["deltas"])
    tile = tune.autotune(20)
    sched = tune.schedule
    del tune
    b = xy.Batch(sc["Ls"], sc["seeds"], sc["betas"], sc["deltas"])
    b.set_tile(*tile)
    b.set_schedule(sched)
    nrec = sc["sweeps"] // sc["measure_every"]
    bobs = torch.empty((n, nrec, 8), dtype=torch.float64, device="cuda")
    b.sweep(20)
    ms_b = timed(lambda: b.sweep(sc["sweeps"], sc["measure_every"], out=bobs), stream)
    g_b = float(sites) * sc["sweeps"] / (ms_b * 1e-3) / 1e9
    # the same scan as one persistent launch per call (same tile shape)
    b.set_schedule(xy.XY_BATCH_PERSISTENT)
    b.sweep(20)
    ms_pk = timed(lambda: b.sweep(sc["sweeps"], sc["measure_every"], out=bobs), stream)
    g_pk = float(sites) * sc["sweeps"] / (ms_pk * 1e-3) / 1e9
    del b, bobs
    per_sweeps = 1000
    lats = [xy.Lattice(L, seed=s, beta=bb, delta=d) for L, s, bb, d in
            zip(sc["Ls"], sc["seeds"], sc["betas"], sc["deltas"])]
    for lt in lats:
        lt.sweep(20)

    def per_lattice():
        for lt in lats:
            lt.sweep(per_sweeps, sc["measure_every"])
    ms_p = timed(per_lattice, stream)
    g_p = float(sites) * per_sweeps / (ms_p * 1e-3) / 1e9
    ex["batched_scan_96"] = {
        "lattices": n, "sites": sites, "sweeps": sc["sweeps"], "tile": list(tile),
        "schedule": BATCH_SCHEDULES[sched],
        "batched_gupd_s": round(g_b, 2), "batched_ms": round(ms_b, 2),
        "per_lattice_gupd_s": round(g_p, 2), "per_lattice_sweeps_timed": per_sweeps,
        "speedup": round(g_b / g_p, 2),
        "persistent_gupd_s": round(g_pk, 2), "persistent_speedup": round(g_pk / g_p, 2)}
    del lats
    torch.cuda.empty_cache()

    # parallel tempering over the same scan: ladders of equal L, rounds of 10 sweeps
    tb = xy.Batch(sc["Ls"], sc["seeds"], sc["betas"], sc["deltas"])
    tb.set_tile(*tile)
    tb.set_schedule(sched)
    rounds, K = sc["sweeps"] // sc["measure_every"], sc["measure_every"]
    tb.tempering(2, K, 1)
    trec = torch.empty((rounds, n, 8), dtype=torch.float64, device="cuda")
    trung = torch.empty((rounds, n), dtype=torch.int32, device="cuda")
    ms_t = timed(lambda: tb.tempering(rounds, K, 1, out=trec, rungs=trung), stream)
    moved = float((trung[1:] != trung[:-1]).float().mean())
    ex["tempering_scan_96"] = {"gupd_s": round(float(sites) * rounds * K / (ms_t * 1e-3) / 1e9, 2),
                               "rounds": rounds, "sweeps_per_round": K, "ms": round(ms_t, 2),
                               "rung_change_rate": round(moved, 4),
                               "vs_batched_sweeps": round(float(sites) * rounds * K / (ms_t * 1e-3) / 1e9 / g_b, 3)}
    del tb, trec, trung
    torch.cuda.empty_cache()

    # FP16 vs FP32 storage at L = 8192
    pc = workloads.PRECISION
    res = {}
    for prec in ("fp32", "fp16"):
        scratch = xy.Lattice(pc["L"], seed=pc["seed"] + 1000, beta=1.0, delta=pc["delta"], precision=prec)
        tuned_x = scratch.autotune(20)
        del scratch
        lt = xy.Lattice(pc["L"], seed=pc["seed"], beta=1.0, delta=pc["delta"], precision=prec, plan=tuned_x)
        lt.sweep(20)
        ms_x = timed(lambda: lt.sweep(200, 10), stream)
        res[prec] = round(float(pc["L"]) ** 2 * 200 / (ms_x * 1e-3) / 1e9, 2)
        del lt
    ex["L8192_storage_gupd_s"] = res
    # algorithmic bytes of a fused sweep: 8 B per update in FP32, 4 B in FP16
    ex["L8192_storage_alg_GBps"] = {"fp32": round(res["fp32"] * 8.0, 1), "fp16": round(res["fp16"] * 4.0, 1)}

    # four replicas of L = 4096 in one float4 state vs the same four as single lattices
    qc = workloads.QUAD_4096
    qd = xy.Quad(qc["L"], qc["seeds"], qc["betas"], [qc["delta"]] * 4)
    qd.sweep(10, 10)
    qobs = torch.empty((qc["sweeps"] // qc["measure_every"], 4, 8), dtype=torch.float64, device="cuda")
    ms_q = timed(lambda: qd.sweep(qc["sweeps"], qc["measure_every"], out=qobs), stream)
    tile_q = qd.tile
    del qd, qobs
    singles = [xy.Lattice(qc["L"], seed=s_, beta=b_, delta=qc["delta"], plan=main_plan)
               for s_, b_ in zip(qc["seeds"], qc["betas"])]
    for lt in singles:
        lt.sweep(10, 10)

    def four_singles():
        for lt in singles:
            lt.sweep(qc["sweeps"], qc["measure_every"])
    ms_s = timed(four_singles, stream)
    del singles
    torch.cuda.empty_cache()
    upd = 4.0 * qc["L"] ** 2 * qc["sweeps"]
    ex["quad_L4096"] = {"gupd_s": round(upd / (ms_q * 1e-3) / 1e9, 2), "tile": list(tile_q),
                        "alg_GBps_8B": round(upd / (ms_q * 1e-3) / 1e9 * 8.0, 1),
                        "four_single_lattices_gupd_s": round(upd / (ms_s * 1e-3) / 1e9, 2),
                        "sweeps": qc["sweeps"], "betas": qc["betas"]}

    # HMC on the four-replica texel (a vector of four accept decisions) against the
    # same trajectories of the four single lattices
    ex["quad_hmc_L4096"] = quad_hmc_leg(stream)

    # batched HMC over the temperature scan (one accept per lattice) against the
    # same trajectories run lattice by lattice
    hb = workloads.HMC_SCAN
    sc = workloads.temperature_scan()
    sites = sum(L * L for L in sc["Ls"])
    bh = xy.Batch(sc["Ls"], sc["seeds"], sc["betas"], sc["deltas"])
    bh.sweep(hb["therm"])
    bh.hmc(1, hb["n_md"], hb["eps"])
    hout = torch.empty((len(sc["Ls"]), hb["traj"], 9), dtype=torch.float64, device="cuda")
    ms_bh = timed(lambda: bh.hmc(hb["traj"], hb["n_md"], hb["eps"], out=hout), stream)
    rbh = xy.hmc_records(hout)
    del bh
    torch.cuda.empty_cache()
    singles = [xy.Lattice(L, seed=s_, beta=b_, delta=1.0) for L, s_, b_ in zip(sc["Ls"], sc["seeds"], sc["betas"])]
    for lt in singles:
        lt.sweep(hb["therm"])
        lt.hmc(1, hb["n_md"], hb["eps"])
    ntr = hb["traj_per_lattice_timed"]

    def hmc_singles():
        for lt in singles:
            lt.hmc(ntr, hb["n_md"], hb["eps"])
    ms_sh = timed(hmc_singles, stream)
    del singles
    torch.cuda.empty_cache()
    g_bh = float(sites) * hb["n_md"] * hb["traj"] / (ms_bh * 1e-3) / 1e9
    g_sh = float(sites) * hb["n_md"] * ntr / (ms_sh * 1e-3) / 1e9
    ex["hmc_batch_scan_96"] = {"g_site_steps_s": round(g_bh, 2), "trajectories": hb["traj"], "n_md": hb["n_md"],
                               "eps": hb["eps"], "ms": round(ms_bh, 2),
                               "accept_rate": round(float(rbh["accepted"].mean()), 3),
                               "per_lattice_g_site_steps_s": round(g_sh, 2), "speedup": round(g_bh / g_sh, 2)}

    # hybrid Monte Carlo trajectories (the paper's update)
    for name, hc in (("hmc_L4096", workloads.HMC_4096), ("hmc_L16384", workloads.HMC_16384)):
        lt = xy.Lattice(hc["L"], seed=hc["seed"], beta=hc["beta"])
        lt.sweep(hc["therm"])
        lt.hmc(2, hc["n_md"], hc["eps"])
        out = torch.empty((hc["traj"], 9), dtype=torch.float64, device="cuda")
        ms_h = timed(lambda: lt.hmc(hc["traj"], hc["n_md"], hc["eps"], out=out), stream)
        r = xy.hmc_records(out)
        steps = float(hc["L"]) ** 2 * hc["n_md"] * hc["traj"]
        g_s = steps / (ms_h * 1e-3) / 1e9
        # algorithmic bytes per site of one trajectory: momenta and saved angles
        # (read 4, write 8), ceil(n_md / k) passes of angle + momentum read and
        # written (16 B each), the final half kick (read 8, plus the angle written
        # back into the state, 4, when the pass count is odd)
        k = lt.hmc_steps_per_pass
        passes = -(-hc["n_md"] // k)
        traj_bytes = 12.0 + ALG_BYTES_HMC_STEP * passes + 8.0 + (4.0 if passes % 2 else 0.0)
        gbs = float(hc["L"]) ** 2 * traj_bytes * hc["traj"] / (ms_h * 1e-3) / 1e9
        ex[name] = {"g_site_steps_s": round(g_s, 2), "trajectories": hc["traj"], "n_md": hc["n_md"],
                    "eps": hc["eps"], "ms": round(ms_h, 2), "accept_rate": round(float(r["accepted"].mean()), 3),
                    "mean_dH": round(float(r["dH"].mean()), 4), "steps_per_pass": k,
                    "alg_bytes_per_site_traj": traj_bytes, "hbm_GBps": round(gbs, 1),
                    "frac_hbm": round(gbs / HBM_PEAK_GBS, 4)}
        del lt, out
        torch.cuda.empty_cache()
    return ex


def quad_hmc_leg(stream, singles=True):
    import torch

    from paper_0811_2111_amd import workloads, xy
    hc = workloads.QUAD_HMC_4096
    qd = xy.Quad(hc["L"], hc["seeds"], hc["betas"])
    qd.sweep(hc["therm"])
    qd.hmc(1, hc["n_md"], hc["eps"])
    out = torch.empty((hc["traj"], 4, 9), dtype=torch.float64, device="cuda")
    ms_q = timed(lambda: qd.hmc(hc["traj"], hc["n_md"], hc["eps"], out=out), stream)
    r = xy.hmc_records(out)
    k = qd.hmc_steps_per_pass
    del qd
    torch.cuda.empty_cache()
    steps = 4.0 * float(hc["L"]) ** 2 * hc["n_md"] * hc["traj"]
    # algorithmic bytes per replica site of a trajectory: the begin (read 4, write
    # 8), ceil(n_md / k) passes of angle + momentum read and written (16 B), the
    # end (read 8, plus the angles written back, 4, when the pass count is odd)
    passes = -(-hc["n_md"] // k)
    traj_bytes = 12.0 + ALG_BYTES_HMC_STEP * passes + 8.0 + (4.0 if passes % 2 else 0.0)
    gbs = 4.0 * float(hc["L"]) ** 2 * traj_bytes * hc["traj"] / (ms_q * 1e-3) / 1e9
    res = {"g_replica_site_steps_s": round(steps / (ms_q * 1e-3) / 1e9, 2), "trajectories": hc["traj"],
           "n_md": hc["n_md"], "eps": hc["eps"], "betas": hc["betas"], "ms": round(ms_q, 2),
           "accept_rate": round(float(r["accepted"].mean()), 3), "steps_per_pass": k,
           "alg_bytes_per_replica_site_traj": traj_bytes,
           "hbm_GBps": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBS, 4)}
    if singles:
        lats = [xy.Lattice(hc["L"], seed=s_, beta=b_) for s_, b_ in zip(hc["seeds"], hc["betas"])]
        for lt in lats:
            lt.sweep(hc["therm"])
            lt.hmc(1, hc["n_md"], hc["eps"])

        def four():
            for lt in lats:
                lt.hmc(hc["traj"], hc["n_md"], hc["eps"])
        ms_s = timed(four, stream)
        res["four_single_lattices_g_site_steps_s"] = round(steps / (ms_s * 1e-3) / 1e9, 2)
        del lats
        torch.cuda.empty_cache()
    return res


def cpu_baseline(cfg, sweeps):
    """The FP64 C oracle as it stands (single-threaded) on `sweeps` sweeps of the
    same lattice from its hot start; only the sweeps are timed."""
    import oracle
    L = cfg["L"]
    th = oracle.hot_start(cfg["seed"], L, "f32")
    t0 = time.perf_counter()
    oracle.run(cfg["seed"], th, cfg["beta"], cfg["delta"], sweeps, 0, prec="f32")
    dt = time.perf_counter() - t0
    n, model = host_cpu()
    return {"value": round(float(L) * L * sweeps / dt / 1e9, 6), "unit": "Gupd/s", "cores": 1, "kind": "oracle",
            "sample": "%d sweep(s) of the L=%d lattice (beta=%g, delta=%g) from its hot start, %.1f s on one core"
                      % (sweeps, L, cfg["beta"], cfg["delta"], dt),
            "host_cpus": n, "cpu_model": model}


if __name__ == "__main__":
    main()
