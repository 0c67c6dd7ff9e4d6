"""The benchmark's command-line contract, on the CPU: it runs on one GPU only and
says so when asked for more, before touching any device."""
from __future__ import annotations

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_help_lists_the_profile_legs():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0
    for leg in ("l4096", "l16384", "batch", "hmc", "quad", "fp16", "tempering", "small"):
        assert leg in r.stdout


def _bench_module():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_traffic_is_reported_only_for_the_profiled_kernel_sources(tmp_path):
    """The roofline's `traffic` comes from the counter profile only while the
    kernel sources hash as they did when the counters were taken."""
    import json
    b = _bench_module()
    entry = {"bytes_per_launch": 123.0}
    good = {"kernel_sources_sha256": b.kernel_sources_hash(), "entries": {"4096/256,16,1": entry}}
    stale = dict(good, kernel_sources_sha256="0" * 64)
    for doc, plan, want in [(good, (2, 256, 16, 1), 123.0), (good, (2, 128, 32, 1), None),
                            (good, (3, 256, 16, 1), None), (stale, (2, 256, 16, 1), None)]:
        f = tmp_path / "traffic.json"
        f.write_text(json.dumps(doc))
        b.TRAFFIC_FILE = str(f)
        assert b.measured_traffic(4096, plan) == want, (plan, doc is good)
