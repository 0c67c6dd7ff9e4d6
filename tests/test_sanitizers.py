"""Memory and undefined-behaviour checks of the host code, on the CPU.

* The oracle (oracle/*.c) is rebuilt with gcc's AddressSanitizer and
  UndefinedBehaviorSanitizer and its pin tests run against that build (the
  sanitizer runtimes preloaded into the test process).
* The host runtime (csrc/xy_runtime.cpp: argument validation, workspace
  carve-up, plan choice and the tune-cache parser) is rebuilt host-only with the
  same sanitizers, linked with the library's normal kernel objects, and the
  library's CPU tests run against that build.
A sanitizer report fails the run (UBSan halts on the first error; leak checks
are off, since the Python interpreter itself is not instrumented).
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_0811_2111_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ENV_SAN = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:halt_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _run_pytest(files, extra_env):
    env = dict(os.environ)
    env.update(ENV_SAN)
    env.update(extra_env)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu"]
                       + files, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    return out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_pins_under_asan_ubsan(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    srcs = sorted(glob.glob(os.path.join(ROOT, "oracle", "*.c")))
    subprocess.run(["gcc", "-O1", "-g", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                    "-o", lib] + srcs + ["-lm"], check=True)
    undef = subprocess.run(["nm", "-u", lib], capture_output=True, text=True, check=True).stdout
    assert "__asan_report" in undef and "__ubsan_handle" in undef      # really instrumented
    pre = ":".join(subprocess.run(["gcc", "-print-file-name=" + n], capture_output=True, text=True,
                                  check=True).stdout.strip() for n in ("libasan.so", "libubsan.so"))
    out = _run_pytest(["tests/test_oracle_pins.py", "tests/test_hmc_pins.py", "tests/test_pt_pins.py"],
                      {"LD_PRELOAD": pre, "XY_ORACLE_LIB": lib})
    assert " passed" in out


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_host_runtime_under_asan_ubsan(tmp_path):
    objs = [o for o in glob.glob(os.path.join(ROOT, "paper_0811_2111_amd", "_build", "*.o"))
            if not os.path.basename(o).startswith("xy_runtime")]
    if not objs:
        pytest.skip("the library's objects are not built (run __graft_entry__.build())")
    rt = str(tmp_path / "xy_runtime_san.o")
    lib = str(tmp_path / "libxyhip_san.so")
    subprocess.run([HIPCC, "-x", "hip", "--cuda-host-only", "-O1", "-g", "-std=c++17", "-fPIC",
                    "-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-omit-frame-pointer",
                    "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c", os.path.join(CSRC, "xy_runtime.cpp"),
                    "-o", rt], check=True, capture_output=True)
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address,undefined",
                    "-o", lib, rt] + objs, check=True, capture_output=True)
    undef = subprocess.run(["nm", rt], capture_output=True, text=True, check=True).stdout
    assert "__asan_report" in undef and "__ubsan_handle" in undef
    rts = glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not rts:
        pytest.skip("clang's ASan runtime not found")
    out = _run_pytest(["tests/test_library_cpu.py"], {"LD_PRELOAD": rts[0], "XY_LIB": lib})
    assert " passed" in out
