"""The host-side plan builder (csrc/plan.cpp) under AddressSanitizer and
UndefinedBehaviorSanitizer: tests/host/plan_check.cpp builds plans for edge
cases, random batches and a batch wide enough for the stage and combine
buckets, under every multiplier option and scan schedule, and checks the
invariants of their workspace maps, schedules and launch orders.  Host code
only (g++), no device."""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2407_05433_amd", "csrc")
ROCM_INCLUDE = "/opt/rocm/include"


def test_plan_builder_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.isdir(os.path.join(ROCM_INCLUDE, "hip")):
        pytest.skip("g++ or the HIP headers are not available")
    exe = str(tmp_path / "plan_check")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__", "-I" + ROCM_INCLUDE, "-I" + os.path.join(ROOT, "include"),
           "-I" + CSRC, os.path.join(CSRC, "plan.cpp"), os.path.join(HERE, "host", "plan_check.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
    assert "0 failures" in r.stdout, out[-2000:]
