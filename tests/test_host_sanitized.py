"""The host planning logic of the FP32 sweeps (paper_2412_08076_amd/csrc/rm_geometry.h:
window partitions with their halos, kernel configurations and tile tables) built with
AddressSanitizer and UndefinedBehaviorSanitizer and checked by tests/host/plan_check.cpp on
the CPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_plan_logic_under_sanitizers(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "plan_check")
    cmd = [cxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "paper_2412_08076_amd", "csrc"),
           os.path.join(ROOT, "tests", "host", "plan_check.cpp"), "-o", exe]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert run.returncode == 0, run.stderr[-4000:]
    assert "plan checks passed" in run.stdout
