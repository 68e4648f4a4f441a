"""The batched-launch planner (the host code that cuts interaction lists into
wave tasks, pairs, splits and deals them) built on its own with
AddressSanitizer and UndefinedBehaviorSanitizer, and run over random item
sets by tests/plan_check.cpp, which checks the invariants the batched kernels
rely on (every pair of every list computed exactly once, lane and slot
bounds, sublist order, error statuses)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_planner_invariants_under_sanitizers(tmp_path):
    exe = str(tmp_path / "plan_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_1203_4037_amd", "csrc"),
           os.path.join(ROOT, "tests", "plan_check.cpp"),
           os.path.join(ROOT, "paper_1203_4037_amd", "csrc", "planner.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert "planner checks passed" in r.stdout
