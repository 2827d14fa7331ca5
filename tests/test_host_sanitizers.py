"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the planner (parsing, loss cases, lowering, geometry, index tables) built
with g++ -fsanitize=address,undefined and driven over valid, malformed and
random model strings by csrc/host_check/planner_check.cpp."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2602_02759_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ is not available")
def test_planner_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "planner_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", CSRC, os.path.join(CSRC, "host_check", "planner_check.cpp"),
           os.path.join(CSRC, "planner.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failed checks" in r.stdout
