"""The host-only planning code (csrc/nfs_host.cpp, csrc/pair_plan.cpp) built
with g++ under AddressSanitizer and UndefinedBehaviorSanitizer and run
against tests/host/host_checks.cpp: descriptor validation, the stored-mode
set and tiled slot layout, the binning table, the workspace layout, the
pair launch groups and the twiddle table. CPU only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1209_3362_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_planning_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "host_checks")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
           os.path.join(ROOT, "tests", "host", "host_checks.cpp"),
           os.path.join(CSRC, "nfs_host.cpp"), os.path.join(CSRC, "pair_plan.cpp"),
           "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    p = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert p.returncode == 0, p.stdout + p.stderr
    assert "all host checks passed" in p.stdout
