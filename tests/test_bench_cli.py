"""bench.py's command-line contract that holds without a GPU: more than one
GPU is refused with a JSON error line and exit status 2, and so is a run on
a machine with no GPU visible (never a silent CPU fallback)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*args):
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                       capture_output=True, text=True, cwd=ROOT, timeout=300)
    return p.returncode, p.stdout.strip().splitlines()


def test_more_than_one_gpu_is_refused():
    rc, lines = run_bench("--gpus", "2")
    assert rc == 2
    msg = json.loads(lines[-1])
    assert "one GPU" in msg["error"]


def test_no_gpu_is_an_error_not_a_fallback():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    rc, lines = run_bench("--steps", "1", "--warmup", "0", "--no-cpu-baseline")
    assert rc == 2
    assert json.loads(lines[-1]) == {"error": "no GPU visible"}
