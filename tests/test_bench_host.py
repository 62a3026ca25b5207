"""bench.py's host-side contract, without a GPU: more than one GPU is
refused with a message (this solver has no multi-GPU path), and without a
HIP device the benchmark stops with an error instead of falling back to the
CPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=300, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def test_no_device_no_fallback():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a HIP device is present")
    r = _run("--no-cpu", "--steps", "1", "--warmup", "0")
    assert r.returncode == 1
    assert "needs a HIP device" in r.stderr
    assert r.stdout.strip() == ""
