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


def _csv(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        f.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for i, (k, c, v) in enumerate(rows):
            f.write(f'{i},"{k}",{c},{v}\n')


def test_counter_summary_scales_by_the_copy_and_drops_returned_launches(tmp_path):
    """--summarize-counters: per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) of the
    dominant kernel, scaled by what the same counter reads for the 512 MiB
    copy, averaged over the launches that did work."""
    import json
    kern = "k_arn_project<double, float>"
    name = f"sd::(anonymous namespace)::{kern}(sd::Sell<double>, float const*)"
    copy_kib = 512 * 1024
    _csv(str(tmp_path / "f" / "host" / "1_run_counter_collection.csv"),
         [(name, "FETCH_SIZE", 1000.0), (name, "FETCH_SIZE", 3000.0),
          (name, "FETCH_SIZE", 0.5), ("__amd_rocclr_copyBuffer", "FETCH_SIZE", copy_kib / 2)])
    _csv(str(tmp_path / "w" / "host" / "1_run_counter_collection.csv"),
         [(name, "WRITE_SIZE", 100.0), (name, "WRITE_SIZE", 100.0), (name, "WRITE_SIZE", 0.0),
          ("__amd_rocclr_copyBuffer", "WRITE_SIZE", copy_kib)])
    run = {"config": "C2", "precision": "mixed", "kernel": kern, "launches": 2,
           "alg_bytes_per_launch": 2.0e6, "copy_bytes": copy_kib * 1024,
           "kernels_hip_sha256": "x"}
    with open(tmp_path / "run.json", "w") as f:
        json.dump(run, f)
    out = tmp_path / "traffic.json"
    r = _run("--summarize-counters", str(tmp_path / "f"), str(tmp_path / "w"),
             "--counter-out", str(tmp_path / "run.json"), "--traffic-out", str(out))
    assert r.returncode == 0, r.stderr
    t = json.load(open(out))
    assert t["fetch_launches_counted"] == 2 and t["write_launches_counted"] == 2
    assert abs(t["fetch_scale"] - 2.0) < 1e-12 and abs(t["write_scale"] - 1.0) < 1e-12
    assert abs(t["fetch_bytes_per_launch"] - 2000.0 * 1024 * 2) < 1e-6
    assert abs(t["hbm_bytes_per_launch"] - (4096000.0 + 102400.0)) < 1e-6
    assert t["kernel"] == kern
