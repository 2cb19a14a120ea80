"""Host-side logic of bench.py (no GPU): the one-GPU refusal and the counter-traffic lookup that
feeds roofline.traffic, which must apply only to the kernel source the counters were taken on."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr + r.stdout
    assert r.stdout.strip() == ""   # no JSON line


def test_traffic_uses_the_committed_counters_for_this_source(monkeypatch):
    with open(os.path.join(ROOT, "profiles", "pmc_traffic.json")) as f:
        doc = json.load(f)
    name, k = next(iter(sorted(doc["kernels"].items())))
    if doc["source_sha"] != bench.kernel_source_sha():
        # counters taken on another version of the kernels do not apply
        assert bench.measured_traffic(name, 10.0) == (None, None)
        monkeypatch.setattr(bench, "kernel_source_sha", lambda: doc["source_sha"])
    gbs, per_launch = bench.measured_traffic(name, 10.0)
    want = 1024.0 * (k["fetch_kib"] * doc["copy_factor_fetch"] + k["write_kib"] * doc["copy_factor_write"])
    assert per_launch == want
    assert abs(gbs - want / 10e-6 / 1e9) <= 1e-9 * gbs
    # the calibration is a plain copy: fetched KiB are half the copy's bytes, written KiB all of them
    assert abs(doc["copy_factor_fetch"] - 2.0) < 0.01 and abs(doc["copy_factor_write"] - 1.0) < 0.01


def test_traffic_is_null_for_other_sources_and_unknown_kernels(monkeypatch):
    assert bench.measured_traffic("no_such_kernel", 10.0) == (None, None)
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: "0000000000000000")
    with open(os.path.join(ROOT, "profiles", "pmc_traffic.json")) as f:
        name = next(iter(json.load(f)["kernels"]))
    assert bench.measured_traffic(name, 10.0) == (None, None)
