"""CPU checks of bench.py's host logic: the HBM-traffic figure of the
roofline object is taken from the committed rocprofv3 counter summary of the
run's dominant kernel, scaled by the copy calibration, and only while that
kernel's sources still hash to the recorded value; runs on more than one GPU
are refused."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _summary(prec, L):
    path = os.path.join(ROOT, "profiles", f"{bench.KERNELS[prec][0]}_{prec}_lattice{L}_pmc.txt")
    kv = {}
    for line in open(path):
        parts = line.split()
        if len(parts) == 2 and not line.startswith("#"):
            kv[parts[0]] = parts[1]
    return kv


def test_traffic_from_summary(monkeypatch):
    kv = _summary("fp64", 20)
    monkeypatch.setattr(bench, "kernel_source_hash", lambda prec="fp64": kv["source_sha256"])
    want = (float(kv["fetch_kib_per_launch"]) * float(kv["fetch_factor"])
            + float(kv["write_kib_per_launch"]) * float(kv["write_factor"])) * 1024.0
    got = bench.traffic_per_launch("fp64", 20)
    assert got == round(want)
    # the copy calibration is close to 2 for FETCH_SIZE and 1 for WRITE_SIZE
    assert 1.9 < float(kv["fetch_factor"]) < 2.1 and float(kv["write_factor"]) == 1.0


def test_traffic_null_when_sources_changed(monkeypatch):
    monkeypatch.setattr(bench, "kernel_source_hash", lambda prec="fp64": "0" * 64)
    assert bench.traffic_per_launch("fp64", 20) is None


def test_traffic_null_without_summary():
    assert bench.traffic_per_launch("fp64", 7) is None


def test_dominant_kernel_sources_exist():
    for prec, (name, srcs) in bench.KERNELS.items():
        for f in srcs:
            assert os.path.exists(os.path.join(ROOT, f)), (prec, f)
        assert len(bench.kernel_source_hash(prec)) == 64


def test_more_than_one_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)
