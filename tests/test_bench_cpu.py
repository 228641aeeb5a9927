"""The benchmark's host-side pieces: the roofline arithmetic, the oracle baseline leg on a
small sample, and the refusal of more than one GPU."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_roofline_fraction():
    r = bench.roofline(nodes=10 ** 6, bytes_per_node=68, ms=0.0085)   # 68 MB in 8.5 us
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert abs(r["achieved"] - 8000.0) < 0.1 and abs(r["frac"] - 1.0) < 1e-4


def test_cpu_baseline_reports_the_oracle():
    out = bench.cpu_baseline(n=64, steps=20)
    assert out["kind"] == "oracle" and out["unit"] == "MLUPS"
    assert out["value"] > 0 and out["cores"] >= 1 and "64x64" in out["sample"]


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr and p.stdout == ""
