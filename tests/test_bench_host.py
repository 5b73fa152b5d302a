"""Host-side pieces of bench.py (no GPU): the roofline arithmetic, the gate on
the committed traffic figure, and the one-GPU limit of the command line."""
import hashlib
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_roofline_counts_flop_per_pair_and_per_source_point():
    b = load_bench()
    # 1000 launches of 2e6 pairs over 30000 source points each, 20 ms of kernel time in all
    prof = {"pair_kernel_ms": 20.0, "launches": 1000, "pairs": 2_000_000_000, "source_points": 30_000_000}
    r = b.roofline(prof)
    flop = 76 * 2e9 + 230 * 3e7
    assert r["achieved"] == pytest.approx(flop / 0.020 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / 157.3)
    assert r["avg_launch_us"] == pytest.approx(20.0)
    assert r["pairs_per_launch"] == pytest.approx(2e6)
    assert r["kernel_pairs_per_s"] == pytest.approx(2e9 / 0.020)
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s" and r["peak"] == 157.3
    assert b.roofline({"pair_kernel_ms": 0.0, "launches": 0, "pairs": 0, "source_points": 0})["achieved"] == 0.0


def test_traffic_reported_only_for_the_profiled_sources_and_cell_shape(tmp_path, monkeypatch):
    b = load_bench()
    text = open(b.HBM_PROFILE).read()
    vals = dict(line.split(":", 1) for line in text.splitlines() if ":" in line and not line.startswith("#"))
    shape = tuple(float(v) for v in vals["cell_fraction"].split())
    pkg = os.path.join(ROOT, "paper_2606_10019_amd")
    digest = hashlib.sha256(b"".join(open(os.path.join(pkg, f), "rb").read() for f in b.KERNEL_SOURCES)).hexdigest()
    expect = float(vals["traffic_bytes_per_launch"]) if vals["sources_sha256"].strip() == digest else None
    assert b.measured_traffic(shape) == expect
    assert b.measured_traffic((shape[0], shape[1] / 2)) is None          # another cell shape
    stale = tmp_path / "hbm.txt"
    stale.write_text(text.replace(vals["sources_sha256"].strip(), "0" * 64))
    monkeypatch.setattr(b, "HBM_PROFILE", str(stale))
    assert b.measured_traffic(shape) is None                              # other sources
    monkeypatch.setattr(b, "HBM_PROFILE", str(tmp_path / "missing.txt"))
    assert b.measured_traffic(shape) is None


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
