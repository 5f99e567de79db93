"""Host-side logic of bench.py (no GPU): the roofline arithmetic, the
counter records keyed by kernel and grid, the algorithmic work counts and
the command-line contract."""
import json
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

GRIDS = {"euler": (2048, 1024), "sw": (1024, 1024), "elastic": (2048, 2048),
         "psystem": (4800, 4800), "euler_axisym": (1280, 320), "sw_godunov": (1024, 1024),
         "sw_strang": (1024, 1024)}


def _labels():
    """Every kernel@grid key a bench line can look up."""
    out = {}
    for name, w in bench.WORKLOADS.items():
        nx, ny = GRIDS.get(name, (2048, 1024))
        for prec, bpc in w[3].items():
            key = f"{w[5].format(R=bench.KERNEL_PRECISION[prec])}@{nx}x{ny}"
            out[key] = (name, prec, bpc * nx * ny)
    return out


def test_counter_records_are_keyed_by_kernel_and_grid():
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        d = json.load(f)
    labels = _labels()
    assert len(set(labels)) == len(labels), "two bench lines share a counter key"
    assert re.fullmatch(r"[0-9a-f]{16}", d["source_hash"])
    for key, rec in d["kernels"].items():
        assert re.fullmatch(r".+@\d+x\d+", key), key
        assert key in labels, f"record {key} matches no bench line"
        _, _, alg = labels[key]
        # a launch moves at least its compulsory bytes and, with halos and
        # line granularity, not several times more
        assert rec["algorithmic_bytes_per_launch"] == round(alg)
        assert 0.9 * alg <= rec["bytes_per_launch"] <= 2.0 * alg, key
        assert os.path.exists(os.path.join(ROOT, "profiles", rec["profile"])), rec["profile"]


def test_counter_lookup_rejects_other_grids_and_stale_sources(monkeypatch):
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        d = json.load(f)
    key = next(iter(d["kernels"]))
    kernel, grid = key.split("@")
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: d["source_hash"])
    assert bench.measured_counters(key) == d["kernels"][key]
    assert bench.measured_counters(f"{kernel}@7x7") is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.measured_counters(key) is None


def test_roofline_is_the_hbm_fraction_of_the_average_launch(monkeypatch):
    monkeypatch.setattr(bench, "measured_counters", lambda key: None)
    cells = 2048 * 1024
    # 192 accepted + 4 rejected attempts of 3 launches in 45 ms
    r = dict(steps=192, rejected=4, gpu_ms=45.0, cells=cells, grid="2048x1024")
    out = bench.roofline(r, 3, 256 / 3, 1040.0, "k", "f64")
    launches = 3 * 196
    avg_s = 45e-3 / launches
    assert out["launches"] == launches
    assert out["avg_launch_us"] == pytest.approx(avg_s * 1e6, abs=0.01)
    gbs = 256 / 3 * cells / avg_s / 1e9
    assert out["bound"] == "hbm" and out["unit"] == "GB/s" and out["peak"] == 8000.0
    assert out["achieved"] == pytest.approx(gbs, abs=0.1)
    assert out["frac"] == pytest.approx(gbs / 8000.0, abs=1e-4)
    assert out["traffic"] is None and out["kernel"] == "k@2048x1024"
    assert out["alu"]["frac"] == pytest.approx(1040.0 * cells / avg_s / 1e12 / 78.6, abs=1e-4)


def test_measured_bound_compares_issue_with_hbm_busy(monkeypatch):
    cells = 1024 * 1024
    r = dict(steps=100, rejected=0, gpu_ms=100 * 50e-3, cells=cells, grid="1024x1024")
    # 50 us per launch: 200 MB of measured traffic is half of the 8 TB/s peak
    rec = dict(bytes_per_launch=200e6, valu_issue_share=0.3, profile="p.md")
    monkeypatch.setattr(bench, "measured_counters", lambda key: rec)
    out = bench.roofline(r, 1, 48, 554.0, "k", "f64")
    assert out["traffic"] == 200e6 and out["profile"] == "p.md"
    assert out["hbm_busy_measured"] == pytest.approx(0.5, abs=1e-3)
    assert out["bound_measured"] == "hbm"
    rec["valu_issue_share"] = 0.7
    assert bench.roofline(r, 1, 48, 554.0, "k", "f64")["bound_measured"] == "alu"


def test_weno_stage_flop_counts():
    assert bench.euler_stage_flops(5) == 1040.0
    # order 2r - 1: 8 edge pairs of candidates 2r(2r-1), indicators
    # r(r^2 + 3r - 4) and weights (48 at r = 4, else 11r + 2), plus 238
    for order, r in ((7, 4), (9, 5), (17, 9)):
        w = 48 if r == 4 else 11 * r + 2
        assert bench.euler_stage_flops(order) == 8 * (2 * r * (2 * r - 1) + r * (r * r + 3 * r - 4) + w) + 238


def test_default_steps_fill_whole_graphs():
    assert bench.DEFAULT_STEPS % 16 == 0
    for w in bench.WORKLOADS.values():
        if w[7] is not None:
            steps, warmup = w[7]
            assert steps % 16 == 0 and warmup % 16 == 0


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr or "single MI355X" in p.stderr
    assert p.stdout == ""
