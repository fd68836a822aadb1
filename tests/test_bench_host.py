"""Host-only checks of the benchmark script: the one-GPU guard, the committed
counter summary against the kernel sources, and the counter arithmetic on small
synthetic rocprofv3 tables."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_committed_counters_and_the_kernel_sources():
    """The bench reports the committed traffic only while the counters were taken
    on the current kernel sources; then every input byte was read once."""
    d = json.load(open(bench.COUNTERS_JSON))
    if d["kernel_hash"] != bench.kernel_hash():
        assert bench.traffic_from_profiles(d["algorithmic_bytes_per_launch"]) is None
        assert bench.utilisation_from_profiles(0.16) is None
        return
    assert d["kernel"] == "hp::k_nest_f32_lean<4>"
    # every input byte read once: traffic within 1 % above the algorithmic bytes
    assert 1.0 <= d["traffic_over_algorithmic"] < 1.01
    assert bench.traffic_from_profiles(d["algorithmic_bytes_per_launch"]) == d["traffic_bytes_per_launch"]
    u = bench.utilisation_from_profiles(0.16)
    assert u is not None and 0.0 < u["valu_share"] < 1.0


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, grid, value in rows:
            w.writerow({"Kernel_Name": name, "Grid_Size": grid, "Counter_Name": counter, "Counter_Value": value})


def test_counter_scaling(tmp_path, monkeypatch):
    """FETCH_SIZE is scaled by what it reads for the 1 GiB copy (here half of it,
    so scale 2), WRITE_SIZE likewise (here all of it, scale 1); the largest copy
    dispatch is taken as the calibration copy."""
    out = tmp_path / "counters.json"
    monkeypatch.setattr(bench, "COUNTERS_JSON", str(out))
    kern = "void hp::k_nest_f32_lean<4>(hp::DevPlan const*, float const*, void*, unsigned char*)"
    copy = "__amd_rocclr_copyBuffer"
    f, w = tmp_path / "fetch.csv", tmp_path / "write.csv"
    _counter_csv(f, "FETCH_SIZE", [(kern, 2097152, 1000.0), (kern, 2097152, 1002.0), (copy, 1024, 3.0),
                                   (copy, 2097152, 524288.0)])
    _counter_csv(w, "WRITE_SIZE", [(kern, 2097152, 8.0), (kern, 2097152, 8.0), (copy, 2097152, 1048576.0)])
    bench.ingest_counters(str(f), str(w), "k_nest_f32_lean<4>", 2_000_000)
    d = json.load(open(out))
    assert d["counters"]["FETCH_SIZE"]["scale"] == 2.0
    assert d["counters"]["FETCH_SIZE"]["bytes_per_launch"] == 1001 * 1024 * 2
    assert d["counters"]["WRITE_SIZE"]["scale"] == 1.0
    assert d["counters"]["WRITE_SIZE"]["bytes_per_launch"] == 8 * 1024
    assert d["traffic_bytes_per_launch"] == 1001 * 1024 * 2 + 8 * 1024
    assert d["kernel_hash"] == bench.kernel_hash()


def test_counter_ingest_needs_the_calibration_copy(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "COUNTERS_JSON", str(tmp_path / "counters.json"))
    f, w = tmp_path / "fetch.csv", tmp_path / "write.csv"
    _counter_csv(f, "FETCH_SIZE", [("k_nest_f32_lean<4>", 64, 1.0)])
    _counter_csv(w, "WRITE_SIZE", [("k_nest_f32_lean<4>", 64, 1.0)])
    with pytest.raises(SystemExit):
        bench.ingest_counters(str(f), str(w), "k_nest_f32_lean<4>", 100)
    assert not (tmp_path / "counters.json").exists()


def test_percentiles():
    xs = list(range(1, 101))
    assert bench.pct(xs, 50) == 50
    assert bench.pct(xs, 99) == 99
    assert bench.pct(xs, 100) == 100
    assert bench.pct([7.0], 99) == 7.0
