"""Host-side logic of bench.py (no GPU): the one-GPU refusal, the committed
traffic summaries it reads for the roofline's `traffic`, and the algorithmic
bytes those summaries quote (16 B per region-box cell loaded, 16 B per owned
cell merged, summed over a launch's tiles)."""
import json
import math
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_cs_0502039_amd import workloads  # noqa: E402

PROFILES = [w for w in ("square_4096", "cubic_256")
            if os.path.exists(os.path.join(ROOT, "profiles", f"traffic_{w}.json"))]


def load_profile(workload):
    with open(os.path.join(ROOT, "profiles", f"traffic_{workload}.json")) as f:
        return json.load(f)


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("workload", PROFILES)
def test_traffic_entries_are_the_scaled_counters(workload):
    doc = load_profile(workload)
    cal = doc["copy_calibration"]
    # the copy kernel reads and writes the same bytes once
    assert cal["fetch_kib"] * cal["fetch_scale"] == pytest.approx(cal["bytes"] / 1024, rel=1e-3)
    assert cal["write_kib"] * cal["write_scale"] == pytest.approx(cal["bytes"] / 1024, rel=1e-3)
    for e in doc["entries"]:
        hbm = 1024 * (e["fetch_kib_per_launch"] * cal["fetch_scale"] +
                      e["write_kib_per_launch"] * cal["write_scale"])
        assert e["hbm_bytes_per_launch"] == pytest.approx(hbm, rel=1e-4)


@pytest.mark.parametrize("workload", PROFILES)
def test_algorithmic_bytes_follow_the_tile_partition(workload):
    """Per direction the lattice is cut into ceil(L / tile) tiles, each loaded
    with `ghost` cells and a one-cell frozen ring on both sides."""
    doc = load_profile(workload)
    L = getattr(workloads, workload)()["L"]
    for e in doc["entries"]:
        t = e["tuning"]
        ntiles, box = 1, 1
        for d, side in enumerate(L):
            n = math.ceil(side / t["tile"][d])
            ntiles *= n
            box *= side + n * (2 * t["ghost"][d] + 2)
        assert e["tiles"] == ntiles
        assert e["algorithmic_bytes_per_launch"] == 16 * box + 16 * math.prod(L)


@pytest.mark.parametrize("workload", PROFILES)
def test_measured_traffic_needs_matching_sources_and_schedule(workload, tmp_path, monkeypatch):
    doc = load_profile(workload)
    entry = doc["entries"][0]
    fresh = doc["kernel_source_sha256"] == bench.kernel_source_digest()
    got = bench.measured_traffic(workload, entry["tuning"])
    assert got == (entry["hbm_bytes_per_launch"] if fresh else None)
    # another block size or tile shape: counters taken on another kernel launch
    other = dict(entry["tuning"], block=entry["tuning"]["block"] // 2)
    assert bench.measured_traffic(workload, other) is None
    other = dict(entry["tuning"], tile=[x + 1 for x in entry["tuning"]["tile"]])
    assert bench.measured_traffic(workload, other) is None
    # a copy of the tree whose visit sources differ from the profiled ones
    root = tmp_path / "repo"
    shutil.copytree(os.path.join(ROOT, "profiles"), root / "profiles")
    shutil.copytree(os.path.join(ROOT, "paper_cs_0502039_amd", "csrc"),
                    root / "paper_cs_0502039_amd" / "csrc")
    monkeypatch.setattr(bench, "ROOT", str(root))
    before = bench.kernel_source_digest()
    src = root / "paper_cs_0502039_amd" / "csrc" / bench.VISIT_SOURCES[0]
    src.write_text(src.read_text() + "\n")
    assert bench.kernel_source_digest() != before
    assert bench.measured_traffic(workload, entry["tuning"]) is None
    # with the digest of the edited sources the entry is found again
    doc["kernel_source_sha256"] = bench.kernel_source_digest()
    (root / "profiles" / f"traffic_{workload}.json").write_text(json.dumps(doc))
    assert bench.measured_traffic(workload, entry["tuning"]) == entry["hbm_bytes_per_launch"]
