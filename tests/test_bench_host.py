"""Host-side logic of bench.py (no GPU): the one-GPU guard, the staleness
check of the committed HBM counters, and the one-thread limit of the oracle
timings."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_committed_counters_match_the_sources():
    """The committed counter file names the source hash it was taken on; the
    benchmark reports its traffic only while that hash is current."""
    with open(bench.TRAFFIC_FILE) as fh:
        t = json.load(fh)
    assert t["kernel"] == bench.SWEEP_KERNEL
    for rec in t["records"]:
        w = rec["workload"]
        assert bench.measured_traffic(w["domain"], w["N"]) == (
            rec["bytes_per_launch"] if t["source_hash"] == bench.source_hash() else None)


def test_counters_of_another_workload_give_no_traffic(monkeypatch, tmp_path):
    with open(bench.TRAFFIC_FILE) as fh:
        t = json.load(fh)
    t["source_hash"] = bench.source_hash()
    t["records"] = [{"workload": {"domain": "flower", "N": 4096}, "bytes_per_launch": 1.0}]
    p = tmp_path / "traffic.json"
    p.write_text(json.dumps(t))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(p))
    assert bench.measured_traffic("flower", 4096) == 1.0
    assert bench.measured_traffic("flower", 16384) is None
    assert bench.measured_traffic("ellipse", 4096) is None


def test_stale_counters_give_no_traffic(monkeypatch, tmp_path):
    with open(bench.TRAFFIC_FILE) as fh:
        t = json.load(fh)
    t["source_hash"] = "0" * 16
    p = tmp_path / "traffic.json"
    p.write_text(json.dumps(t))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(p))
    assert bench.measured_traffic() is None


def test_source_hash_ignores_comments(monkeypatch, tmp_path):
    src = os.path.join(ROOT, "paper_2505_05105_amd", "csrc")
    d = tmp_path / "paper_2505_05105_amd" / "csrc"
    d.mkdir(parents=True)
    for name in ("smoother.hip", "mgfem_internal.h"):
        with open(os.path.join(src, name)) as fh:
            (d / name).write_text(fh.read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.source_hash()
    (d / "smoother.hip").write_text((d / "smoother.hip").read_text() + "\n// a comment\n/* another */\n")
    assert bench.source_hash() == h0
    (d / "smoother.hip").write_text((d / "smoother.hip").read_text() + "\nint extra_symbol;\n")
    assert bench.source_hash() != h0


def test_oracle_timings_run_on_one_thread():
    threadpoolctl = pytest.importorskip("threadpoolctl")
    with bench._one_thread():
        info = threadpoolctl.threadpool_info()
        assert all(i["num_threads"] == 1 for i in info)
