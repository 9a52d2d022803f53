"""Host logic of bench.py on the CPU: the one-GPU limit and the rule that the
measured HBM traffic is reported only while the kernel sources match the ones
the counters were taken from."""
import hashlib
import json
import os
import shutil
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def _fake_root(tmp_path, traffic=12345):
    srcs = ["a/kernel.hip", "a/steps.h"]
    h = hashlib.sha1()
    for i, s in enumerate(srcs):
        p = tmp_path / s
        p.parent.mkdir(parents=True, exist_ok=True)
        p.write_bytes(f"source {i}\n".encode())
        h.update(p.read_bytes())
    (tmp_path / "profiles").mkdir()
    rec = {"sources": srcs, "sources_sha1": h.hexdigest(), "traffic_bytes": traffic + 0.4}
    (tmp_path / "profiles" / "region_melded_traffic.json").write_text(json.dumps(rec))
    return srcs


def test_traffic_reported_while_sources_match(tmp_path, monkeypatch):
    srcs = _fake_root(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench._measured_traffic() == 12345
    # any edit of a listed source voids the record
    (tmp_path / srcs[1]).write_bytes(b"edited\n")
    assert bench._measured_traffic() is None


def test_traffic_missing_record_or_source_is_none(tmp_path, monkeypatch):
    srcs = _fake_root(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.remove(tmp_path / srcs[0])
    assert bench._measured_traffic() is None
    shutil.rmtree(tmp_path / "profiles")
    assert bench._measured_traffic() is None


def test_committed_record_names_existing_sources():
    with open(os.path.join(ROOT, "profiles", "region_melded_traffic.json")) as f:
        rec = json.load(f)
    assert rec["kernel"] == "region_melded_kernel"
    assert all(os.path.exists(os.path.join(ROOT, s)) for s in rec["sources"])
    assert rec["traffic_bytes"] > 0 and rec["fetch_factor"] > 0 and rec["write_factor"] > 0
