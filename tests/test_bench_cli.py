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
    assert bench._measured_traffic("region_melded_traffic.json") == 12345
    # any edit of a listed source voids the record
    (tmp_path / srcs[1]).write_bytes(b"edited\n")
    assert bench._measured_traffic("region_melded_traffic.json") is None


def test_traffic_missing_record_or_source_is_none(tmp_path, monkeypatch):
    srcs = _fake_root(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.remove(tmp_path / srcs[0])
    assert bench._measured_traffic("region_melded_traffic.json") is None
    shutil.rmtree(tmp_path / "profiles")
    assert bench._measured_traffic("region_melded_traffic.json") is None


def test_committed_record_names_existing_sources():
    with open(os.path.join(ROOT, "profiles", "region_melded_traffic.json")) as f:
        rec = json.load(f)
    assert rec["kernel"] == "region_melded_kernel"
    assert all(os.path.exists(os.path.join(ROOT, s)) for s in rec["sources"])
    assert rec["traffic_bytes"] > 0 and rec["fetch_factor"] > 0 and rec["write_factor"] > 0


def test_sort_roofline_takes_the_kernel_with_the_largest_total():
    import numpy as np
    plan = {"log_tile": 13,
            "passes": [{"kind": "local", "steps": 91}, {"kind": "regs", "steps": 1},
                       {"kind": "merge", "steps": 13}, {"kind": "regs", "steps": 2},
                       {"kind": "merge", "steps": 13}]}
    n = 1 << 20
    launches = [[1.0, 0.2, 0.5, 0.2, 0.5], [1.2, 0.2, 0.7, 0.2, 0.7]]
    roof, per = bench._sort_roofline(np, plan, launches, n)
    assert per["merge"]["launches_per_sort"] == 2
    assert abs(per["merge"]["avg_launch_us"] - 600.0) < 1e-6
    assert abs(per["merge"]["ms_per_sort"] - 1.2) < 1e-9
    assert roof["kind"] == "merge"  # 1.2 ms per sort against 1.1 (local) and 0.2 (each regs)
    assert roof["kernel"].startswith("bitonic_pass_regs_kernel<true, 13, 13, 13>")
    assert roof["launches_per_sort"] == 2
    assert abs(roof["achieved"] - 16 * n / 600e-6 / 1e9) < 0.1
    assert abs(roof["frac"] - roof["achieved"] / bench.HBM_PEAK_GBS) < 1e-4


def test_sort_roofline_counts_each_streaming_pass_kernel_apart():
    import numpy as np
    # the register passes together outweigh the merge tail, but each step count
    # is a kernel of its own; the merge tail is the largest single kernel
    plan = {"log_tile": 13,
            "passes": [{"kind": "regs", "steps": 1}, {"kind": "merge", "steps": 13},
                       {"kind": "regs", "steps": 2}, {"kind": "merge", "steps": 13},
                       {"kind": "regs", "steps": 3}]}
    launches = [[0.5, 0.6, 0.5, 0.6, 0.5]]
    roof, per = bench._sort_roofline(np, plan, launches, 1 << 20)
    assert per["regs"]["ms_per_sort"] > per["merge"]["ms_per_sort"]
    assert roof["kind"] == "merge"


def test_cpu_info_reports_model_and_counts():
    info = bench._cpu_info()
    assert info["host_logical_cpus"] >= 1 and info["affinity_cpus"] >= 1
    assert 1 <= bench._oracle_threads() <= 16


def test_pairs_check_accepts_the_sorted_order_with_high_keys():
    # keys on both sides of 2^31: the composite must order them as unsigned
    import pytest
    torch = pytest.importorskip("torch")
    kin = torch.tensor([0xFFFFFFF0, 5, 0x80000000, 5, 0x7FFFFFFF, 0xFFFFFFF0],
                       dtype=torch.int64).to(torch.int32)
    order = sorted(range(6), key=lambda i: ((int(kin[i]) & 0xFFFFFFFF), i))
    p = torch.tensor(order, dtype=torch.int32)
    k = kin[p.long()]
    bench._check_pairs_sorted(torch, kin, k, p)  # passes
    bad = p.clone()
    bad[[0, 5]] = bad[[5, 0]]
    with pytest.raises(SystemExit):
        bench._check_pairs_sorted(torch, kin, kin[bad.long()], bad)
    # equal keys out of payload order
    swapped = p.clone()
    i, j = [n for n in range(6) if int(k[n]) == 5]
    swapped[[i, j]] = swapped[[j, i]]
    with pytest.raises(SystemExit):
        bench._check_pairs_sorted(torch, kin, kin[swapped.long()], swapped)
