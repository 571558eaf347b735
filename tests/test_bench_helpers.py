"""CPU tests of the benchmark's bookkeeping: the HBM-traffic figure is taken
from a committed counter summary only while the kernel sources it names hash
to the stored value and the launch is the one it was taken on; the traffic
fields are a rate in GB/s, GB per launch and a ratio; the host description
has the fields the CPU baseline reports."""
import hashlib
import json
import os

import pytest

import bench


def _fake_counters(root, src_text, pivots=10):
    os.makedirs(os.path.join(root, "profiles"))
    os.makedirs(os.path.join(root, "src"))
    with open(os.path.join(root, "src", "k.hip"), "w") as f:
        f.write(src_text)
    h = hashlib.sha256(src_text.encode()).hexdigest()
    d = {"kernel_sources": ["src/k.hip"], "kernel_source_sha256": h, "pivots": pivots,
         "fetch_size_kib": 100.0, "fetch_scale": 2.0, "write_size_kib": 300.0, "write_scale": 1.0}
    with open(os.path.join(root, "profiles", "k_counters.json"), "w") as f:
        json.dump(d, f)


def test_counter_traffic_is_gated_by_the_source_hash(tmp_path, monkeypatch):
    root = str(tmp_path)
    _fake_counters(root, "kernel v1")
    monkeypatch.setattr(bench, "ROOT", root)
    # (100 * 2 + 300 * 1) KiB
    assert bench.counter_traffic("k", 10) == pytest.approx(500.0 * 1024)
    assert bench.counter_traffic("k", 11) is None          # another launch
    assert bench.counter_traffic("missing", 10) is None    # no summary
    with open(os.path.join(root, "src", "k.hip"), "w") as f:
        f.write("kernel v2")                               # sources changed since
    assert bench.counter_traffic("k", 10) is None


def test_traffic_fields():
    none = bench.traffic_fields(None, 10.0, 1e9)
    assert none == {"traffic": None, "traffic_GB_per_launch": None, "traffic_over_algorithmic": None}
    f = bench.traffic_fields(2e9, 500.0, 1e9)   # 2 GB in 0.5 s, algorithmic 1 GB
    assert f["traffic"] == pytest.approx(4.0)
    assert f["traffic_GB_per_launch"] == pytest.approx(2.0)
    assert f["traffic_over_algorithmic"] == pytest.approx(2.0)


def test_host_description():
    h = bench.host_cpu()
    assert set(h) == {"model", "sockets", "physical_cores", "logical_cpus_allowed"}
    assert h["sockets"] >= 1 and h["physical_cores"] >= 1 and h["logical_cpus_allowed"] >= 1


def test_batched_cpu_baseline_solves_every_lp():
    from paper_1804_04737_amd import lpgen
    lps = lpgen.batch_lps(12, 8, 40, 3)
    r = bench.batch_cpu_baseline(lps, 4)
    assert r["statuses_optimal"] == 12 and r["threads"] == 4 and r["LPs_per_s"] > 0
