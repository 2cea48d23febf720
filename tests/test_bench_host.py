"""Host-side logic of bench.py (no GPU): the single-GPU guard and the
counter-traffic bookkeeping that reports `traffic` only for the kernel
source the counters were taken on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]


def test_traffic_follows_the_kernel_source(monkeypatch):
    import hashlib

    import bench
    t = dict(bench.KERNEL_TRAFFIC["cocg_fused"])
    with open(os.path.join(ROOT, t["src"]), "rb") as f:
        current = hashlib.sha256(f.read()).hexdigest()[:16]
    # pin the entry to the source as it stands, so the arithmetic is checked
    # whether or not the counters are current
    monkeypatch.setitem(bench.KERNEL_TRAFFIC, "cocg_fused", dict(t, sha256_16=current))
    expect = 1024 * (bench.FETCH_SCALE * t["fetch_kib"] + bench.WRITE_SCALE * t["write_kib"])
    assert bench.measured_traffic("cocg_fused") == int(expect)
    # scaled by the algorithmic bytes of this run over those of the counter run
    half = 0.5 * t["alg_bytes_per_launch"]
    assert bench.measured_traffic("cocg_fused", half) == pytest.approx(0.5 * expect, rel=1e-9)
    # a changed source (another hash) reports no traffic
    monkeypatch.setitem(bench.KERNEL_TRAFFIC, "cocg_fused", dict(t, sha256_16="0" * 16))
    assert bench.measured_traffic("cocg_fused") is None
    assert bench.measured_traffic("no_such_kernel") is None


def test_every_traffic_entry_names_an_existing_source():
    import bench
    for name, t in bench.KERNEL_TRAFFIC.items():
        assert os.path.exists(os.path.join(ROOT, t["src"])), name
        assert t["fetch_kib"] > 0 and t["write_kib"] > 0 and t["alg_bytes_per_launch"] > 0
