"""Host-side Python logic that needs no GPU: the serving loop's arrival
process and the benchmark's roofline bookkeeping (the traffic figure is
reported only while the profiled kernel sources are unchanged and, for the
plain scatter, the live run bins rounds from the threshold the counters were
taken at)."""
import json
import os
import shutil

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_poisson_arrivals():
    from paper_1604_07515_amd import serve
    rng = np.random.default_rng(3)
    arr = serve.poisson_arrivals(20000, 500.0, rng)
    assert np.all(np.diff(arr) >= 0) and arr[0] > 0
    gaps = np.diff(np.concatenate(([0.0], arr)))
    assert abs(gaps.mean() - 1 / 500.0) < 0.05 / 500.0       # exponential mean 1/qps
    assert abs(gaps.std() - 1 / 500.0) < 0.05 / 500.0        # and std 1/qps
    assert np.all(serve.poisson_arrivals(5, 0.0, rng) == 0)  # closed loop: all at once


def test_roofline_bytes_model():
    import bench
    tm = {"scatter": {"launches": 4, "ms": 2.0, "units": 1_000_000, "entries": 10_000}}
    r = bench.roofline(tm, "no-such-kernel")
    by = 20 * 1_000_000 + 24 * 10_000
    assert abs(r["achieved"] - by / 2e-3 / 1e9) < 1e-9
    assert abs(r["frac"] - r["achieved"] / 8000.0) < 1e-12
    assert r["traffic"] is None and r["avg_launch_us"] == 500.0
    assert r["algorithmic_bytes_per_launch"] == by / 4


def test_traffic_requires_unchanged_sources(tmp_path, monkeypatch):
    import bench
    prof = os.path.join(ROOT, "profiles", "scatter_hbm_traffic_rmat22.md")
    block = open(prof).read().split("```json", 1)[1].split("```", 1)[0]
    rec = json.loads(block)
    key = next(iter(rec))
    # a copy of the tree's sources: the recorded hash matches only the
    # unmodified files, and a one-byte change voids the traffic figure
    fake = tmp_path / "repo"
    for src in rec[key]["sources"]:
        dst = fake / src
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copy(os.path.join(ROOT, src), dst)
    (fake / "profiles").mkdir()
    shutil.copy(prof, fake / "profiles" / os.path.basename(prof))
    monkeypatch.setattr(bench, "ROOT", str(fake))
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(fake / "profiles" / os.path.basename(prof)))
    emin = rec[key].get("plain_bin_min_edges")
    live = bench.measured_traffic(key, emin)
    current = bench.hashlib.sha256()
    for src in rec[key]["sources"]:
        current.update(open(os.path.join(ROOT, src), "rb").read())
    if current.hexdigest()[:16] == rec[key]["source_sha256_16"]:
        assert live is not None and live["traffic_bytes_per_launch"] > 0
    else:
        assert live is None  # the sources changed since the counters were taken
    if emin is not None:
        # counters taken at one binning threshold say nothing of another
        assert bench.measured_traffic(key, -1 if emin > 0 else 524288) is None
    victim = fake / rec[key]["sources"][0]
    victim.write_bytes(victim.read_bytes() + b"\n")
    assert bench.measured_traffic(key) is None
    assert bench.measured_traffic("no-such-kernel") is None
