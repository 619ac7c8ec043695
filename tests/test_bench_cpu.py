"""Host-side logic of bench.py: byte accounting, the profiled-traffic lookup and
the single-GPU guard.  No GPU is used."""

import hashlib
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_sweep_bytes_match_the_workload_arithmetic():
    # 2048 x 2048, N = 20, float32, R_spec as an array: each complex half spectrum
    # is 2048 * 1025 * 8 bytes, each real field 2048 * 2048 * 4
    N, ny, nx, s = 20, 2048, 2048, 4
    half = 2048 * 1025 * 8
    field = 2048 * 2048 * 4
    rspec = 2048 * 1025 * 4
    b = bench.sweep_bytes(N, ny, nx, s, True)
    assert b["sweep1"] == 21 * field + 21 * half
    assert b["sweep2"] == 21 * half + rspec + 20 * half == 696_934_400
    assert b["sweep3"] == 20 * half + 20 * field
    assert b["path"] == 41 * field + rspec == 696_262_656
    # a scalar R adds no bytes
    b0 = bench.sweep_bytes(N, ny, nx, s, False)
    assert b["sweep2"] - b0["sweep2"] == rspec and b0["sweep1"] == b["sweep1"]


def _fake_profiles(tmp_path, records, sources_text):
    os.makedirs(tmp_path / "profiles")
    os.makedirs(tmp_path / "src")
    for name, text in sources_text.items():
        (tmp_path / "src" / name).write_text(text)
    with open(tmp_path / "profiles" / "kernels_traffic.json", "w") as f:
        json.dump({"kernels": records}, f)


def _hash(tmp_path, files):
    h = hashlib.sha256()
    for f in files:
        h.update((tmp_path / f).read_bytes())
    return h.hexdigest()[:16]


def test_profiled_traffic_takes_the_nearest_current_record(tmp_path, monkeypatch):
    _fake_profiles(tmp_path, [], {"a.hpp": "kernel a", "b.hpp": "kernel b"})
    good = _hash(tmp_path, ["src/a.hpp"])
    recs = [
        # same family, durations 100 us and 200 us, sources current
        {"name": "ns::k2_spectral<float, 128, 20, false>", "avg_ns": 100e3, "fetch_bytes": 1.0, "write_bytes": 2.0,
         "sources": ["src/a.hpp"], "sources_sha256_16": good},
        {"name": "ns::k2_spectral<float, 128, 20, true>", "avg_ns": 200e3, "fetch_bytes": 10.0, "write_bytes": 20.0,
         "sources": ["src/a.hpp"], "sources_sha256_16": good},
        # stale sources: never used
        {"name": "ns::k2_spectral<float, 64, 20, false>", "avg_ns": 190e3, "fetch_bytes": 7.0, "write_bytes": 7.0,
         "sources": ["src/b.hpp"], "sources_sha256_16": "0" * 16},
        # no counters: never used
        {"name": "ns::k1_forward<float, 2048, 16, 4, false>", "avg_ns": 150e3, "fetch_bytes": None,
         "write_bytes": 5.0, "sources": ["src/a.hpp"], "sources_sha256_16": good},
    ]
    with open(tmp_path / "profiles" / "kernels_traffic.json", "w") as f:
        json.dump({"kernels": recs}, f)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.profiled_traffic("k2_spectral", 0.105) == 3.0
    assert bench.profiled_traffic("k2_spectral", 0.195) == 30.0
    # beyond 25% of every current record's duration: no figure
    assert bench.profiled_traffic("k2_spectral", 0.300) is None
    # excluded substrings drop records however close their duration
    assert bench.profiled_traffic("k2_spectral", 0.195, exclude=("true>",)) is None
    assert bench.profiled_traffic("k2_spectral", 0.105, exclude=("true>",)) == 3.0


def test_profiled_traffic_family_with_bracket_skips_batched_kernels(tmp_path, monkeypatch):
    _fake_profiles(tmp_path, [], {"a.hpp": "kernel a"})
    good = _hash(tmp_path, ["src/a.hpp"])
    recs = [
        {"name": "ns::k2_spectral<float, 128, 20, 0>", "avg_ns": 245e3, "fetch_bytes": 300.0, "write_bytes": 400.0,
         "sources": ["src/a.hpp"], "sources_sha256_16": good},
        # a batched launch that happens to take about as long
        {"name": "ns::k2_spectral_batch<float, 128, 16>", "avg_ns": 244e3, "fetch_bytes": 100.0, "write_bytes": 100.0,
         "sources": ["src/a.hpp"], "sources_sha256_16": good},
    ]
    with open(tmp_path / "profiles" / "kernels_traffic.json", "w") as f:
        json.dump({"kernels": recs}, f)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.profiled_traffic("k2_spectral", 0.2437) == 200.0
    assert bench.profiled_traffic("k2_spectral<", 0.2437) == 700.0
    assert bench.profiled_traffic("k1_forward", 0.150) is None
    assert bench.profiled_traffic("k3_inverse", 0.150) is None


def test_profiled_traffic_drops_records_whose_sources_changed(tmp_path, monkeypatch):
    _fake_profiles(tmp_path, [], {"a.hpp": "kernel a"})
    rec = {"name": "ns::k3_inverse<float, 2048, 16, 4, false>", "avg_ns": 100e3, "fetch_bytes": 1.0,
           "write_bytes": 1.0, "sources": ["src/a.hpp"], "sources_sha256_16": _hash(tmp_path, ["src/a.hpp"])}
    with open(tmp_path / "profiles" / "kernels_traffic.json", "w") as f:
        json.dump({"kernels": [rec]}, f)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.profiled_traffic("k3_inverse", 0.1) == 2.0
    (tmp_path / "src" / "a.hpp").write_text("kernel a, edited")
    assert bench.profiled_traffic("k3_inverse", 0.1) is None


def test_more_than_one_gpu_is_refused_without_touching_a_device():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
