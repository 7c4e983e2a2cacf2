"""Host-side checks of the benchmark's bookkeeping (no GPU): the algorithmic
bytes behind the roofline, the traffic records' source check, and the
one-GPU guard."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
from inputs import C2, C3  # noqa: E402


def test_algorithmic_bytes_per_launch():
    """Per particle: momentum reads cell, offsets, azimuth, p, w (32 B) and
    writes p (12 B); position reads the same 32 B and writes cell, offsets,
    azimuth (16 B).  Per cell (modes 0 and 1): 72 B and 48 B.  The field
    update moves 36 B per cell for mode 0 and 144 B more for mode 1; the
    envelope update 28 B."""
    n = 2048 * 256 * 16
    ab = bench.algorithmic_bytes(C2, n)
    assert ab["per_particle"] == {"k_momentum": 44, "k_position": 48, "k_field": 0, "k_envelope": 0}
    assert ab["per_cell"] == {"k_momentum": 72, "k_position": 48, "k_field": 180, "k_envelope": 28}
    assert ab["k_momentum"] == 44 * n + 72 * 2048 * 256 == 406_847_488
    assert ab["k_position"] == 48 * n + 48 * 2048 * 256 == 427_819_008
    assert ab["k_field"] == 180 * 2048 * 256
    m0 = bench.algorithmic_bytes(dict(C3, n_modes=1), 10)
    assert m0["per_cell"] == {"k_momentum": 24, "k_position": 24, "k_field": 36, "k_envelope": 28}


def test_traffic_records_follow_the_sources(tmp_path, monkeypatch):
    """A committed traffic record is reported only while the HIP sources hash
    to the digest recorded with the counters."""
    for wl in ("c2_lwfa_2048x256", "c3_bandwidth_4096x512"):
        for k in ("k_momentum", "k_position"):
            rec = json.load(open(os.path.join(ROOT, "profiles", f"traffic_{k}_{wl}.json")))
            assert rec["bytes_per_launch"] > 0 and rec["dispatches"] > 0
            if rec["source_sha256_16"] == bench.source_digest():
                assert bench.traffic_record(k, wl) == rec["bytes_per_launch"]
    monkeypatch.setattr(bench, "source_digest", lambda: "0" * 16)
    assert bench.traffic_record("k_momentum", "c2_lwfa_2048x256") is None
    assert bench.traffic_record("k_momentum", "no_such_workload") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout
