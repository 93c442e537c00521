"""bench.py checks that need no GPU: the one-GPU contract and the counter summary gate."""
from __future__ import annotations

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "single GPU" in r.stderr + r.stdout


def test_measured_traffic_requires_matching_sources(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    f = tmp_path / "traffic.txt"
    k = "k_mp_p2<double, 2048>"
    body = f"kernel = {k}\nphase = row\ntraffic_bytes_per_launch = 123\nalgorithmic_bytes_per_launch = 100\n"
    f.write_text(body + "source_sha256 = not-the-digest\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic("row", k, 100) is None                      # taken with other device sources
    f.write_text(body + f"source_sha256 = {bench.source_digest()}\n")
    assert bench.measured_traffic("row", k, 100) == 123.0
    assert bench.measured_traffic("col_fwd", k, 100) is None                  # another phase
    assert bench.measured_traffic("row", "k_mp_p2<double, 4096>", 100) is None  # plan ran another row length
    assert bench.measured_traffic("row", k, 200) is None                      # launch of other bytes (rank, chunks)
