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


def _pmc_db(path, counter, rows):
    """A rocprofv3-style counter database: (kernel name, KiB) per dispatch, in order."""
    import sqlite3
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (dispatch_id integer, kernel_name text, counter_name text, "
                "value real)")
    con.executemany("insert into counters_collection values (?, ?, ?, ?)",
                    [(i, k, counter, v) for i, (k, v) in enumerate(rows)])
    con.commit()
    con.close()


def test_write_traffic_scales_by_the_copy_and_names_the_fixed_shapes(tmp_path, monkeypatch):
    import json
    import pytest
    sys.path.insert(0, ROOT)
    import bench
    copy_kib = bench.COPY_BYTES / 1024
    p2 = "void thx::k_mp_p2<double, 4096>(thx::cpx<double>*, int)"
    timed = [("void thx::k_trace_marker(int)", 0.0), (p2, 1000.0), ("void thx::k_unpack<double>(int)", 10.0),
             ("void thx::k_trace_marker(int)", 0.0)]
    # FETCH_SIZE reads half of the copy's bytes (factor 2), WRITE_SIZE all of them (factor 1)
    _pmc_db(tmp_path / "f.db", "FETCH_SIZE", [("__amd_rocclr_copyBuffer", copy_kib / 2)] + timed)
    _pmc_db(tmp_path / "w.db", "WRITE_SIZE", [("__amd_rocclr_copyBuffer", copy_kib)] + [(k, 3 * v) for k, v in timed])
    log = tmp_path / "run.log"
    log.write_text(json.dumps({"headline_only": True, "prec": "fp64", "log2n": 20, "autotuned": False,
                               "shapes": [4096, 2048], "fft_geometry": [4096, 256, 16],
                               "phase_bytes": {"row": 5 * 1024 * 1000, "col_fwd": 1, "col_inv": 1}}) + "\n")
    out = tmp_path / "traffic.txt"
    bench.write_traffic(str(tmp_path / "f.db"), str(tmp_path / "w.db"), str(log), str(out))
    kv = dict(line.split(" = ", 1) for line in out.read_text().splitlines() if " = " in line and line[0] != "#")
    assert kv["kernel"] == "k_mp_p2<double, 4096>" and kv["phase"] == "row"
    assert float(kv["fetch_factor"]) == 2.0 and float(kv["write_factor"]) == 1.0
    assert int(kv["traffic_bytes_per_launch"]) == (2 * 1000 + 3000) * 1024  # 2 x read + 1 x written KiB
    assert kv["source_sha256"] == bench.source_digest()
    text = out.read_text()
    assert "--shapes 4096 2048" in text and "--no-autotune" not in text
    assert "2048 workgroups per launch" in text
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    assert bench.measured_traffic("row", "k_mp_p2<double, 4096>", 5 * 1024 * 1000) == (2 * 1000 + 3000) * 1024
    # the two counter runs timed different kernels: refused
    _pmc_db(tmp_path / "w2.db", "WRITE_SIZE", [("__amd_rocclr_copyBuffer", copy_kib)] +
            [(k.replace("4096", "2048"), v) for k, v in timed])
    with pytest.raises(SystemExit):
        bench.write_traffic(str(tmp_path / "f.db"), str(tmp_path / "w2.db"), str(log), str(tmp_path / "t2.txt"))
