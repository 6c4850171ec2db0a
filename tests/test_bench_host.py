"""Host-side logic of the benchmark (CPU tier): the one-GPU guard and the
summaries it builds from rocprofv3 databases (synthetic databases here)."""
import json
import os
import sqlite3
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _trace_db(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    con = sqlite3.connect(path)
    con.execute("create table kernels (name text, duration integer)")
    con.executemany("insert into kernels values (?, ?)", rows)
    con.commit()
    con.close()


def test_trace_summary_table(tmp_path, capsys):
    # durations in ns, as rocprofv3 stores them
    _trace_db(str(tmp_path / "host" / "rc_results.db"),
              [("row_kernel", 18000), ("row_kernel", 20000), ("copy", 10000)])
    bench.trace_summary(str(tmp_path))
    out = capsys.readouterr().out.splitlines()
    assert out[2] == "| `row_kernel` | 2 | 19.00 | 18.00 | 20.00 | 79.2% |"
    assert out[3] == "| `copy` | 1 | 10.00 | 10.00 | 10.00 | 20.8% |"


def test_trace_summary_needs_one_database(tmp_path):
    with pytest.raises(SystemExit):
        bench.trace_summary(str(tmp_path))


def _pmc_db(path, kern_kib, copy_kib):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (kernel_name text, value real)")
    con.executemany("insert into counters_collection values (?, ?)",
                    [("void bfp::row_kernel<bfp::ModeFP16, 12, 2, 0, false, true>(bfp::RowArgs)", v)
                     for v in kern_kib] +
                    [("void bfp::copy_kernel(uint4 const*, uint4*, long long)", copy_kib)])
    con.commit()
    con.close()


def test_traffic_summary_scales_each_counter_by_the_copy(tmp_path, monkeypatch, capsys):
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    _pmc_db(str(tmp_path / "f" / "x" / "pmc_results.db"), [16000.0, 16400.0], 16384.0)
    _pmc_db(str(tmp_path / "w" / "x" / "pmc_results.db"), [32768.0], 32768.0)
    bench.traffic_summary([("fp16", str(tmp_path / "f"), str(tmp_path / "w"))])
    rec = json.loads(out.read_text())
    m = rec["modes"]["fp16"]
    # fetch: 16200 KiB x (32768 / 16384); write: 32768 KiB x 1
    assert m["traffic_bytes"] == (16200 * 2 + 32768) * 1024
    assert m["fetch_factor"] == 2.0 and m["write_factor"] == 1.0
    assert rec["kernel_source_sha256"] == bench.kernel_source_sha256()
    assert "(0.994 x algorithmic 67108864 B)" in capsys.readouterr().out


def test_measured_traffic_only_for_the_sources_it_was_taken_on(tmp_path, monkeypatch):
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    rec = {"kernel_sources": bench.KERNEL_SOURCES, "kernel_source_sha256": bench.kernel_source_sha256(),
           "modes": {"fp16": {"traffic_bytes": 123}}}
    out.write_text(json.dumps(rec))
    assert bench.measured_traffic("fp16") == 123
    assert bench.measured_traffic("fp32") is None
    rec["kernel_source_sha256"] = "0" * 64
    out.write_text(json.dumps(rec))
    assert bench.measured_traffic("fp16") is None
