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


def test_trace_summary_tail_keeps_the_last_library_dispatches(tmp_path, capsys):
    # the timed region: the last K dispatches of the library's kernels
    # (demangled bfp:: names and mangled _ZN3bfp ones), runtime copies left out
    path = str(tmp_path / "host" / "t_results.db")
    os.makedirs(os.path.dirname(path))
    con = sqlite3.connect(path)
    con.execute("create table kernels (name text, start integer, duration integer)")
    con.executemany("insert into kernels values (?, ?, ?)", [
        ("void bfp::row_kernel<x>(bfp::RowArgs)", 1, 90000),       # autotuning, dropped
        ("__amd_rocclr_copyBuffer", 2, 5000),
        ("void bfp::row_kernel<x>(bfp::RowArgs)", 3, 30000),
        ("_ZN3bfp17phase_grad_kernelE", 4, 60000),
        ("__amd_rocclr_copyBuffer", 5, 7000),
        ("void bfp::row_kernel<x>(bfp::RowArgs)", 6, 32000)])
    con.commit()
    con.close()
    bench.trace_summary(str(tmp_path), tail=3)
    out = capsys.readouterr().out.splitlines()
    assert out[2] == "| `void bfp::row_kernel<x>(bfp::RowArgs)` | 2 | 31.00 | 30.00 | 32.00 | 50.8% |"
    assert out[3] == "| `_ZN3bfp17phase_grad_kernelE` | 1 | 60.00 | 60.00 | 60.00 | 49.2% |"
    assert len(out) == 4


def test_traffic_summary_uses_each_modes_bytes(tmp_path, monkeypatch, capsys):
    # FP32 storage: 128 MiB per launch, the calibration copy moves 64 MiB each way
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    _pmc_db(str(tmp_path / "f" / "x" / "pmc_results.db"), [32768.0], 32768.0)
    _pmc_db(str(tmp_path / "w" / "x" / "pmc_results.db"), [65536.0], 65536.0)
    bench.traffic_summary([("fp32", str(tmp_path / "f"), str(tmp_path / "w"))])
    m = json.loads(out.read_text())["modes"]["fp32"]
    assert m["algorithmic_bytes"] == 134217728
    assert m["fetch_factor"] == 2.0 and m["write_factor"] == 1.0
    assert m["traffic_bytes"] == 134217728
    assert "(1.000 x algorithmic 134217728 B)" in capsys.readouterr().out


def test_parse_tuning():
    assert bench.parse_tuning("1,8,1,0") == (1, 8, 1, 0)
    assert bench.parse_tuning("0,-1,2,1") == (0, -1, 2, 1)
    with pytest.raises(SystemExit):
        bench.parse_tuning("1,8,1")
