"""Host-side parts of bench.py: the algorithmic byte count behind the roofline,
the guard that uses committed traffic counters only for the kernel sources
they were taken from, and the refusal of more than one GPU."""
import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_algorithmic_bytes(bench):
    M, N = 1024, 524288
    # LayerNorm: x read and y written (4 B each), gamma and beta once, mean and rstd per row
    assert bench.algorithmic_bytes("layernorm_fwd", M, N) == 8 * M * N + 8 * N + 8 * M == 4299169792
    # RMSNorm: gamma once, rstd per row
    assert bench.algorithmic_bytes("rmsnorm_fwd", M, N) == 8 * M * N + 4 * N + 4 * M


def test_traffic_used_only_for_the_sources_it_was_taken_from(bench, tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2609_01864_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "a.hip").write_text("kernel one\n")
    build_py = tmp_path / "paper_2609_01864_amd" / "build.py"
    build_py.write_text("FLAGS = ['-O3']\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    key = "layernorm_fwd:N=524288:plan=2,16"
    assert bench.traffic_for(key) is None  # no profile
    (tmp_path / "profiles").mkdir()
    prof = tmp_path / "profiles" / "traffic.json"
    prof.write_text(json.dumps({"kernels": {key: {"bytes_per_launch": 123, "source_hash": bench.source_hash()}}}))
    assert bench.traffic_for(key) == 123
    assert bench.traffic_for("rmsnorm_fwd:N=8192:plan=1,1") is None  # no entry for that launch
    (csrc / "a.hip").write_text("kernel two\n")  # the kernel changed since the counters were taken
    assert bench.traffic_for(key) is None
    (csrc / "a.hip").write_text("kernel one\n")
    assert bench.traffic_for(key) == 123
    build_py.write_text("FLAGS = ['-O2']\n")  # so did its compiler flags
    assert bench.traffic_for(key) is None
    prof.write_text("{not json")
    assert bench.traffic_for(key) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
