"""Host logic of bench.py that needs no GPU: the single-GPU guard and the
gate that reports HBM traffic only from counters taken on the current
source."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)


def test_traffic_gate_follows_the_source(tmp_path, monkeypatch):
    src = tmp_path / "kernel.hip"
    src.write_text("__global__ void k() {}\n")
    summary = tmp_path / "k_pmc.txt"
    summary.write_text("# counters\nsource_sha1 = %s\nhbm_bytes_per_unit = 1.5e+08\n" % bench.src_sha1([str(src)]))
    monkeypatch.setitem(bench.PMC, "k_test", (str(summary), [str(src)]))
    assert bench.read_traffic("k_test") == 1.5e8
    src.write_text("__global__ void k() { /* changed */ }\n")
    assert bench.read_traffic("k_test") is None
    monkeypatch.setitem(bench.PMC, "k_test", (str(tmp_path / "missing.txt"), [str(src)]))
    assert bench.read_traffic("k_test") is None


def test_committed_summaries_name_existing_sources():
    for kernel, (path, srcs) in bench.PMC.items():
        assert os.path.exists(path), kernel
        assert all(os.path.exists(s) for s in srcs), kernel
