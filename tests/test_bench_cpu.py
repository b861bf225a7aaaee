"""Host-side pieces of bench.py (no GPU): the one-GPU guard, the byte
accounting, the rule that the profiled HBM traffic is reported only for the
kernel source it was measured on, and the CPU oracle baseline on a small
sample."""
import hashlib
import os
import subprocess
import sys

import pytest

import bench
from paper_1506_07207_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_algorithmic_bytes_per_tracer_and_cell():
    # read and write of the 8-byte position word and the 8-byte velocity
    assert bench.BYTES_PER_TRACER == 2 * (8 + 8)
    # E read, P and D read and cleared, E written: 4 x 8 bytes per cell
    assert bench.BYTES_PER_CELL == 4 * 8
    # a deposit alone reads the position word once
    assert bench.DEPOSIT_BYTES_PER_TRACER == 8


def _traffic_file(tmp_path, digest, value):
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "k_tracers_fp64_mixed4096_traffic.md").write_text(
        "# summary\n\n    kernel_source_sha256_16=%s\n    traffic_bytes_per_launch=%d\n" % (digest, value))
    src = tmp_path / "paper_1506_07207_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "sic_kernels.hip").write_text("// kernel source\n")
    return hashlib.sha256(b"// kernel source\n").hexdigest()[:16]


def test_traffic_reported_only_for_the_profiled_source_and_shape(tmp_path, monkeypatch):
    digest = _traffic_file(tmp_path, "0" * 16, 0)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    shape = {"tile_chunks": 256, "block_threads": 512, "grid_blocks": 131072}
    assert bench.profiled_traffic("fp64", 4096, shape) is None  # stale: another source was profiled
    (tmp_path / "profiles" / "k_tracers_fp64_mixed4096_traffic.md").write_text(
        "    kernel_source_sha256_16=%s\n    launch_shape=256,512,131072\n"
        "    traffic_bytes_per_launch=123456789\n" % digest)
    assert bench.profiled_traffic("fp64", 4096, shape) == 123456789.0
    # only for the workload, precision and launch shape that were profiled
    assert bench.profiled_traffic("split_u32", 4096, shape) is None
    assert bench.profiled_traffic("fp64", 512, shape) is None
    assert bench.profiled_traffic("fp64", 4096, dict(shape, tile_chunks=128)) is None


def test_committed_traffic_summary_is_machine_readable():
    path = os.path.join(ROOT, "profiles", "k_tracers_fp64_mixed4096_traffic.md")
    kv = dict(line.strip().split("=", 1) for line in open(path) if "=" in line and " " not in line.strip())
    assert len(kv["kernel_source_sha256_16"]) == 16
    assert len(kv["launch_shape"].split(",")) == 3
    assert float(kv["traffic_bytes_per_launch"]) > 0


def test_host_cores_follows_the_thread_share(monkeypatch):
    monkeypatch.setenv("OMP_NUM_THREADS", "3")
    assert 1 <= bench.host_cores() <= 3
    monkeypatch.setenv("OMP_NUM_THREADS", "")
    assert bench.host_cores() >= 1


@pytest.mark.timeout(300)
def test_cpu_baseline_runs_the_oracle_on_worker_processes():
    specs = I.batch_mix(6)
    rate, n_inst, secs = bench.cpu_baseline(specs, 0.5, 2)
    assert n_inst >= 2  # every worker times at least one whole instance
    assert rate > 0 and secs > 0
