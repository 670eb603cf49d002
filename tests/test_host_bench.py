"""Host logic of the benchmark and the build bookkeeping (no GPU needed):
the heavy kernel's algorithmic bytes, when the stored traffic counters
apply, the source digests that detect stale builds and stale counters, and
the single-GPU refusal."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

import bench  # noqa: E402
from paper_1812_00283_amd import bfc, build  # noqa: E402


def test_heavy_kernel_bytes_per_unit():
    # 4 bytes per wedge, 16 per middle arc, 8 per start
    assert bench.heavy_kernel_bytes({"wedges_heavy": 1, "middles_heavy": 0, "starts_heavy": 0}) == 4
    assert bench.heavy_kernel_bytes({"wedges_heavy": 0, "middles_heavy": 1, "starts_heavy": 0}) == 16
    assert bench.heavy_kernel_bytes({"wedges_heavy": 0, "middles_heavy": 0, "starts_heavy": 1}) == 8
    assert bench.heavy_kernel_bytes({"wedges_heavy": 10, "middles_heavy": 3, "starts_heavy": 2}) == 40 + 48 + 16


def test_stored_traffic_applies_only_to_its_sources_workload_and_defaults(monkeypatch):
    t = bench.HEAVY_TRAFFIC
    w = bench.DEFAULT_WORKLOAD
    monkeypatch.setattr(bench, "sources_sha256", lambda: t["sources_sha256"])
    rec = t["workloads"][w]
    expect = rec["read_requests"] * t["bytes_per_read_request"] + 1024.0 * rec["write_kib"] * t["write_factor"]
    assert bench.heavy_traffic(w, tuned=False) == pytest.approx(expect)
    assert bench.heavy_traffic(w, tuned=True) is None
    assert bench.heavy_traffic("no-such-workload", tuned=False) is None
    monkeypatch.setattr(bench, "sources_sha256", lambda: "0" * 64)
    assert bench.heavy_traffic(w, tuned=False) is None


def test_heavy_sources_digest_follows_the_kernel_files(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_1812_00283_amd" / "csrc"
    csrc.mkdir(parents=True)
    for n in bench.HEAVY_SOURCES:
        shutil.copy(os.path.join(ROOT, "paper_1812_00283_amd", "csrc", n), csrc / n)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    d0 = bench.sources_sha256()
    with open(csrc / "count.hip", "a") as f:
        f.write("\n// changed\n")
    assert bench.sources_sha256() != d0


def test_library_digest_detects_a_stale_build(tmp_path, monkeypatch):
    lib = tmp_path / "libbfc.so"
    lib.write_bytes(b"")
    monkeypatch.setattr(bfc, "LIB_PATH", str(lib))
    assert not bfc.library_matches_sources()  # no digest recorded
    (tmp_path / "libbfc.so.sources").write_text(build.sources_digest() + "\n")
    assert bfc.library_matches_sources()
    (tmp_path / "libbfc.so.sources").write_text("0" * 64 + "\n")
    assert not bfc.library_matches_sources()


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
