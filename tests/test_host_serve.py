"""Host logic of the served form (no GPU needed): device-footprint
accounting used by admission, result digests and latency statistics."""
import hashlib
import os

import numpy as np
import pytest
import torch

from paper_1812_00283_amd import bfc, build, serve


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(bfc.LIB_PATH):
        build.build()
    return bfc.load(torch_memory=False)


def test_output_bytes_per_request_kind():
    assert serve.out_bytes(100, 7, 9, "total") == 0
    assert serve.out_bytes(100, 7, 9, "vertex") == 8 * 16
    assert serve.out_bytes(100, 7, 9, "edge") == 8 * 100


def test_job_bytes_cover_graph_upload_and_outputs(lib):
    for m, nu, nl in [(0, 0, 0), (10, 3, 4), (5_000_000, 1_000_000, 300_000)]:
        est = bfc.estimate_device_bytes(m, nu, nl)
        assert est > 0
        for kind in ("total", "vertex", "edge"):
            assert serve.job_bytes(m, nu, nl, kind) == est + 8 * m + serve.out_bytes(m, nu, nl, kind)
    # larger graphs never need less
    a = bfc.estimate_device_bytes(1_000_000, 1000, 1000)
    b = bfc.estimate_device_bytes(2_000_000, 1000, 1000)
    c = bfc.estimate_device_bytes(2_000_000, 2000, 1000)
    assert a < b < c


def test_digest_is_sha256_of_little_endian_int64_and_the_sum():
    a = torch.tensor([1, -2, 3], dtype=torch.int64)
    b = torch.tensor([7], dtype=torch.int32)
    h, s = serve.digest(a, b)
    ref = hashlib.sha256(np.array([1, -2, 3], "<i8").tobytes() + np.array([7], "<i8").tobytes()).hexdigest()
    assert h == ref and s == 9


def test_latency_stats():
    jobs = []
    for i in range(100):
        j = serve.Job(index=i, kind="total", key=i, edges=np.zeros((1, 2), np.int32), n_upper=1, n_lower=1)
        j.arrival, j.done = 10.0, 10.0 + (i + 1) / 1000.0  # 1..100 ms
        jobs.append(j)
    st = serve.latency_stats(jobs)
    assert st["max_ms"] == pytest.approx(100.0)
    assert st["mean_ms"] == pytest.approx(50.5)
    assert st["p50_ms"] == pytest.approx(50.5)
    assert 99.0 <= st["p99_ms"] <= 100.0
