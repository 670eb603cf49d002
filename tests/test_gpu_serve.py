"""Served form: results in the continuous-batching mix equal results alone.

A seeded arrival trace (the served workload's generator, with smaller graphs
so the oracle can check every request) is served twice: by the batched,
caching, multi-stream server under a tight HBM budget, and one request at a
time by the plain server.  Every request's output must be identical in both,
every output must equal the oracle's (totals by value, per-vertex and
per-edge arrays by the digest of the whole array), and admitted work must
never exceed the budget.
"""
import hashlib

import numpy as np
import pytest

import graphgen as gg
import oracle
from paper_1812_00283_amd import serve

pytestmark = pytest.mark.gpu


def oracle_result(g, kind):
    """The oracle's answer in the server's result form: the total, or
    (sha256 of the int64 little-endian arrays, their sum)."""
    if kind == "total":
        return oracle.total(g)
    arrays = oracle.vertex_counts(g) if kind == "vertex" else (oracle.edge_counts(g),)
    h = hashlib.sha256()
    s = 0
    for a in arrays:
        x = np.ascontiguousarray(a, dtype="<i8")
        h.update(x.tobytes())
        s += int(x.sum())
    return h.hexdigest(), s


def make_jobs(reqs, graphs):
    return [serve.Job(r.index, r.kind, r.follow_up_of if r.follow_up_of >= 0 else r.index,
                      graphs[r.follow_up_of if r.follow_up_of >= 0 else r.index].edges,
                      r.graph.n_upper, r.graph.n_lower) for r in reqs]


def test_mix_equals_alone_and_oracle(gpu_lib):
    reqs = gg.serve_schedule(rate=200.0, duration_s=0.6, m_lo=2_000, m_hi=300_000)
    roots = {r.index: r.graph for r in reqs if r.follow_up_of < 0}
    built = dict(zip(roots, gg.spec_graphs(list(roots.values()))))
    arrivals = [r.arrival_s for r in reqs]
    print(f"{len(reqs)} requests, {len(roots)} graphs", flush=True)

    mixed = make_jobs(reqs, built)
    budget = 3 * max(serve.job_bytes(g.m, g.n_upper, g.n_lower, "edge") for g in built.values())
    srv = serve.Server(budget, slots=4, batch_small_edges=50_000)
    serve.replay(mixed, arrivals, srv, time_scale=0.25)
    assert srv.peak <= budget
    alone = make_jobs(reqs, built)
    serve.replay(alone, arrivals, serve.Server(1 << 40, plain=True), time_scale=0.0)
    assert any(j.batched for j in mixed) and any(j.cache_hit for j in mixed)
    for a, b in zip(mixed, alone):
        assert a.result == b.result, (a.index, a.kind)
    kinds = set()
    for jb in mixed:
        assert jb.result == oracle_result(built[jb.key], jb.kind), (jb.index, jb.kind)
        kinds.add(jb.kind)
    assert kinds == {"total", "vertex", "edge"}
