"""Full-size benchmark workloads on the GPU against the oracle.

The oracle's results for these graphs are stored in golden/workloads.json by
golden/make_golden.py (which calls only the oracle): totals, |W|, and SHA-256
digests of the full per-vertex and per-edge int64 arrays.  The GPU outputs are
hashed the same way, so every element is compared.  A few vertices and edges
are also recomputed live by the oracle one at a time (Eq. 1 and Eq. 8).  On
the 200M-edge graph the sort-based count (both wedge directions) is checked
against the stored total and |W| as well.
"""
import hashlib
import json
import os

import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
from gpu_util import to_dev

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "workloads.json")


def golden(name):
    if not os.path.exists(GOLDEN):
        pytest.skip("no stored oracle results")
    with open(GOLDEN) as f:
        d = json.load(f)
    if name not in d:
        pytest.skip(f"no stored oracle results for {name}")
    return d[name]


def digest(t: torch.Tensor) -> str:
    return hashlib.sha256(t.cpu().numpy().astype("<i8").tobytes()).hexdigest()


def run_workload(gpu_lib, name, per_vertex=True, per_edge=True, live_samples=8, sorted_count=False, tuning=None):
    rec = golden(name)
    g = gg.workload(name)
    print(f"{name}: generated m={g.m} tuning={tuning}", flush=True)
    assert g.sha256() == rec["edges_sha256"], "generator output changed"
    with gpu_lib.Graph(to_dev(g), g.n_upper, g.n_lower) as h:
        if tuning:
            h.set_tuning(**tuning)
        tot, wed = h.count_total()
        print(f"{name}: total={tot} wedges={wed}", flush=True)
        assert tot == rec["total"]
        assert wed == rec["vp_wedges"]
        if sorted_count:
            # Algorithm 6's pair sort over the wedges of Algorithm 2 and of
            # Algorithm 3: same total, |W| pairs in both (Lemma 3), in many
            # memory-bounded chunks
            for d in (0, 1):
                st, pairs, chunks = h.count_total_sorted(direction=d)
                print(f"{name}: sorted direction {d}: total={st} pairs={pairs} chunks={chunks}", flush=True)
                assert st == rec["total"] and pairs == rec["vp_wedges"] and chunks > 2
        if per_vertex:
            up, lo = h.count_per_vertex()
            torch.cuda.synchronize()
            for k, v in rec["sample_upper"].items():
                assert int(up[int(k)]) == v, ("upper", k)
            for k, v in rec["sample_lower"].items():
                assert int(lo[int(k)]) == v, ("lower", k)
            assert digest(up) == rec["vertex_upper_sha256"]
            assert digest(lo) == rec["vertex_lower_sha256"]
            assert int(up.sum()) == int(lo.sum()) == 2 * tot
        if per_edge:
            be = h.count_per_edge()
            torch.cuda.synchronize()
            for k, v in rec["sample_edges"].items():
                assert int(be[int(k)]) == v, ("edge", k)
            assert digest(be) == rec["edge_sha256"]
            assert int(be.sum()) == 4 * tot
        if live_samples and (per_vertex or per_edge):
            rng = np.random.default_rng(99)
            with oracle.Single(g) as s:
                for i in rng.choice(g.m, live_samples, replace=False):
                    u, v = (int(x) for x in g.edges[i])
                    if per_edge:
                        assert int(be[int(i)]) == s.edge(u, v)
                    if per_vertex:
                        assert int(up[u]) == s.vertex(0, u)
                        assert int(lo[v]) == s.vertex(1, v)


def test_uniform_2k_3k_20k(gpu_lib):
    run_workload(gpu_lib, "uniform-2k-3k-20k")


def test_chunglu_1m_500k_20m(gpu_lib):
    run_workload(gpu_lib, "chunglu-1m-500k-20m")


def test_chunglu_16m_4m_200m_planted(gpu_lib):
    run_workload(gpu_lib, "chunglu-16m-4m-200m-planted", live_samples=4, sorted_count=True)


def test_chunglu_1m_500k_20m_vpp(gpu_lib):
    """Algorithm 3's wedges on the 20M-edge graph: every output identical."""
    run_workload(gpu_lib, "chunglu-1m-500k-20m", live_samples=4, tuning={"vpp": 3})


def test_chunglu_16m_4m_200m_planted_vpp(gpu_lib):
    run_workload(gpu_lib, "chunglu-16m-4m-200m-planted", per_vertex=False, live_samples=4, tuning={"vpp": 3})


def test_chunglu_1m_500k_20m_band(gpu_lib):
    """Top bands of 65,536 ranks on the 20M-edge graph: every output identical."""
    run_workload(gpu_lib, "chunglu-1m-500k-20m", live_samples=4, tuning={"top_band": 65536})


def test_chunglu_16m_4m_200m_planted_band(gpu_lib):
    run_workload(gpu_lib, "chunglu-16m-4m-200m-planted", per_vertex=False, live_samples=4,
                 tuning={"top_band": 65536})
