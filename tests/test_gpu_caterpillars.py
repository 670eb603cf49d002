"""Caterpillars (three-paths) and the bipartite clustering coefficient of
Section 1 from the HIP library against the oracle: exact int64 counts on
small graphs, batches (the sum over their graphs) and the benchmark
workloads (counts stored by golden/make_caterpillars.py, which calls only the
oracle); the coefficient 4 B_G / C_G is compared bit for bit, both sides
dividing the same integers in double precision.
"""
import json
import os

import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
from gpu_util import to_dev

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "caterpillars.json")


def small_graphs():
    yield gg.complete_bipartite(7, 9)
    yield gg.even_cycle(6)
    yield gg.random_forest(3, 400, 300)
    for i in range(8):
        yield gg.random_small(500 + i, 3 + 5 * i, 4 + 3 * i, 0.3)
    yield gg.chung_lu(41, 3000, 2000, 25000, 2.1, 2.1, 800.0)
    yield gg.Graph(np.zeros((0, 2), np.int32), 3, 2)


def test_small_graphs_match_oracle(gpu_lib):
    for g in small_graphs():
        with gpu_lib.Graph(to_dev(g), g.n_upper, g.n_lower) as h:
            assert h.caterpillars() == oracle.caterpillars(g), g.name
            assert h.clustering_coefficient() == oracle.clustering_coefficient(g), g.name


def test_batch_is_the_sum_over_its_graphs(gpu_lib):
    graphs = [gg.random_small(900 + i, 6 + i, 5 + 2 * i, 0.35) for i in range(12)]
    graphs.append(gg.complete_bipartite(5, 8))
    b = gg.concat(graphs)
    with gpu_lib.build_batch(torch.from_numpy(b.edges).cuda(), b.offsets, b.n_upper, b.n_lower) as h:
        assert h.caterpillars() == sum(oracle.caterpillars(g) for g in graphs)


@pytest.mark.parametrize("name", ["uniform-2k-3k-20k", "chunglu-1m-500k-20m", "chunglu-16m-4m-200m-planted"])
def test_workloads_match_stored_oracle_counts(gpu_lib, name):
    with open(GOLDEN) as f:
        rec = json.load(f)[name]
    g = gg.workload(name)
    assert g.sha256() == rec["edges_sha256"], "generator output changed"
    print(f"{name}: generated m={g.m}", flush=True)
    with gpu_lib.Graph(to_dev(g), g.n_upper, g.n_lower) as h:
        assert h.caterpillars() == rec["caterpillars"]
        if g.m <= 20_000_000:
            tot, _ = h.count_total()
            assert h.clustering_coefficient() == 4.0 * tot / rec["caterpillars"]
