"""Sort-based total count (Algorithm 6 with device memory for disk) from the
HIP library against the oracle (Lemma 1): exact int64 totals on small and
power-law graphs, with chunk limits that split the start ranges into many
chunks (down to one pair, so every start past the limit is a chunk of its
own), on a batch (the sum over its graphs) and on the benchmark workloads
against the oracle's stored totals.
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

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "workloads.json")


def sorted_total(bfc, g, max_pairs=0, with_max=False):
    with bfc.Graph(to_dev(g), g.n_upper, g.n_lower) as h:
        t, chunks = h.count_total_sorted(max_pairs)
        if with_max:
            return t, chunks, h.info()["wedges"], h.schedule_info()["max_start_wedges"]
        return t, chunks, h.info()["wedges"]


def test_small_graphs(gpu_lib):
    rng = np.random.default_rng(31)
    graphs = [gg.complete_bipartite(a, b) for a, b in [(1, 1), (2, 2), (3, 5), (17, 9), (64, 64), (300, 100)]]
    graphs += [gg.even_cycle(2), gg.even_cycle(9), gg.random_forest(4, 300, 200), gg.paper_fig3()]
    graphs += [gg.random_small(3100 + i, int(rng.integers(1, 40)), int(rng.integers(1, 40)),
                               float(rng.uniform(0.05, 1.0))) for i in range(60)]
    for g in graphs:
        want = oracle.total(g)
        for mp in (0, 1, 5, 64):
            t, chunks, wedges = sorted_total(gpu_lib, g, mp)
            assert t == want, (g.name, mp, t, want)
            if mp == 1:
                # one chunk per start with at least one wedge
                assert chunks == int((oracle.vp_wedges(g, per_start=True)[1] > 0).sum())


def test_empty_and_isolated(gpu_lib):
    for g in [gg.Graph(np.zeros((0, 2), np.int32), 4, 7), gg.Graph(np.zeros((0, 2), np.int32), 0, 0),
              gg.from_pairs([(2, 3)], 5, 5)]:
        t, chunks, _ = sorted_total(gpu_lib, g)
        assert t == 0 and chunks == 0


@pytest.mark.parametrize("max_pairs", [0, 1000, 100_000])
def test_power_law_graphs(gpu_lib, max_pairs):
    for g in [gg.chung_lu(41, 3000, 2000, 25000, 2.1, 2.1, 800.0),
              gg.chung_lu(31, 90_000, 70_000, 600_000, 2.0, 2.1, 4000.0, blocks=3, block=40, density=0.9)]:
        t, chunks, wedges, wmax = sorted_total(gpu_lib, g, max_pairs, with_max=True)
        assert t == oracle.total(g)
        if max_pairs:
            # a chunk holds at most max_pairs pairs plus one start's wedges
            assert chunks >= wedges // (max_pairs + wmax) and chunks > 1


def test_matches_hash_count_and_batch(gpu_lib):
    b = gg.concat([gg.random_small(700 + i, 30 + i, 20 + 2 * i, 0.3) for i in range(20)])
    e = torch.from_numpy(b.edges).cuda()
    with gpu_lib.build_batch(e, b.offsets, b.n_upper, b.n_lower) as h:
        per_graph = h.count_total_batch().cpu().numpy()
        t, _ = h.count_total_sorted()
        assert t == int(per_graph.sum())
    g = gg.workload("uniform-2k-3k-20k")
    with gpu_lib.Graph(to_dev(g), g.n_upper, g.n_lower) as h:
        assert h.count_total_sorted()[0] == h.count_total()[0] == oracle.total(g)


@pytest.mark.parametrize("name,max_pairs", [("chunglu-1m-500k-20m", 0), ("chunglu-1m-500k-20m", 1 << 28)])
def test_full_size_workload(gpu_lib, name, max_pairs):
    with open(GOLDEN) as f:
        rec = json.load(f)[name]
    g = gg.workload(name)
    t, chunks, wedges = sorted_total(gpu_lib, g, max_pairs)
    assert wedges == rec["vp_wedges"]
    assert t == rec["total"]
    assert chunks >= (2 if max_pairs else 1)
