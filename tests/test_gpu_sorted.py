"""Sort-based total count (Algorithm 6 with device memory for disk) from the
HIP library against the oracle (Lemma 1), over the wedges of Algorithm 2
(direction 0) and of Algorithm 3 (direction 1, BFC-VP++): exact int64 totals
and pair counts (the oracle's processed-wedge counts of each algorithm) on
small and power-law graphs, with chunk limits that split the start ranges
into many chunks (down to one pair, so every start with wedges is a chunk of
its own), on a batch (the sum over its graphs) and on the benchmark workload
against the oracle's stored total and |W|.
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


def sorted_total(bfc, g, max_pairs=0, direction=0):
    with bfc.Graph(to_dev(g), g.n_upper, g.n_lower) as h:
        return h.count_total_sorted(max_pairs, direction=direction)


def wedges_of(g, direction, per_start=False):
    return (oracle.vpp_wedges if direction else oracle.vp_wedges)(g, per_start=per_start)


@pytest.mark.parametrize("direction", [0, 1])
def test_small_graphs(gpu_lib, direction):
    rng = np.random.default_rng(31)
    graphs = [gg.complete_bipartite(a, b) for a, b in [(1, 1), (2, 2), (3, 5), (17, 9), (64, 64), (300, 100)]]
    graphs += [gg.even_cycle(2), gg.even_cycle(9), gg.random_forest(4, 300, 200), gg.paper_fig3()]
    graphs += [gg.random_small(3100 + i, int(rng.integers(1, 40)), int(rng.integers(1, 40)),
                               float(rng.uniform(0.05, 1.0))) for i in range(60)]
    for g in graphs:
        want = oracle.total(g)
        wedges, per = wedges_of(g, direction, per_start=True)
        for mp in (0, 1, 5, 64):
            t, pairs, chunks = sorted_total(gpu_lib, g, mp, direction)
            assert t == want and pairs == wedges, (g.name, mp, t, want, pairs, wedges)
            if mp == 1:
                # one chunk per start with at least one wedge
                assert chunks == int((per > 0).sum())


def test_empty_and_isolated(gpu_lib):
    for g in [gg.Graph(np.zeros((0, 2), np.int32), 4, 7), gg.Graph(np.zeros((0, 2), np.int32), 0, 0),
              gg.from_pairs([(2, 3)], 5, 5)]:
        for d in (0, 1):
            t, pairs, chunks = sorted_total(gpu_lib, g, 0, d)
            assert t == 0 and pairs == 0 and chunks == 0


@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("max_pairs", [0, 1000, 100_000])
def test_power_law_graphs(gpu_lib, max_pairs, direction):
    for g in [gg.chung_lu(41, 3000, 2000, 25000, 2.1, 2.1, 800.0),
              gg.chung_lu(31, 90_000, 70_000, 600_000, 2.0, 2.1, 4000.0, blocks=3, block=40, density=0.9)]:
        t, pairs, chunks = sorted_total(gpu_lib, g, max_pairs, direction)
        wedges, per = wedges_of(g, direction, per_start=True)
        assert t == oracle.total(g) and pairs == wedges
        if max_pairs:
            # a chunk holds at most max_pairs pairs plus one start's wedges
            assert chunks >= wedges // (max_pairs + int(per.max())) and chunks > 1


def test_matches_hash_count_and_batch(gpu_lib):
    b = gg.concat([gg.random_small(700 + i, 30 + i, 20 + 2 * i, 0.3) for i in range(20)])
    e = torch.from_numpy(b.edges).cuda()
    with gpu_lib.build_batch(e, b.offsets, b.n_upper, b.n_lower) as h:
        per_graph = h.count_total_batch().cpu().numpy()
        for d in (0, 1):
            t, pairs, _ = h.count_total_sorted(direction=d)
            assert t == int(per_graph.sum()) and pairs == int(h.batch_wedges().sum())
    g = gg.workload("uniform-2k-3k-20k")
    with gpu_lib.Graph(to_dev(g), g.n_upper, g.n_lower) as h:
        assert h.count_total_sorted()[0] == h.count_total()[0] == oracle.total(g)
        assert h.count_total_sorted(direction=1)[0] == oracle.total(g)
        with pytest.raises(gpu_lib.BfcError) as e:
            h.count_total_sorted(direction=2)
        assert e.value.status == 1


@pytest.mark.parametrize("direction,max_pairs", [(0, 0), (0, 1 << 28), (1, 0)])
def test_full_size_workload(gpu_lib, direction, max_pairs):
    name = "chunglu-1m-500k-20m"
    with open(GOLDEN) as f:
        rec = json.load(f)[name]
    g = gg.workload(name)
    t, pairs, chunks = sorted_total(gpu_lib, g, max_pairs, direction)
    # Lemma 3: both directions process |W| wedges
    assert pairs == rec["vp_wedges"]
    assert t == rec["total"]
    assert chunks >= (3 if max_pairs else 1)
