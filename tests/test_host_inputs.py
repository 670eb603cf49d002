"""The seeded input recipes (no GPU needed): the served trace, the batch of
graphs and the Chung-Lu generator have the shapes and distributions their
descriptions state."""
import math

import numpy as np

import graphgen as gg


def test_serve_schedule_is_a_poisson_trace_with_the_stated_mix():
    reqs = gg.serve_schedule(rate=200.0, duration_s=60.0)
    t = np.array([r.arrival_s for r in reqs])
    assert np.all(np.diff(t) > 0) and t[0] > 0 and t[-1] <= 60.0
    # about rate x duration requests (Poisson: sd = sqrt(12000) ~ 110)
    assert abs(len(reqs) - 12_000) < 5 * math.sqrt(12_000)
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert abs(gaps.mean() - 1 / 200.0) < 0.05 / 200.0
    # exponential gaps: the coefficient of variation is about 1
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.05
    kinds = np.array([r.kind for r in reqs])
    for k, p in (("total", 0.6), ("vertex", 0.25), ("edge", 0.15)):
        assert abs((kinds == k).mean() - p) < 0.02
    fu = np.array([r.follow_up_of >= 0 for r in reqs])
    assert abs(fu.mean() - 0.3) < 0.02
    for r in reqs:
        if r.follow_up_of >= 0:
            root = reqs[r.follow_up_of]
            assert root.follow_up_of == -1 and root.index < r.index and root.graph == r.graph
        else:
            g = r.graph
            assert 10_000 <= g.m <= 50_000_000 and 2.0 <= g.gamma <= 2.5
            assert g.n_upper >= 2 and g.n_lower >= 2 and g.n_upper * g.n_lower >= g.m
    # same seed, same trace
    again = gg.serve_schedule(rate=200.0, duration_s=60.0)
    assert [(r.arrival_s, r.kind, r.graph) for r in again] == [(r.arrival_s, r.kind, r.graph) for r in reqs]


def test_batch_specs_are_log_uniform_and_alternate_kinds():
    specs = gg.batch_specs()
    assert len(specs) == 4096
    m = np.array([s.m for s in specs], dtype=np.float64)
    assert m.min() >= 1_000 and m.max() <= 1_000_000
    # log-uniform over three decades: each decade holds about a third
    dec = np.floor(np.log10(m)).clip(3, 5)
    for d in (3, 4, 5):
        assert abs((dec == d).mean() - 1 / 3) < 0.04
    assert [s.kind for s in specs[:4]] == ["uniform", "chung_lu", "uniform", "chung_lu"]
    assert len({s.seed for s in specs}) == len(specs)
    for s in specs[:200]:
        assert s.n_upper * s.n_lower >= s.m
        assert 0.2 <= s.n_upper / s.n_lower <= 5.0


def test_concat_lays_graphs_back_to_back():
    gs = [gg.uniform(5 + i, 30 + i, 40, 100 + 10 * i) for i in range(5)]
    b = gg.concat(gs)
    assert b.count == 5 and b.offsets[0] == 0 and b.offsets[-1] == sum(g.m for g in gs)
    for i, g in enumerate(gs):
        np.testing.assert_array_equal(b.graph(i).edges, g.edges)
        assert b.n_upper[i] == g.n_upper and b.n_lower[i] == g.n_lower


def test_chung_lu_degrees_are_heavy_tailed():
    g = gg.chung_lu(21, 200_000, 100_000, 2_000_000, 2.1, 2.1, 20_000.0)
    du = np.bincount(g.edges[:, 0], minlength=g.n_upper)
    dl = np.bincount(g.edges[:, 1], minlength=g.n_lower)
    for d in (du, dl):
        mean = d.mean()
        assert d.max() > 100 * mean  # hubs
        assert np.median(d) < mean  # most vertices below the mean
        # a power-law tail: the top 1% of vertices hold a large share of the edges
        top = np.sort(d)[::-1][: len(d) // 100]
        assert top.sum() > 0.2 * d.sum()
