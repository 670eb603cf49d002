"""Batched form: many graphs in one handle, counted by one set of launches.

Per-graph totals and |W| from bfc_build_batch / bfc_count_total_batch must
equal the oracle's per-graph values, and equal a one-graph-per-handle loop
(bfc_build + bfc_count_total).  The captured HIP graph replays must give
the same totals every time, with eager work in between.
"""
import json
import os

import numpy as np
import pytest
import torch

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "batch.json")


def small_batch(count=60, seed=11):
    rng = np.random.default_rng(seed)
    graphs = []
    for i in range(count):
        kind = i % 4
        if kind == 0:
            g = gg.random_small(seed * 1000 + i, int(rng.integers(1, 25)), int(rng.integers(1, 25)), 0.4)
        elif kind == 1:
            g = gg.complete_bipartite(int(rng.integers(1, 20)), int(rng.integers(1, 20)))
        elif kind == 2:
            g = gg.chung_lu(seed * 1000 + i, 3000, 2000, int(rng.integers(1000, 30000)), 2.1, 2.1, 800.0)
        else:
            g = gg.Graph(np.zeros((0, 2), np.int32), int(rng.integers(0, 5)), int(rng.integers(0, 5)))
        graphs.append(g)
    return graphs


def test_small_batch_matches_oracle_and_plain_loop(gpu_lib):
    graphs = small_batch()
    b = gg.concat(graphs)
    with gpu_lib.build_batch(torch.from_numpy(b.edges).cuda(), b.offsets, b.n_upper, b.n_lower) as h:
        totals = h.count_total_batch().cpu().numpy()
        wedges = h.batch_wedges()
        up, lo = h.count_per_vertex()
        be = h.count_per_edge()
        up, lo, be = up.cpu().numpy(), lo.cpu().numpy(), be.cpu().numpy()
    ou = ol = 0
    for i, g in enumerate(graphs):
        assert totals[i] == oracle.total(g), i
        assert wedges[i] == oracle.vp_wedges(g), i
        o_up, o_lo = oracle.vertex_counts(g)
        np.testing.assert_array_equal(up[ou:ou + g.n_upper], o_up)
        np.testing.assert_array_equal(lo[ol:ol + g.n_lower], o_lo)
        np.testing.assert_array_equal(be[b.offsets[i]:b.offsets[i + 1]], oracle.edge_counts(g))
        ou += g.n_upper
        ol += g.n_lower
        if g.m:
            with gpu_lib.Graph(torch.from_numpy(g.edges).cuda(), g.n_upper, g.n_lower) as p:
                assert p.count_total() == (int(totals[i]), int(wedges[i]))


def test_small_batch_vpp(gpu_lib):
    """Algorithm 3's wedges on a batch: each start's ends stay inside its
    graph's ranks (above the start), so per-graph outputs are unchanged."""
    graphs = small_batch(48, seed=13)
    b = gg.concat(graphs)
    with gpu_lib.build_batch(torch.from_numpy(b.edges).cuda(), b.offsets, b.n_upper, b.n_lower) as h:
        for tun in ({"vpp": 3}, {"vpp": 3, "light_max_wedges": 1, "window_mode": 3, "hash_window_wedges": 16}):
            h.set_tuning(**tun)
            totals = h.count_total_batch().cpu().numpy()
            up, lo = h.count_per_vertex()
            be = h.count_per_edge()
            up, lo, be = up.cpu().numpy(), lo.cpu().numpy(), be.cpu().numpy()
            ou = ol = 0
            for i, g in enumerate(graphs):
                assert totals[i] == oracle.total(g), (i, tun)
                o_up, o_lo = oracle.vertex_counts(g)
                np.testing.assert_array_equal(up[ou:ou + g.n_upper], o_up)
                np.testing.assert_array_equal(lo[ol:ol + g.n_lower], o_lo)
                np.testing.assert_array_equal(be[b.offsets[i]:b.offsets[i + 1]], oracle.edge_counts(g))
                ou += g.n_upper
                ol += g.n_lower


def test_wide_batch_graph_local_keys(gpu_lib):
    """A batch whose upper layer has more than 2^20 vertices in all, every
    graph below 2^20: the light tables pack keys counted from each graph's
    first rank.  Every output, with both wedge directions, must equal the
    oracle's."""
    graphs = [gg.chung_lu(500 + i, 100_000, 60_000, 150_000, 2.1, 2.1, 600.0) for i in range(11)]
    b = gg.concat(graphs)
    assert sum(b.n_upper) >= (1 << 20) and max(b.n_upper) < (1 << 20)
    print(f"wide batch: {len(graphs)} graphs, {sum(b.n_upper)} upper, {b.offsets[-1]} edges", flush=True)
    with gpu_lib.build_batch(torch.from_numpy(b.edges).cuda(), b.offsets, b.n_upper, b.n_lower) as h:
        for tun in ({}, {"vpp": 3}):
            if tun:
                h.set_tuning(**tun)
            totals = h.count_total_batch().cpu().numpy()
            up, lo = h.count_per_vertex()
            be = h.count_per_edge()
            up, lo, be = up.cpu().numpy(), lo.cpu().numpy(), be.cpu().numpy()
            ou = ol = 0
            for i, g in enumerate(graphs):
                assert totals[i] == oracle.total(g), (i, tun)
                o_up, o_lo = oracle.vertex_counts(g)
                np.testing.assert_array_equal(up[ou:ou + g.n_upper], o_up)
                np.testing.assert_array_equal(lo[ol:ol + g.n_lower], o_lo)
                np.testing.assert_array_equal(be[b.offsets[i]:b.offsets[i + 1]], oracle.edge_counts(g))
                ou += g.n_upper
                ol += g.n_lower


def test_per_graph_tuning(gpu_lib):
    """Per-graph settings (what the tuner installs per bucket): every output
    unchanged, through a captured and replayed count too."""
    graphs = small_batch(48, seed=14)
    b = gg.concat(graphs)
    rng = np.random.default_rng(15)
    per = []
    for i in range(len(graphs)):
        per.append({"light_max_wedges": int(rng.choice([1, 16, 256, 2048])),
                    "window_mode": int(rng.choice([1, 2, 3])),
                    "hash_window_wedges": int(rng.choice([16, 512, 8192])),
                    "dense_min_ratio": int(rng.choice([1, 4, 64])),
                    "dense_min_wedges": int(rng.choice([64, 8192]))})
    expect = np.array([oracle.total(g) for g in graphs], np.int64)
    s = torch.cuda.Stream()
    with gpu_lib.build_batch(torch.from_numpy(b.edges).cuda(), b.offsets, b.n_upper, b.n_lower, stream=s) as h:
        h.set_graph_tuning(per)
        tot = h.count_total_batch(stream=s)
        s.synchronize()
        assert (tot.cpu().numpy() == expect).all()
        up, lo = h.count_per_vertex(stream=s)
        be = h.count_per_edge(stream=s)
        up, lo, be = up.cpu().numpy(), lo.cpu().numpy(), be.cpu().numpy()
        ou = ol = 0
        for i, g in enumerate(graphs):
            o_up, o_lo = oracle.vertex_counts(g)
            np.testing.assert_array_equal(up[ou:ou + g.n_upper], o_up)
            np.testing.assert_array_equal(lo[ol:ol + g.n_lower], o_lo)
            np.testing.assert_array_equal(be[b.offsets[i]:b.offsets[i + 1]], oracle.edge_counts(g))
            ou += g.n_upper
            ol += g.n_lower
        out = torch.zeros(len(graphs), dtype=torch.int64, device="cuda")
        h.capture_total(out, stream=s)
        for _ in range(3):
            out.fill_(-1)
            torch.cuda.synchronize()
            h.replay(stream=s)
            torch.cuda.synchronize()
            assert (out.cpu().numpy() == expect).all()
        h.set_graph_tuning([])  # back to the handle's settings
        tot = h.count_total_batch(stream=s)
        s.synchronize()
        assert (tot.cpu().numpy() == expect).all()
        with pytest.raises(gpu_lib.BfcError) as err:
            h.set_graph_tuning(per[:-1])
        assert err.value.status == 1
    g = graphs[2]
    with gpu_lib.Graph(torch.from_numpy(g.edges).cuda(), g.n_upper, g.n_lower) as h1:
        with pytest.raises(gpu_lib.BfcError) as err:
            h1.set_graph_tuning([{}])
        assert err.value.status == 1


def test_batch_errors(gpu_lib):
    e = torch.tensor([[0, 0], [1, 1], [2, 0]], dtype=torch.int32, device="cuda")
    with pytest.raises(gpu_lib.BfcError) as err:   # edge 2 is outside graph 1's upper layer
        gpu_lib.build_batch(e, [0, 2, 3], [2, 2], [2, 2])
    assert err.value.status == 2
    with pytest.raises(gpu_lib.BfcError) as err:   # duplicate inside graph 0
        gpu_lib.build_batch(torch.tensor([[0, 0], [0, 0]], dtype=torch.int32, device="cuda"), [0, 2], [2], [2])
    assert err.value.status == 3


def test_capture_and_replay(gpu_lib):
    graphs = small_batch(40, seed=12)
    b = gg.concat(graphs)
    expect = np.array([oracle.total(g) for g in graphs], np.int64)
    with gpu_lib.build_batch(torch.from_numpy(b.edges).cuda(), b.offsets, b.n_upper, b.n_lower) as h:
        h.set_tuning(light_max_wedges=64)
        out = torch.full((len(graphs),), -1, dtype=torch.int64, device="cuda")
        with pytest.raises(gpu_lib.BfcError) as err:  # the default stream cannot be captured
            h.capture_total(out, stream=torch.cuda.default_stream())
        assert err.value.status == 1
        s = torch.cuda.Stream()
        h.capture_total(out, stream=s)
        for k in range(4):
            out.fill_(-7)
            torch.cuda.synchronize()
            h.replay(stream=s)
            s.synchronize()
            np.testing.assert_array_equal(out.cpu().numpy(), expect)
            # eager work between replays, on the same handle
            eager = h.count_total_batch().cpu().numpy()
            np.testing.assert_array_equal(eager, expect)
            assert h.count_total()[0] == int(expect.sum())


def test_batch_4096_workload(gpu_lib):
    if not os.path.exists(GOLDEN):
        pytest.skip("no stored oracle results")
    with open(GOLDEN) as f:
        rec = json.load(f).get("batch-4096")
    if rec is None:
        pytest.skip("no stored oracle results for the batch")
    b = gg.batch_workload()
    print(f"batch: {b.count} graphs, {int(b.offsets[-1])} edges", flush=True)
    assert b.sha256() == rec["sha256"]
    with gpu_lib.build_batch(torch.from_numpy(b.edges).cuda(), b.offsets, b.n_upper, b.n_lower) as h:
        totals = h.count_total_batch().cpu().numpy()
        wedges = h.batch_wedges()
    np.testing.assert_array_equal(totals, np.array(rec["totals"], np.int64))
    np.testing.assert_array_equal(wedges, np.array(rec["vp_wedges"], np.int64))
