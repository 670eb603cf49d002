"""Parity of the HIP path with the CPU oracle (bit-exact: the path is integer).

Every case runs bfc_build, bfc_count_total, bfc_count_per_vertex and
bfc_count_per_edge through the C ABI and compares each output element by
element with the oracle's plain definitions (Lemma 1, Eq. 8), and |W| with
the oracle's count of the wedges Algorithm 2 processes.
"""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
from gpu_util import check_against_oracle, gpu_all, to_dev

pytestmark = pytest.mark.gpu


def test_paper_fig3(gpu_lib):
    g = gg.paper_fig3()
    tot, wed, up, lo, be = gpu_all(gpu_lib, g)
    assert tot == 999000 and wed == 2000
    assert up[0] == up[1] == lo[1000] == lo[1001] == 499500
    assert (up[2:] == 999).all() and (lo[:1000] == 999).all() and (be == 999).all()
    check_against_oracle(gpu_lib, g)


def test_paper_fig2a(gpu_lib):
    g = gg.paper_fig2a()
    tot, wed, up, lo, be = gpu_all(gpu_lib, g)
    assert tot == 0 and wed == 2000
    assert not up.any() and not lo.any() and not be.any()


@pytest.mark.parametrize("a,b", [(1, 1), (2, 2), (3, 5), (17, 9), (64, 64), (100, 300), (700, 20)])
def test_complete_bipartite(gpu_lib, a, b):
    g = gg.complete_bipartite(a, b)
    c2 = lambda k: k * (k - 1) // 2
    tot, wed, up, lo, be = gpu_all(gpu_lib, g)
    assert tot == c2(a) * c2(b)
    assert (up == (a - 1) * c2(b)).all() and (lo == (b - 1) * c2(a)).all()
    assert (be == (a - 1) * (b - 1)).all()
    assert wed == oracle.vp_wedges(g)


def test_zero_butterfly_graphs(gpu_lib):
    for g in [gg.even_cycle(3), gg.even_cycle(40), gg.random_forest(1, 500, 300), gg.random_forest(2, 50, 900)]:
        tot, wed, up, lo, be = gpu_all(gpu_lib, g)
        assert tot == 0 and not up.any() and not lo.any() and not be.any()
        assert wed == oracle.vp_wedges(g)
    tot, *_ = gpu_all(gpu_lib, gg.even_cycle(2))
    assert tot == 1


def test_random_tiny_graphs(gpu_lib):
    rng = np.random.default_rng(77)
    for i in range(120):
        g = gg.random_small(9000 + i, int(rng.integers(1, 12)), int(rng.integers(1, 12)),
                            float(rng.choice([0.2, 0.5, 0.8, 1.0])))
        check_against_oracle(gpu_lib, g)


def test_random_tiny_graphs_vpp(gpu_lib):
    """Algorithm 3's wedges: the same outputs, and |W| equal to Algorithm 2's
    (Lemma 3), on every tiny graph and on each kernel path."""
    rng = np.random.default_rng(78)
    for i in range(120):
        g = gg.random_small(9500 + i, int(rng.integers(1, 12)), int(rng.integers(1, 12)),
                            float(rng.choice([0.2, 0.5, 0.8, 1.0])))
        tun = [{"vpp": 3}, {"vpp": 3, "light_max_wedges": 1}, {"vpp": 3, "light_max_wedges": 1, "window_mode": 3,
                                                                 "hash_window_wedges": 4},
               {"vpp": 1, "light_max_wedges": 1}, {"vpp": 2}][i % 5]
        check_against_oracle(gpu_lib, g, tun)
        assert oracle.vpp_wedges(g) == oracle.vp_wedges(g)


def test_random_tiny_graphs_band(gpu_lib):
    """Top bands of every width on tiny graphs: the same outputs and |W| as
    Algorithm 2's, on each kernel path."""
    rng = np.random.default_rng(79)
    for i in range(120):
        g = gg.random_small(9700 + i, int(rng.integers(1, 12)), int(rng.integers(1, 12)),
                            float(rng.choice([0.2, 0.5, 0.8, 1.0])))
        band = int(rng.integers(1, 12))
        tun = [{"top_band": band}, {"top_band": band, "light_max_wedges": 1},
               {"top_band": band, "light_max_wedges": 1, "window_mode": 3, "hash_window_wedges": 4},
               {"top_band": band, "light_max_wedges": 1, "window_mode": 2},
               {"top_band": band, "vpp": 2}][i % 5]
        check_against_oracle(gpu_lib, g, tun)


def test_union_of_many_small_graphs(gpu_lib):
    rng = np.random.default_rng(5)
    parts, ou, ol = [], 0, 0
    for i in range(1500):
        nu, nl = int(rng.integers(1, 30)), int(rng.integers(1, 30))
        g = gg.random_small(20000 + i, nu, nl, float(rng.uniform(0.05, 0.9)))
        parts.append(g.edges + np.array([ou, ol], np.int32))
        ou += nu
        ol += nl
    e = np.concatenate(parts)
    e = e[np.random.default_rng(6).permutation(len(e))]
    big = gg.Graph(np.ascontiguousarray(e), ou, ol, "union")
    check_against_oracle(gpu_lib, big)


def test_uniform_workload_2k_3k_20k(gpu_lib):
    check_against_oracle(gpu_lib, gg.workload("uniform-2k-3k-20k"))


@pytest.fixture(scope="module")
def hub_graph():
    # hubs in both layers, layers wider than one dense window (32K ranks)
    return gg.chung_lu(31, 90_000, 70_000, 600_000, 2.0, 2.1, 4000.0, blocks=3, block=40, density=0.9, name="hubs")


@pytest.fixture(scope="module")
def hub_oracle(hub_graph):
    g = hub_graph
    up, lo = oracle.vertex_counts(g)
    return oracle.total(g), oracle.vp_wedges(g), up, lo, oracle.edge_counts(g)


TUNINGS = {
    "default": {},
    # wavefront starts up to 1024 wedges only (the limit of unpacked tables)
    "light-1024": {"light_max_wedges": 1024},
    "all-workgroup": {"light_max_wedges": 1},
    "dense-windows": {"light_max_wedges": 16, "window_mode": 2},
    "hash-windows": {"light_max_wedges": 16, "window_mode": 3},
    "hash-tiny-windows": {"light_max_wedges": 1, "window_mode": 3, "hash_window_wedges": 64},
    "hash-overfull": {"light_max_wedges": 64, "window_mode": 3, "hash_window_wedges": 1 << 30},
    "dense-ratio-1": {"dense_min_ratio": 1},
    "mfma-block-64": {"dense_block": 64},
    "mfma-block-1024": {"dense_block": 1024, "light_max_wedges": 64},
    "mfma-block-4096-hash": {"dense_block": 4096, "window_mode": 3, "hash_window_wedges": 512},
    "mfma-block-32768": {"dense_block": 32768},
    # dense starts with a hash window over their low end ranks: a prefix
    # sized for far too many wedges (split by halving), and small prefixes
    "auto-prefix-overfull": {"light_max_wedges": 64, "hash_window_wedges": 1 << 30},
    "auto-prefix-small": {"light_max_wedges": 64, "dense_min_wedges": 256, "hash_window_wedges": 2048},
    # 256-thread workgroups for small workgroup starts: off, hash windows,
    # tiny (halving) hash windows, and next to the dense block
    "medium-off": {"medium_max_wedges": 0},
    "medium-hash": {"light_max_wedges": 16, "window_mode": 3, "medium_max_wedges": 1 << 30},
    "medium-hash-tiny": {"light_max_wedges": 1, "window_mode": 3, "hash_window_wedges": 32,
                         "medium_max_wedges": 1 << 30},
    "medium-dense-block": {"light_max_wedges": 64, "dense_block": 1024, "medium_max_wedges": 1 << 30},
    # Algorithm 3's wedges (BFC-VP++) through the same kernel paths: ends
    # above the start, middles every neighbour
    "vpp": {"vpp": 3},
    "vpp-light-1024": {"vpp": 3, "light_max_wedges": 1024},
    "vpp-all-workgroup": {"vpp": 3, "light_max_wedges": 1},
    "vpp-dense-windows": {"vpp": 3, "light_max_wedges": 16, "window_mode": 2},
    "vpp-hash-windows": {"vpp": 3, "light_max_wedges": 16, "window_mode": 3},
    "vpp-hash-tiny-windows": {"vpp": 3, "light_max_wedges": 1, "window_mode": 3, "hash_window_wedges": 64},
    "vpp-hash-overfull": {"vpp": 3, "light_max_wedges": 64, "window_mode": 3, "hash_window_wedges": 1 << 30},
    "vpp-dense-ratio-1": {"vpp": 3, "dense_min_ratio": 1},
    "vpp-auto-prefix-overfull": {"vpp": 3, "light_max_wedges": 64, "hash_window_wedges": 1 << 30},
    "vpp-auto-prefix-small": {"vpp": 3, "light_max_wedges": 64, "dense_min_wedges": 256,
                              "hash_window_wedges": 2048},
    # (medium_max_wedges is ignored under vpp: these run on 1024-thread workgroups)
    "vpp-medium-hash": {"vpp": 3, "light_max_wedges": 16, "window_mode": 3, "medium_max_wedges": 1 << 30},
    "vpp-medium-hash-tiny": {"vpp": 3, "light_max_wedges": 1, "window_mode": 3, "hash_window_wedges": 32,
                             "medium_max_wedges": 1 << 30},
    "vpp-ignores-dense-block": {"vpp": 3, "dense_block": 1024, "light_max_wedges": 64},
    # one layer's starts each way (a butterfly's counted pair lies in the
    # layer of its top vertex, so any mix is exact)
    "vpp-upper-only": {"vpp": 1},
    "vpp-lower-only": {"vpp": 2, "light_max_wedges": 64},
    # top bands: a pair with only its higher vertex in the band is counted
    # from the lower one with Algorithm 3's wedges into the band
    "band-64": {"top_band": 64},
    "band-777-odd": {"top_band": 777, "light_max_wedges": 64},
    "band-4096": {"top_band": 4096},
    "band-65536": {"top_band": 65536},
    "band-light-1024": {"top_band": 4096, "light_max_wedges": 1024},
    "band-all-workgroup": {"top_band": 4096, "light_max_wedges": 1},
    "band-dense-windows": {"top_band": 4096, "light_max_wedges": 16, "window_mode": 2},
    "band-hash-windows": {"top_band": 4096, "light_max_wedges": 16, "window_mode": 3},
    "band-hash-tiny-windows": {"top_band": 30000, "light_max_wedges": 1, "window_mode": 3,
                               "hash_window_wedges": 64},
    "band-hash-overfull": {"top_band": 4096, "light_max_wedges": 64, "window_mode": 3,
                           "hash_window_wedges": 1 << 30},
    "band-auto-prefix-small": {"top_band": 30000, "light_max_wedges": 64, "dense_min_wedges": 256,
                               "hash_window_wedges": 2048},
    # (the dense block and the 256-thread shape are not used with a band)
    "band-ignores-dense-block": {"top_band": 4096, "dense_block": 1024, "light_max_wedges": 64},
    "band-medium-ignored": {"top_band": 4096, "light_max_wedges": 16, "window_mode": 3,
                            "medium_max_wedges": 1 << 30},
    # a band in the lower layer only (the upper layer takes Algorithm 3's wedges)
    "band-with-vpp-upper": {"top_band": 4096, "vpp": 1},
}


@pytest.mark.parametrize("name", list(TUNINGS))
def test_hub_graph_every_kernel_path(gpu_lib, hub_graph, hub_oracle, name):
    tun = TUNINGS[name]
    tot, wed, up, lo, be = gpu_all(gpu_lib, hub_graph, tun or None)
    if (tun.get("vpp") or tun.get("top_band")) and tun.get("medium_max_wedges"):
        with gpu_lib.Graph(to_dev(hub_graph), hub_graph.n_upper, hub_graph.n_lower) as h:
            h.set_tuning(**tun)
            assert h.schedule_info()["starts_medium"] == 0
    o_tot, o_wed, o_up, o_lo, o_be = hub_oracle
    assert tot == o_tot and wed == o_wed
    np.testing.assert_array_equal(up, o_up)
    np.testing.assert_array_equal(lo, o_lo)
    np.testing.assert_array_equal(be, o_be)


def test_byte_counters_at_their_limit(gpu_lib):
    """Ends of degree below 256 count in 8-bit dense counters: complete
    bipartite graphs where a pair's count reaches exactly 255 (and layers of
    degree 256, which keep 16-bit counters), and small degrees, on dense
    windows and defaults."""
    for a, b in [(300, 255), (255, 300), (256, 256), (257, 255), (40, 255), (60, 15), (15, 60), (16, 16),
                 (50, 3), (3, 50), (4, 4), (17, 4)]:
        g = gg.complete_bipartite(a, b)
        for tun in (None, {"light_max_wedges": 1, "window_mode": 2}, {"light_max_wedges": 1, "vpp": 3}):
            check_against_oracle(gpu_lib, g, tun)


def test_byte_counters_in_wide_end_ranges(gpu_lib):
    """A start keeps 8-bit windows only where they save a window, which the
    small graphs above never reach.  Here the same blocks sit above 300,000
    isolated edges, so a block start's end range spans three 8-bit windows
    (five 16-bit ones) and its ends, of degree 255 or less, count up to 255
    in the third; also on defaults, where a hash prefix may take the padding."""
    pad = 300_000
    iu = np.arange(pad, dtype=np.int32)
    for a, b in [(40, 255), (255, 255), (3, 255), (255, 3)]:
        k = gg.complete_bipartite(a, b)
        e = np.concatenate([k.edges, np.stack([a + iu, b + iu], axis=1)]).astype(np.int32)
        g = gg.Graph(np.ascontiguousarray(e), a + pad, b + pad, f"K{a},{b}+{pad} isolated edges")
        for tun in ({"light_max_wedges": 1, "window_mode": 2}, None):
            check_against_oracle(gpu_lib, g, tun)


def test_mfma_block_covers_whole_small_graphs(gpu_lib):
    """Block sizes at or above the layer sizes: every start is in the block."""
    for a, b in [(3, 5), (40, 60), (64, 64), (100, 37)]:
        g = gg.complete_bipartite(a, b)
        for k in (64, 128):
            check_against_oracle(gpu_lib, g, {"dense_block": k})
    rng = np.random.default_rng(3)
    for i in range(30):
        g = gg.random_small(4000 + i, int(rng.integers(2, 70)), int(rng.integers(2, 70)), float(rng.uniform(0.1, 0.9)))
        check_against_oracle(gpu_lib, g, {"dense_block": 64, "light_max_wedges": 1 + i % 3})


def test_mfma_block_planted_bicliques(gpu_lib):
    g = gg.chung_lu(77, 20_000, 15_000, 300_000, 2.0, 2.3, 3000.0, blocks=8, block=96, density=0.9, name="planted")
    for k in (0, 256, 2048):
        check_against_oracle(gpu_lib, g, {"dense_block": k} if k else None)


def test_repeat_and_async_and_streams(gpu_lib, hub_graph, hub_oracle):
    o_tot = hub_oracle[0]
    with gpu_lib.Graph(to_dev(hub_graph), hub_graph.n_upper, hub_graph.n_lower) as h:
        out = torch.zeros(1, dtype=torch.int64, device="cuda")
        s2 = torch.cuda.Stream()
        for _ in range(3):
            assert h.count_total()[0] == o_tot
            h.count_total_async(out)
            torch.cuda.synchronize()
            assert int(out.item()) == o_tot
            assert h.count_total(stream=s2)[0] == o_tot
        info = h.info()
        assert info["m"] == hub_graph.m and info["wedges"] == hub_oracle[1]
        assert info["device_bytes"] <= gpu_lib.estimate_device_bytes(hub_graph.m, hub_graph.n_upper,
                                                                     hub_graph.n_lower)


def test_empty_and_degenerate_inputs(gpu_lib):
    empty = gg.Graph(np.zeros((0, 2), np.int32), 4, 7)
    tot, wed, up, lo, be = gpu_all(gpu_lib, empty)
    assert tot == 0 and wed == 0 and up.shape == (4,) and lo.shape == (7,) and be.shape == (0,)
    nothing = gg.Graph(np.zeros((0, 2), np.int32), 0, 0)
    tot, wed, up, lo, be = gpu_all(gpu_lib, nothing)
    assert tot == 0 and up.shape == (0,) and lo.shape == (0,)
    one = gg.from_pairs([(2, 3)], 5, 5)
    tot, wed, up, lo, be = gpu_all(gpu_lib, one)
    assert tot == 0 and wed == 0 and be.tolist() == [0]
    star = gg.from_pairs([(0, v) for v in range(5000)], 1, 5000)
    tot, wed, *_ = gpu_all(gpu_lib, star)
    assert tot == 0 and wed == 0
    # isolated vertices around a K_{3,3}
    k = gg.complete_bipartite(3, 3)
    iso = gg.Graph(k.edges + np.array([10, 20], np.int32), 40, 60)
    tot, wed, up, lo, be = gpu_all(gpu_lib, iso)
    assert tot == 9 and up[10:13].tolist() == [6, 6, 6] and up.sum() == 18 and (be == 4).all()


def test_input_errors(gpu_lib):
    bad = torch.tensor([[0, 0], [5, 1]], dtype=torch.int32, device="cuda")
    with pytest.raises(gpu_lib.BfcError) as e:
        gpu_lib.Graph(bad, 5, 5)
    assert e.value.status == 2
    neg = torch.tensor([[0, -1]], dtype=torch.int32, device="cuda")
    with pytest.raises(gpu_lib.BfcError) as e:
        gpu_lib.Graph(neg, 5, 5)
    assert e.value.status == 2
    dup = torch.tensor([[1, 2], [0, 0], [1, 2]], dtype=torch.int32, device="cuda")
    with pytest.raises(gpu_lib.BfcError) as e:
        gpu_lib.Graph(dup, 5, 5)
    assert e.value.status == 3
    # the library stays usable after errors
    tot, *_ = gpu_all(gpu_lib, gg.complete_bipartite(4, 4))
    assert tot == 36


def test_per_edge_wide_accumulators(gpu_lib):
    """Two hubs of degree 70,000 in opposite layers: (d_u - 1)(d_v - 1) can
    reach 2^32, so per-edge counts use 64-bit accumulators (every other graph
    here fits the 32-bit ones)."""
    rng = np.random.default_rng(123)
    pairs = {(0, v) for v in range(70_000)} | {(u, 0) for u in range(70_000)}
    for u in range(1, 300):
        for v in rng.choice(np.arange(1, 300), 15, replace=False):
            pairs.add((u, int(v)))
    e = np.array(sorted(pairs), np.int32)
    e = e[rng.permutation(len(e))]
    g = gg.Graph(np.ascontiguousarray(e), 70_000, 70_000, "two-hubs")
    du = np.bincount(e[:, 0], minlength=g.n_upper)
    dl = np.bincount(e[:, 1], minlength=g.n_lower)
    assert (int(du.max()) - 1) * (int(dl.max()) - 1) >= 1 << 32
    check_against_oracle(gpu_lib, g)
