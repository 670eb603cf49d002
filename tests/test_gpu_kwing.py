"""k-wing (Section 1) from the HIP library against the oracle's sequential
peeling: the edge set (bit-exact mask) and every edge's butterfly count
within the k-wing, over thresholds that keep everything, part, or nothing.
At the benchmark's full size the oracle checks sampled edge counts of the
returned subgraph one by one (Eq. 8) and the threshold property on all edges.
"""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
from gpu_util import to_dev

pytestmark = pytest.mark.gpu


def gpu_wing(bfc, g, k):
    mask, cnt, w, r = bfc.k_wing(to_dev(g), g.n_upper, g.n_lower, k)
    torch.cuda.synchronize()
    return mask.cpu().numpy(), cnt.cpu().numpy(), w, r


def check(bfc, g, k):
    mask, cnt, w, r = gpu_wing(bfc, g, k)
    o_mask, o_cnt, removed = oracle.k_wing(g, k)
    np.testing.assert_array_equal(mask, o_mask, err_msg=f"{g.name} k={k}")
    np.testing.assert_array_equal(cnt, o_cnt, err_msg=f"{g.name} k={k}")
    assert w == int(o_mask.sum()) and w == g.m - removed
    assert (r >= 1) == (g.m > 0)
    return w, r


def test_tiny_graphs_every_threshold(gpu_lib):
    rng = np.random.default_rng(8800)
    for i in range(40):
        g = gg.random_small(8800 + i, int(rng.integers(2, 10)), int(rng.integers(2, 10)),
                            float(rng.choice([0.3, 0.6, 0.9, 1.0])))
        top = int(oracle.edge_counts(g).max()) if g.m else 0
        for k in sorted({0, 1, 2, top // 2, top, top + 1}):
            check(gpu_lib, g, k)


def test_bicliques_closed_form(gpu_lib):
    k33, k45 = gg.complete_bipartite(3, 3), gg.complete_bipartite(4, 5)
    e = np.concatenate([k33.edges, k45.edges + np.array([3, 3], np.int32), np.array([[3, 8], [7, 8]], np.int32)])
    g = gg.Graph(np.ascontiguousarray(e), 8, 9, "k33+k45+path")
    for k, want in [(0, g.m), (4, 9 + 20), (5, 20), (12, 20), (13, 0)]:
        mask, cnt, w, r = gpu_wing(gpu_lib, g, k)
        assert w == want == int(mask.sum())
        assert (cnt[:9] == (4 if k <= 4 else 0)).all() and (cnt[9:29] == (12 if k <= 12 else 0)).all()
        assert not mask[29:].any() or k == 0
    check(gpu_lib, g, 5)


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_uniform_workload(gpu_lib, k):
    check(gpu_lib, gg.workload("uniform-2k-3k-20k"), k)


@pytest.mark.parametrize("k", [1, 40, 106, 400, 987])
def test_power_law_graph(gpu_lib, k):
    w, r = check(gpu_lib, gg.chung_lu(41, 3000, 2000, 25000, 2.1, 2.1, 800.0), k)
    if k == 106:
        assert 0 < w < 25000 and r >= 3


@pytest.mark.parametrize("k", [1, 120, 600])
def test_power_law_graph_with_bicliques(gpu_lib, k):
    g = gg.chung_lu(52, 40_000, 30_000, 200_000, 2.0, 2.1, 2000.0, blocks=3, block=30, density=0.9)
    check(gpu_lib, g, k)


def test_empty_degenerate_and_errors(gpu_lib):
    empty = gg.Graph(np.zeros((0, 2), np.int32), 4, 7)
    mask, cnt, w, r = gpu_wing(gpu_lib, empty, 1)
    assert mask.shape == (0,) and w == 0 and r == 0
    forest = gg.random_forest(2, 300, 200)
    mask, cnt, w, r = gpu_wing(gpu_lib, forest, 1)
    assert w == 0 and r == 1 and not mask.any() and not cnt.any()
    mask, cnt, w, r = gpu_wing(gpu_lib, forest, 0)
    assert w == forest.m and r == 1 and mask.all() and not cnt.any()
    dup = torch.tensor([[1, 2], [0, 0], [1, 2]], dtype=torch.int32, device="cuda")
    with pytest.raises(gpu_lib.BfcError) as e:
        gpu_lib.k_wing(dup, 5, 5, 1)
    assert e.value.status == 3
    bad = torch.tensor([[0, 0], [5, 1]], dtype=torch.int32, device="cuda")
    with pytest.raises(gpu_lib.BfcError) as e:
        gpu_lib.k_wing(bad, 5, 5, 1)
    assert e.value.status == 2
    # the library stays usable; without the counts output as well
    g = gg.complete_bipartite(4, 4)
    mask, cnt, w, r = gpu_lib.k_wing(to_dev(g), 4, 4, 9, counts=False)
    assert cnt is None and w == 16 and bool(mask.all())


def _csr(src, dst, n):
    order = np.lexsort((dst, src))
    off = np.zeros(n + 1, np.int64)
    np.add.at(off, src + 1, 1)
    return np.cumsum(off), dst[order]


def test_full_size_workload_properties(gpu_lib):
    """chunglu-1m-500k-20m at k = 10,000 (the benchmark's k-wing workload)."""
    k = 10_000
    g = gg.workload("chunglu-1m-500k-20m")
    mask, cnt, w, r = gpu_wing(gpu_lib, g, k)
    assert 0 < w < g.m and r > 1 and w == int(mask.sum())
    # every edge of the k-wing is in at least k of its butterflies; no count outside it
    assert (cnt[mask] >= k).all() and not cnt[~mask].any()
    we = g.edges[mask]
    wing = gg.Graph(np.ascontiguousarray(we), g.n_upper, g.n_lower, "wing")
    du = np.bincount(we[:, 0], minlength=g.n_upper).astype(np.int64)
    dl = np.bincount(we[:, 1], minlength=g.n_lower).astype(np.int64)
    # cost of one Eq. 8 evaluation on the wing: the upper degrees summed over N(v)
    reach = np.bincount(we[:, 1], weights=du[we[:, 0]], minlength=g.n_lower)
    rng = np.random.default_rng(12)
    idx = np.flatnonzero(mask)
    cheap = idx[reach[g.edges[idx, 1]] <= 2_000_000]
    sample = rng.choice(cheap, size=min(150, len(cheap)), replace=False)
    with oracle.Single(wing) as one:
        for i in sample:
            u, v = (int(x) for x in g.edges[i])
            assert one.edge(u, v) == cnt[i], (i, u, v)
    # maximality of the k-wing: an edge outside it, added back alone, lies in
    # fewer than k butterflies of the wing plus itself (else the union would
    # be a larger subgraph with every edge at k or more)
    uoff, unbr = _csr(we[:, 0], we[:, 1], g.n_upper)
    loff, lnbr = _csr(we[:, 1], we[:, 0], g.n_lower)
    out = np.flatnonzero(~mask)
    e_out = g.edges[out]
    cost = dl[e_out[:, 1]] * np.maximum(du[e_out[:, 0]], 1)
    pick = rng.choice(out[cost <= 400_000], size=150, replace=False)
    for i in pick:
        u, v = (int(x) for x in g.edges[i])
        nu = unbr[uoff[u]:uoff[u + 1]]
        c = 0
        for u2 in lnbr[loff[v]:loff[v + 1]]:
            c += np.intersect1d(nu, unbr[uoff[u2]:uoff[u2 + 1]], assume_unique=True).size
        assert c < k, (i, u, v, c)
