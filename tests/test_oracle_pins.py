"""Pins of the CPU oracle against facts it does not compute itself.

Every check here is independent of ``oracle.c``: brute-force enumeration of
2x2 bicliques written in plain Python (Def. 2), closed forms for complete
bipartite graphs, graphs with no butterflies, the values the paper prints for
its worked examples (``tests/golden/paper_examples.json``), the sum rules that
follow from Lemma 1 and Eq. 8, and the closed form of the number of wedges
Algorithm 2 processes.  A dropped term, a wrong sign, an off-by-one in an
index or a swapped layer in the oracle fails at least one of them.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import graphgen as gg
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def brute(g):
    """Def. 2 by enumeration: every {u,w} in U and {v,x} in L with all four edges."""
    adj = set(map(tuple, g.edges.tolist()))
    eidx = {e: i for i, e in enumerate(map(tuple, g.edges.tolist()))}
    tot = 0
    bu = [0] * g.n_upper
    bl = [0] * g.n_lower
    be = [0] * g.m
    for u, w in itertools.combinations(range(g.n_upper), 2):
        for v, x in itertools.combinations(range(g.n_lower), 2):
            if (u, v) in adj and (u, x) in adj and (w, v) in adj and (w, x) in adj:
                tot += 1
                for a in (u, w):
                    bu[a] += 1
                for b in (v, x):
                    bl[b] += 1
                for e in ((u, v), (u, x), (w, v), (w, x)):
                    be[eidx[e]] += 1
    return tot, np.array(bu, np.int64), np.array(bl, np.int64), np.array(be, np.int64)


def tiny_graphs(count, seed0=100):
    rng = np.random.default_rng(seed0)
    for i in range(count):
        nu = int(rng.integers(1, 9))
        nl = int(rng.integers(1, 9))
        p = float(rng.choice([0.2, 0.4, 0.6, 0.8, 1.0]))
        yield gg.random_small(seed0 + i, nu, nl, p)


@pytest.mark.parametrize("chunk", range(4))
def test_oracle_equals_brute_force(chunk):
    for g in tiny_graphs(150, seed0=1000 + 150 * chunk):
        tot, bu, bl, be = brute(g)
        assert oracle.total(g) == tot
        assert oracle.total(g, side=0) == tot
        assert oracle.total(g, side=1) == tot
        up, lo = oracle.vertex_counts(g)
        np.testing.assert_array_equal(up, bu)
        np.testing.assert_array_equal(lo, bl)
        np.testing.assert_array_equal(oracle.edge_counts(g, side=0), be)
        np.testing.assert_array_equal(oracle.edge_counts(g, side=1), be)


def test_single_queries_equal_brute_force():
    for g in tiny_graphs(60, seed0=7000):
        tot, bu, bl, be = brute(g)
        with oracle.Single(g) as s:
            for u in range(g.n_upper):
                assert s.vertex(0, u) == bu[u]
            for v in range(g.n_lower):
                assert s.vertex(1, v) == bl[v]
            for i, (u, v) in enumerate(g.edges.tolist()):
                assert s.edge(u, v) == be[i]


def test_vertex_subset_equals_brute_force():
    """Eq. 1 for a listed subset of one layer (the walk the CPU baseline
    times): every listed vertex, in any order, repeated or not, gets the
    brute-force B_x of Def. 2, and an out-of-range id is refused."""
    rng = np.random.default_rng(4242)
    for g in tiny_graphs(120, seed0=9100):
        _, bu, bl, _ = brute(g)
        for side, ref in ((0, bu), (1, bl)):
            n = len(ref)
            k = int(rng.integers(1, 2 * n + 1))
            xs = rng.integers(0, n, size=k)  # with repeats, unsorted
            np.testing.assert_array_equal(oracle.vertex_counts_subset(g, side, xs, 1), ref[xs])
            np.testing.assert_array_equal(oracle.vertex_counts_subset(g, side, xs[::-1], 3), ref[xs[::-1]])
            assert len(oracle.vertex_counts_subset(g, side, np.zeros(0, np.int64))) == 0
            with pytest.raises(RuntimeError):
                oracle.vertex_counts_subset(g, side, np.array([n]))


@pytest.mark.parametrize("a,b", [(3, 7), (40, 25)])
def test_vertex_subset_complete_bipartite(a, b):
    g = gg.complete_bipartite(a, b)
    c2 = lambda k: k * (k - 1) // 2
    assert (oracle.vertex_counts_subset(g, 0, np.arange(a)[::-1]) == (a - 1) * c2(b)).all()
    assert (oracle.vertex_counts_subset(g, 1, np.arange(b)) == (b - 1) * c2(a)).all()


@pytest.mark.parametrize("a,b", [(1, 1), (1, 5), (2, 2), (2, 3), (3, 7), (6, 6), (13, 4), (40, 25)])
def test_complete_bipartite_closed_form(a, b):
    g = gg.complete_bipartite(a, b)
    c2 = lambda k: k * (k - 1) // 2
    assert oracle.total(g) == c2(a) * c2(b)
    up, lo = oracle.vertex_counts(g)
    assert (up == (a - 1) * c2(b)).all()
    assert (lo == (b - 1) * c2(a)).all()
    assert (oracle.edge_counts(g) == (a - 1) * (b - 1)).all()


@pytest.mark.parametrize("k", [2, 3, 4, 7, 50])
def test_even_cycles(k):
    g = gg.even_cycle(k)
    expect = 1 if k == 2 else 0  # C4 is one butterfly; longer even cycles hold none
    assert oracle.total(g) == expect
    up, lo = oracle.vertex_counts(g)
    assert up.sum() == 2 * expect and lo.sum() == 2 * expect


@pytest.mark.parametrize("seed", range(5))
def test_forests_have_no_butterflies(seed):
    g = gg.random_forest(seed, 300, 200)
    assert oracle.total(g) == 0
    up, lo = oracle.vertex_counts(g)
    assert not up.any() and not lo.any()
    assert not oracle.edge_counts(g).any()


def _golden():
    with open(os.path.join(GOLDEN, "paper_examples.json")) as f:
        return json.load(f)


def test_paper_fig3_example1():
    gold = _golden()["paper_fig3"]
    g = gg.paper_fig3()
    nL = g.n_lower
    gid_u = lambda i: nL + i
    # the graph is the paper's: a layer-based start from U processes 1,000,000 wedges
    dl = np.bincount(g.edges[:, 1], minlength=g.n_lower)
    assert int((dl * (dl - 1) // 2).sum()) == gold["ibs_wedges"]["value"]
    assert oracle.vp_wedges(g) == gold["vp_wedges"]["value"]
    assert oracle.total(g) == gold["total"]["value"]
    # Example 1's priority order
    p = oracle.priorities(g)
    order = np.argsort(-p)
    assert list(order[:4]) == [gid_u(1), gid_u(0), 1001, 1000]
    assert order[4] == gid_u(1001) and order[-1] == 0 and order[-2] == 1
    # Example 1's count_wedge maps
    assert oracle.vp_count_wedge(g, gid_u(1)) == {gid_u(0): gold["count_wedge_u1_u0"]["value"]}
    assert oracle.vp_count_wedge(g, 1001) == {1000: gold["count_wedge_v1001_v1000"]["value"]}
    assert oracle.vp_count_wedge(g, gid_u(0)) == {}
    # per-vertex and per-edge values that follow from the structure
    up, lo = oracle.vertex_counts(g)
    assert up[0] == up[1] == 499500 and lo[1000] == lo[1001] == 499500
    assert (up[2:] == 999).all() and (lo[:1000] == 999).all()
    assert (oracle.edge_counts(g) == 999).all()


def test_paper_fig2a():
    gold = _golden()["paper_fig2a"]
    g = gg.paper_fig2a()
    for col, n in ((0, g.n_upper), (1, g.n_lower)):
        d = np.bincount(g.edges[:, col], minlength=n)
        assert int((d * (d - 1) // 2).sum()) == gold["layer_wedges"]["value"]
    assert oracle.vp_wedges(g) == gold["vp_wedges"]["value"]
    assert oracle.total(g) == gold["total"]["value"]


def _wedge_closed_form(g):
    """|W| of Algorithm 2 counted per middle vertex x.  Let h_x be the number
    of neighbours of x with higher priority than x.  The j-th highest of them
    (as a start) reaches every neighbour of x below it, d_x - j ends, so x is
    the middle of sum_{j=1..h_x} (d_x - j) = h_x (d_x - 1) - h_x (h_x - 1) / 2
    processed wedges (derived from Algorithm 2 and Def. 3)."""
    nL = g.n_lower
    du = np.bincount(g.edges[:, 0], minlength=g.n_upper).astype(np.int64)
    dl = np.bincount(g.edges[:, 1], minlength=g.n_lower).astype(np.int64)
    deg = np.concatenate([dl, du])
    gid = np.arange(nL + g.n_upper, dtype=np.int64)
    # priority by (degree, id), computed here with numpy's lexsort
    rank = np.empty_like(gid)
    rank[np.lexsort((gid, deg))] = gid
    a = g.edges[:, 0].astype(np.int64) + nL
    b = g.edges[:, 1].astype(np.int64)
    h = np.zeros_like(deg)
    np.add.at(h, b, (rank[a] > rank[b]).astype(np.int64))
    np.add.at(h, a, (rank[b] > rank[a]).astype(np.int64))
    return int((h * (deg - 1) - h * (h - 1) // 2).sum()), rank


@pytest.mark.parametrize("seed", range(40))
def test_vp_wedges_closed_form_and_bounds(seed):
    rng = np.random.default_rng(seed)
    g = gg.random_small(seed, int(rng.integers(2, 40)), int(rng.integers(2, 40)), float(rng.uniform(0.05, 0.7)))
    w, rank = _wedge_closed_form(g)
    assert oracle.vp_wedges(g) == w
    np.testing.assert_array_equal(oracle.priorities(g), rank)
    du = np.bincount(g.edges[:, 0], minlength=g.n_upper).astype(np.int64)
    dl = np.bincount(g.edges[:, 1], minlength=g.n_lower).astype(np.int64)
    mins = np.minimum(du[g.edges[:, 0]], dl[g.edges[:, 1]])
    # Thm 2 / Lemma 2: |W| <= sum_e min deg <= min(sum_U d^2, sum_L d^2)
    assert w <= int((mins - 1).sum()) <= int(mins.sum()) <= min(int((du ** 2).sum()), int((dl ** 2).sum()))
    # per-start counts add up
    tot, per = oracle.vp_wedges(g, per_start=True)
    assert tot == w == int(per.sum())


@pytest.mark.parametrize("seed", range(30))
def test_vpp_wedges_lemma3_and_enumeration(seed):
    """Algorithm 3's wedges: the end outranks start and middle.  Per middle x
    they are the pairs of neighbours u < w with w above x, the same
    h_x (d_x - 1) - h_x (h_x - 1) / 2 as Algorithm 2 (Lemma 3); per start they
    are enumerated here from the numpy ranks."""
    rng = np.random.default_rng(100 + seed)
    g = gg.random_small(100 + seed, int(rng.integers(2, 25)), int(rng.integers(2, 25)), float(rng.uniform(0.1, 0.8)))
    w, rank = _wedge_closed_form(g)
    tot, per = oracle.vpp_wedges(g, per_start=True)
    assert tot == w == oracle.vp_wedges(g) == int(per.sum())
    nL = g.n_lower
    nb = {}
    for u, v in g.edges.tolist():
        nb.setdefault(nL + u, []).append(v)
        nb.setdefault(v, []).append(nL + u)
    want = np.zeros(nL + g.n_upper, np.int64)
    for x, mids in nb.items():
        for v in mids:
            for y in nb[v]:
                if rank[y] > rank[x] and rank[y] > rank[v]:
                    want[x] += 1
    np.testing.assert_array_equal(per, want)


@pytest.mark.parametrize("seed", range(6))
def test_sum_rules_and_invariances(seed):
    g = gg.random_small(500 + seed, 30, 45, 0.3)
    tot = oracle.total(g)
    up, lo = oracle.vertex_counts(g)
    be = oracle.edge_counts(g)
    # Lemma 1 Eq. 2 and its per-edge analogue: each butterfly has 2 vertices per layer and 4 edges
    assert up.sum() == lo.sum() == 2 * tot
    assert be.sum() == 4 * tot
    # each butterfly through x uses exactly two edges at x
    su = np.zeros(g.n_upper, np.int64)
    sl = np.zeros(g.n_lower, np.int64)
    np.add.at(su, g.edges[:, 0], be)
    np.add.at(sl, g.edges[:, 1], be)
    np.testing.assert_array_equal(2 * up, su)
    np.testing.assert_array_equal(2 * lo, sl)
    # swapping the layers swaps the per-vertex outputs
    sw = gg.Graph(np.ascontiguousarray(g.edges[:, ::-1]), g.n_lower, g.n_upper)
    assert oracle.total(sw) == tot
    up2, lo2 = oracle.vertex_counts(sw)
    np.testing.assert_array_equal(up2, lo)
    np.testing.assert_array_equal(lo2, up)
    np.testing.assert_array_equal(oracle.edge_counts(sw), be)
    # relabelling vertices and reordering edges permutes the outputs
    rng = np.random.default_rng(seed)
    pu = rng.permutation(g.n_upper)
    pl = rng.permutation(g.n_lower)
    pe = rng.permutation(g.m)
    e2 = np.stack([pu[g.edges[pe, 0]], pl[g.edges[pe, 1]]], axis=1).astype(np.int32)
    g2 = gg.Graph(np.ascontiguousarray(e2), g.n_upper, g.n_lower)
    up3, lo3 = oracle.vertex_counts(g2)
    np.testing.assert_array_equal(up3[pu], up)
    np.testing.assert_array_equal(lo3[pl], lo)
    np.testing.assert_array_equal(oracle.edge_counts(g2), be[pe])
    # disjoint union adds
    e3 = np.concatenate([g.edges, g2.edges + np.array([g.n_upper, g.n_lower], np.int32)])
    g3 = gg.Graph(np.ascontiguousarray(e3), 2 * g.n_upper, 2 * g.n_lower)
    assert oracle.total(g3) == 2 * tot


def test_isolated_vertices_and_empty_graph():
    g = gg.random_small(9, 10, 12, 0.5)
    big = gg.Graph(g.edges.copy(), g.n_upper + 50, g.n_lower + 70)
    assert oracle.total(big) == oracle.total(g)
    empty = gg.Graph(np.zeros((0, 2), np.int32), 5, 3)
    assert oracle.total(empty) == 0
    assert oracle.vp_wedges(empty) == 0
    assert oracle.edge_counts(empty).shape == (0,)
    up, lo = oracle.vertex_counts(empty)
    assert not up.any() and not lo.any()


def test_uniform_workload_small_is_pinned_by_brute_force_on_subgraph():
    """The smallest benchmark workload, cut to a subgraph brute force can enumerate."""
    g = gg.workload("uniform-2k-3k-20k")
    e = g.edges[(g.edges[:, 0] < 60) & (g.edges[:, 1] < 400)]
    sub = gg.Graph(np.ascontiguousarray(e), 60, 400)
    assert oracle.total(sub) == brute(sub)[0]


def test_generator_determinism_and_shape():
    a = gg.workload("uniform-2k-3k-20k")
    b = gg.workload("uniform-2k-3k-20k")
    assert a.sha256() == b.sha256()
    keys = a.edges[:, 0].astype(np.int64) * a.n_lower + a.edges[:, 1]
    assert len(np.unique(keys)) == a.m == 20000
    assert a.edges[:, 0].max() < 2000 and a.edges[:, 1].max() < 3000 and a.edges.min() >= 0
    c = gg.chung_lu(11, 3000, 2000, 30000, 2.1, 2.1, 500.0, blocks=2, block=20, density=0.9)
    keys = c.edges[:, 0].astype(np.int64) * c.n_lower + c.edges[:, 1]
    assert len(np.unique(keys)) == c.m == 30000


def brute_three_paths(g):
    """Three-paths by enumeration: walks x-y-z-t over four distinct vertices,
    each path counted once (a walk and its reverse are the same path)."""
    nb = {}
    for u, v in g.edges.tolist():
        a, b = ("U", u), ("L", v)
        nb.setdefault(a, set()).add(b)
        nb.setdefault(b, set()).add(a)
    walks = 0
    for x in nb:
        for y in nb[x]:
            for z in nb[y]:
                if z == x:
                    continue
                for t in nb[z]:
                    if t != y and t != x:
                        walks += 1
    assert walks % 2 == 0
    return walks // 2


def test_caterpillars_equal_three_path_enumeration():
    for g in tiny_graphs(200, seed0=9100):
        assert oracle.caterpillars(g) == brute_three_paths(g)


@pytest.mark.parametrize("a,b", [(1, 1), (1, 5), (2, 2), (2, 3), (3, 7), (13, 4)])
def test_caterpillars_complete_bipartite(a, b):
    # every edge of K_{a,b} is the middle of (a - 1)(b - 1) three-paths
    g = gg.complete_bipartite(a, b)
    assert oracle.caterpillars(g) == a * b * (a - 1) * (b - 1)
    if a >= 2 and b >= 2:
        # 4 C(a,2) C(b,2) = a b (a - 1)(b - 1): complete bipartite graphs have coefficient 1
        assert oracle.clustering_coefficient(g) == 1.0


@pytest.mark.parametrize("k", [2, 3, 5])
def test_caterpillars_even_cycles_and_forests(k):
    # in C_{2k} every edge's ends have degree 2: one three-path per edge
    assert oracle.caterpillars(gg.even_cycle(k)) == 2 * k
    g = gg.random_forest(k, 200, 150)
    assert oracle.clustering_coefficient(g) == 0.0


# ---------------------------------------------------------------- k-wing

def brute_k_wing(g, k):
    """The k-wing by its definition (Section 1): the largest edge subset in which
    every edge lies in at least k butterflies of the subset.  Subsets with that
    property are closed under union (counts only grow with more edges), so the
    k-wing is the union of all of them; enumerated over every subset."""
    m = g.m
    edges = list(map(tuple, g.edges.tolist()))
    idx = {e: i for i, e in enumerate(edges)}
    flies = []
    for u, w in itertools.combinations(range(g.n_upper), 2):
        for v, x in itertools.combinations(range(g.n_lower), 2):
            four = [(u, v), (u, x), (w, v), (w, x)]
            if all(e in idx for e in four):
                flies.append([idx[e] for e in four])
    union = 0
    for s in range(1 << m):
        c = [0] * m
        for f in flies:
            if all(s >> i & 1 for i in f):
                for i in f:
                    c[i] += 1
        if all(c[i] >= k for i in range(m) if s >> i & 1):
            union |= s
    mask = np.array([bool(union >> i & 1) for i in range(m)])
    cnt = np.zeros(m, np.int64)
    for f in flies:
        if all(mask[i] for i in f):
            for i in f:
                cnt[i] += 1
    return mask, cnt


def small_wing_graphs(count, seed0):
    rng = np.random.default_rng(seed0)
    made = 0
    i = 0
    while made < count:
        i += 1
        g = gg.random_small(seed0 + i, int(rng.integers(2, 5)), int(rng.integers(2, 6)),
                            float(rng.choice([0.5, 0.7, 0.9, 1.0])))
        if 0 < g.m <= 13:
            made += 1
            yield g


def test_k_wing_equals_definition_by_enumeration():
    for g in small_wing_graphs(60, 7300):
        top = int(oracle.edge_counts(g).max()) if g.m else 0
        for k in range(0, top + 2):
            mask, cnt = brute_k_wing(g, k)
            o_mask, o_cnt, removed = oracle.k_wing(g, k)
            np.testing.assert_array_equal(o_mask, mask)
            np.testing.assert_array_equal(o_cnt, cnt)
            assert removed == g.m - int(mask.sum())


def _disjoint_union(parts):
    es, ou, ol = [], 0, 0
    for g in parts:
        es.append(g.edges + np.array([ou, ol], np.int32))
        ou += g.n_upper
        ol += g.n_lower
    return gg.Graph(np.ascontiguousarray(np.concatenate(es)), ou, ol, "union")


def test_k_wing_bicliques_and_pendants():
    # K_{3,3}: 4 butterflies per edge; K_{4,5}: 12; a path hanging off K_{4,5}
    # and a tree lie in none
    k33, k45 = gg.complete_bipartite(3, 3), gg.complete_bipartite(4, 5)
    tree = gg.random_forest(3, 30, 20)
    g = _disjoint_union([k33, k45, tree])
    # a two-edge path from K_{4,5}'s first upper vertex through a new lower
    # vertex to a new upper vertex
    extra = np.array([[k33.n_upper, g.n_lower], [g.n_upper, g.n_lower]], np.int32)
    g = gg.Graph(np.ascontiguousarray(np.concatenate([g.edges, extra])), g.n_upper + 1, g.n_lower + 1, "g")
    n33, n45 = k33.m, k45.m
    for k, keep33, keep45 in [(1, True, True), (4, True, True), (5, False, True), (12, False, True),
                              (13, False, False)]:
        mask, cnt, removed = oracle.k_wing(g, k)
        assert mask[:n33].all() == keep33 and (not mask[:n33].any()) == (not keep33)
        assert mask[n33:n33 + n45].all() == keep45 and (not mask[n33:n33 + n45].any()) == (not keep45)
        assert not mask[n33 + n45:].any()
        assert (cnt[:n33] == (4 if keep33 else 0)).all() and (cnt[n33:n33 + n45] == (12 if keep45 else 0)).all()
        assert removed == g.m - int(mask.sum())
    mask, cnt, removed = oracle.k_wing(g, 0)
    assert mask.all() and removed == 0
    np.testing.assert_array_equal(cnt, oracle.edge_counts(g))


@pytest.mark.parametrize("k", [1, 2, 3])
def test_k_wing_even_cycles_and_forests(k):
    # C_4 is one butterfly; longer even cycles and forests have none
    mask, cnt, _ = oracle.k_wing(gg.even_cycle(2), k)
    assert mask.all() == (k <= 1) and (cnt == (1 if k <= 1 else 0)).all()
    for g in (gg.even_cycle(5), gg.random_forest(k, 300, 200)):
        mask, cnt, removed = oracle.k_wing(g, k)
        assert not mask.any() and removed == g.m


@pytest.mark.parametrize("seed,k", [(41, 3), (42, 10), (43, 40)])
def test_k_wing_equals_batch_peeling_on_medium_graphs(seed, k):
    """Every edge below k in a graph containing the k-wing lies outside it, so
    removing all of them at once and recounting (Eq. 8) until none is below k
    reaches the same subgraph as removing them one at a time."""
    g = gg.chung_lu(seed, 1500, 1200, 12000, 2.1, 2.2, 300.0, blocks=2, block=12, density=0.8)
    keep = np.arange(g.m)
    while True:
        sub = gg.Graph(np.ascontiguousarray(g.edges[keep]), g.n_upper, g.n_lower, "sub")
        c = oracle.edge_counts(sub)
        if (c >= k).all():
            break
        keep = keep[c >= k]
    mask, cnt, removed = oracle.k_wing(g, k)
    want = np.zeros(g.m, bool)
    want[keep] = True
    np.testing.assert_array_equal(mask, want)
    full = np.zeros(g.m, np.int64)
    full[keep] = c
    np.testing.assert_array_equal(cnt, full)
    assert 0 < mask.sum() < g.m
