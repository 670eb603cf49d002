"""Seeded synthetic bipartite graphs: the inputs shared by the oracle and the GPU path.

This module only produces edge lists.  It contains none of the butterfly
arithmetic; the CPU oracle (``oracle/``) and the HIP library both read its
output and neither depends on the other.

An edge list is an ``int32`` array of shape ``[m, 2]`` holding
``(upper, lower)`` pairs with ids that are 0-based per layer, the input form
of the counting problem (a bipartite graph G=(U, L, E) with E a subset of
U x L, Section 2 of the paper).

Random streams come from ``gen.c`` (SplitMix64 seeding, xoshiro256**,
Vose alias sampling, Fisher-Yates), single threaded, so every graph is a pure
function of its seed.
"""
from __future__ import annotations

import ctypes
import hashlib
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build_library() -> str:
    """Compiles ``gen.c`` into ``libgraphgen.so`` with gcc (host code only)."""
    cmd = ["gcc", "-O2", "-shared", "-fPIC", "-Wall", "-Wextra", "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build_library()
    lib = ctypes.CDLL(_LIB_PATH)
    i64, u64, f64 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    p32 = ctypes.POINTER(ctypes.c_int32)
    lib.gg_uniform.argtypes = [u64, i64, i64, i64, p32]
    lib.gg_uniform.restype = i64
    lib.gg_chung_lu.argtypes = [u64, i64, i64, i64, f64, f64, f64, i64, i64, f64, p32]
    lib.gg_chung_lu.restype = i64
    lib.gg_doubles.argtypes = [u64, i64, ctypes.POINTER(ctypes.c_double)]
    lib.gg_doubles.restype = None
    lib.gg_subseed.argtypes = [u64, u64]
    lib.gg_subseed.restype = u64
    _lib = lib
    return lib


@dataclass
class Graph:
    """A bipartite edge list: ``edges[i] = (upper id, lower id)``."""

    edges: np.ndarray  # int32 [m, 2], C-contiguous
    n_upper: int
    n_lower: int
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.edges.shape[0])

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.array([self.n_upper, self.n_lower, self.m], dtype=np.int64).tobytes())
        h.update(np.ascontiguousarray(self.edges, dtype=np.int32).tobytes())
        return h.hexdigest()


def _out(m: int) -> np.ndarray:
    return np.empty((m, 2), dtype=np.int32)


def uniform(seed: int, n_upper: int, n_lower: int, m: int, name: str = "") -> Graph:
    """m distinct (upper, lower) cells drawn uniformly without replacement."""
    out = _out(m)
    got = _load().gg_uniform(seed, n_upper, n_lower, m, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if got != m:
        raise ValueError(f"uniform generator failed ({got})")
    return Graph(out, n_upper, n_lower, name)


def chung_lu(seed: int, n_upper: int, n_lower: int, m: int, gamma_upper: float, gamma_lower: float,
             cap: float, blocks: int = 0, block: int = 0, density: float = 0.0, name: str = "") -> Graph:
    """Bipartite Chung-Lu graph with Pareto expected degrees and optional planted bicliques.

    Expected-degree weights are ``(1-q)^(-1/(gamma-1))`` for uniform q (a
    degree pdf with exponent gamma), scaled to sum to the number of sampled
    edges and capped at ``cap``.  Endpoints are drawn independently in
    proportion to the weights; repeats are dropped and the draw is topped up
    until exactly m distinct edges exist.  ``blocks`` bicliques of
    ``block x block`` vertices on disjoint random vertex sets are planted
    first, each cell kept with probability ``density``; they count toward m.
    """
    out = _out(m)
    got = _load().gg_chung_lu(seed, n_upper, n_lower, m, gamma_upper, gamma_lower, cap, blocks, block, density,
                              out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if got != m:
        raise ValueError(f"chung-lu generator failed ({got})")
    return Graph(out, n_upper, n_lower, name)


def doubles(seed: int, count: int) -> np.ndarray:
    """``count`` uniform doubles in [0, 1) from the xoshiro256** stream of ``seed``."""
    out = np.empty(count, dtype=np.float64)
    _load().gg_doubles(seed, count, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def subseed(seed: int, index: int) -> int:
    return int(_load().gg_subseed(seed, index))


# ---------------------------------------------------------------- workloads
# The five benchmark workloads.  Sizes and shapes follow the paper's
# experimental graphs (hubs in both layers, 1e7..1e9 edges); the real
# datasets are replaced by these seeded synthetic graphs.

WORKLOADS = {
    "uniform-2k-3k-20k": dict(seed=0, kind="uniform", n_upper=2000, n_lower=3000, m=20000),
    "chunglu-1m-500k-20m": dict(seed=1, kind="chung_lu", n_upper=1_000_000, n_lower=500_000, m=20_000_000,
                                gamma_upper=2.1, gamma_lower=2.1, cap=50_000.0),
    "chunglu-16m-4m-200m-planted": dict(seed=2, kind="chung_lu", n_upper=16_777_216, n_lower=4_194_304,
                                        m=200_000_000, gamma_upper=2.0, gamma_lower=2.3, cap=50_000.0,
                                        blocks=64, block=512, density=0.9),
}


def workload(name: str) -> Graph:
    spec = dict(WORKLOADS[name])
    seed = spec.pop("seed")
    kind = spec.pop("kind")
    if kind == "uniform":
        return uniform(seed, name=name, **spec)
    return chung_lu(seed, name=name, **spec)


# Batched workload: 4,096 independent graphs (seed 3).
BATCH_SEED = 3
BATCH_COUNT = 4096


@dataclass
class GraphSpec:
    index: int
    seed: int
    kind: str  # "uniform" | "chung_lu"
    n_upper: int
    n_lower: int
    m: int
    gamma: float


def _split_sides(n: int, ratio: float, m: int) -> tuple[int, int]:
    """Splits n vertices into |U|/|L| = ratio (at least 2 per side, enough cells for m edges)."""
    nu = max(2, int(round(n * ratio / (1.0 + ratio))))
    nl = max(2, n - nu)
    while nu * nl < m:  # tiny graphs: grow the smaller side until m cells exist
        if nu <= nl:
            nu += 1
        else:
            nl += 1
    return nu, nl


def batch_specs(seed: int = BATCH_SEED, count: int = BATCH_COUNT, m_lo: int = 1_000, m_hi: int = 1_000_000) -> list[GraphSpec]:
    """Per-graph parameters: m log-uniform in [m_lo, m_hi], |U|/|L| uniform in [0.25, 4],
    n = |U|+|L| = round(m/8), graphs alternating uniform / Chung-Lu (exponent 2.1)."""
    u = doubles(seed, 2 * count)
    specs = []
    for g in range(count):
        m = int(round(math.exp(math.log(m_lo) + u[2 * g] * (math.log(m_hi) - math.log(m_lo)))))
        ratio = 0.25 + u[2 * g + 1] * 3.75
        nu, nl = _split_sides(max(4, int(round(m / 8))), ratio, m)
        kind = "uniform" if g % 2 == 0 else "chung_lu"
        specs.append(GraphSpec(g, subseed(seed, g), kind, nu, nl, m, 2.1))
    return specs


def spec_graphs(specs: list[GraphSpec], threads: int = 16) -> list[Graph]:
    """Generates many graphs in parallel (each from its own seed, so the
    result does not depend on the thread count)."""
    from concurrent.futures import ThreadPoolExecutor

    _load()
    with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        return list(ex.map(spec_graph, specs))


@dataclass
class Batch:
    """Graphs laid out back to back: graph g owns edge rows [offsets[g], offsets[g+1])."""

    edges: np.ndarray        # int32 [sum m, 2]
    offsets: np.ndarray      # int64 [G+1]
    n_upper: np.ndarray      # int32 [G]
    n_lower: np.ndarray      # int32 [G]

    @property
    def count(self) -> int:
        return len(self.n_upper)

    def graph(self, g: int) -> Graph:
        e = self.edges[self.offsets[g]:self.offsets[g + 1]]
        return Graph(np.ascontiguousarray(e), int(self.n_upper[g]), int(self.n_lower[g]), f"g{g}")

    def sha256(self) -> str:
        h = hashlib.sha256()
        for a in (self.offsets, self.n_upper, self.n_lower, self.edges):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()


def concat(graphs: list[Graph]) -> Batch:
    offsets = np.zeros(len(graphs) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum([g.m for g in graphs])
    edges = np.empty((int(offsets[-1]), 2), dtype=np.int32)
    for i, g in enumerate(graphs):
        edges[offsets[i]:offsets[i + 1]] = g.edges
    return Batch(edges, offsets, np.array([g.n_upper for g in graphs], np.int32),
                 np.array([g.n_lower for g in graphs], np.int32))


def batch_workload(count: int = BATCH_COUNT, threads: int = 16) -> Batch:
    """The batched workload: ``count`` graphs from batch_specs (seed 3)."""
    return concat(spec_graphs(batch_specs(count=count), threads))


def spec_graph(s: GraphSpec) -> Graph:
    if s.kind == "uniform":
        return uniform(s.seed, s.n_upper, s.n_lower, s.m, name=f"g{s.index}")
    cap = float(min(50_000, s.n_upper, s.n_lower))
    return chung_lu(s.seed, s.n_upper, s.n_lower, s.m, s.gamma, s.gamma, cap, name=f"g{s.index}")


# Served workload (seed 4): Poisson arrivals, Chung-Lu requests.
SERVE_SEED = 4


@dataclass
class Request:
    index: int
    arrival_s: float
    kind: str  # "total" | "vertex" | "edge"
    graph: GraphSpec
    follow_up_of: int  # -1 for a new graph, else the index of an earlier request whose graph it reuses


def serve_schedule(seed: int = SERVE_SEED, rate: float = 200.0, duration_s: float = 60.0,
                   m_lo: int = 10_000, m_hi: int = 50_000_000, follow_up: float = 0.3,
                   max_requests: int | None = None) -> list[Request]:
    """Arrival trace: exponential inter-arrival times at ``rate``; request kind
    total/vertex/edge with probabilities 0.6/0.25/0.15; a fraction ``follow_up``
    of requests re-query the graph of a uniformly chosen earlier request;
    new graphs are Chung-Lu with exponent uniform in [2.0, 2.5] and m
    log-uniform in [m_lo, m_hi], n = round(m/8), |U|/|L| uniform in [0.25, 4]."""
    cap_req = int(rate * duration_s * 2 + 100)
    u = doubles(seed, 7 * cap_req)
    t = 0.0
    reqs: list[Request] = []
    for i in range(cap_req):
        r = u[7 * i: 7 * i + 7]
        t += -math.log(1.0 - r[0]) / rate
        if t > duration_s or (max_requests is not None and len(reqs) >= max_requests):
            break
        kind = "total" if r[1] < 0.6 else ("vertex" if r[1] < 0.85 else "edge")
        if reqs and r[2] < follow_up:
            j = min(int(r[3] * len(reqs)), len(reqs) - 1)
            base = reqs[j]
            root = base.follow_up_of if base.follow_up_of >= 0 else base.index
            reqs.append(Request(i, t, kind, reqs[root].graph, root))
            continue
        m = int(round(math.exp(math.log(m_lo) + r[4] * (math.log(m_hi) - math.log(m_lo)))))
        ratio = 0.25 + r[5] * 3.75
        gamma = 2.0 + r[6] * 0.5
        nu, nl = _split_sides(max(4, int(round(m / 8))), ratio, m)
        reqs.append(Request(i, t, kind, GraphSpec(i, subseed(seed, i), "chung_lu", nu, nl, m, gamma), -1))
    return reqs


# ------------------------------------------------------- structured graphs

def complete_bipartite(a: int, b: int) -> Graph:
    """K_{a,b}: every upper vertex joined to every lower vertex."""
    uu, ll = np.meshgrid(np.arange(a, dtype=np.int32), np.arange(b, dtype=np.int32), indexing="ij")
    return Graph(np.stack([uu.ravel(), ll.ravel()], axis=1).copy(), a, b, f"K{a},{b}")


def from_pairs(pairs, n_upper: int, n_lower: int, name: str = "") -> Graph:
    e = np.asarray(list(pairs), dtype=np.int32).reshape(-1, 2)
    return Graph(np.ascontiguousarray(e), n_upper, n_lower, name)


def paper_fig2a() -> Graph:
    """The graph of the paper's Fig. 2(a), as described in its introduction:
    u0 joined to v0..v999, v1000 joined to u1..u1000, and v_i joined to u_{i+1}
    for i = 0..999 (3,000 edges, |U| = 1,001, |L| = 1,001)."""
    pairs = [(0, i) for i in range(1000)]
    pairs += [(i, 1000) for i in range(1, 1001)]
    pairs += [(i + 1, i) for i in range(1000)]
    return from_pairs(pairs, 1001, 1001, "paper-fig2a")


def paper_fig3() -> Graph:
    """The hub graph of the paper's Fig. 3 (Example 1): u0 and u1 joined to
    v0..v999; v1000 and v1001 joined to u2..u1001 (4,000 edges,
    |U| = |L| = 1,002)."""
    pairs = [(u, v) for u in (0, 1) for v in range(1000)]
    pairs += [(u, v) for v in (1000, 1001) for u in range(2, 1002)]
    return from_pairs(pairs, 1002, 1002, "paper-fig3")


def even_cycle(k: int) -> Graph:
    """The cycle C_{2k} on u0 v0 u1 v1 ... (k upper and k lower vertices)."""
    pairs = [(i, i) for i in range(k)] + [((i + 1) % k, i) for i in range(k)]
    pairs = sorted(set(pairs))
    return from_pairs(pairs, k, k, f"C{2 * k}")


def random_forest(seed: int, n_upper: int, n_lower: int) -> Graph:
    """A random bipartite forest: each vertex after the first attaches to at most
    one earlier vertex of the other layer (no cycles, so no butterflies)."""
    rng = np.random.default_rng(seed)
    order = [(0, i) for i in range(n_upper)] + [(1, i) for i in range(n_lower)]
    rng.shuffle(order)
    seen = {0: [], 1: []}
    pairs = []
    for side, i in order:
        other = seen[1 - side]
        if other and rng.random() < 0.85:
            j = other[int(rng.integers(len(other)))]
            pairs.append((i, j) if side == 0 else (j, i))
        seen[side].append(i)
    return from_pairs(pairs, n_upper, n_lower, "forest")


def random_small(seed: int, n_upper: int, n_lower: int, p: float) -> Graph:
    """Erdos-Renyi style bipartite graph: each cell present with probability p."""
    rng = np.random.default_rng(seed)
    mask = rng.random((n_upper, n_lower)) < p
    uu, ll = np.nonzero(mask)
    e = np.stack([uu, ll], axis=1).astype(np.int32)
    e = e[rng.permutation(len(e))]
    return Graph(np.ascontiguousarray(e), n_upper, n_lower, f"er{seed}")
