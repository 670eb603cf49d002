"""CPU oracle for exact butterfly counts -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never calls it and
shares no code with it.

The arithmetic lives in ``oracle.c`` (plain C, OpenMP over start vertices):

* ``vertex_counts``  -- Lemma 1, Eq. 1: B_x = sum_{y in 2hop(x)} C(|N(x) & N(y)|, 2)
* ``total``          -- Lemma 1, Eq. 2: B_G = 1/2 sum_{x in one layer} B_x
* ``edge_counts``    -- Section 6.1, Eq. 8: B_(u,v) = sum_{w in N(v), w != u} (|N(u) & N(w)| - 1)
* ``vertex_one`` / ``edge_one`` -- the same two formulas for a single vertex or edge
* ``vp_wedges``      -- the number of wedges Algorithm 2 (BFC-VP) processes under
  the priority of Definition 3 (the denominator of the wedges/s metric)
* ``vpp_wedges``     -- the number of wedges Algorithm 3 (BFC-VP++) processes (the
  end outranks start and middle); equal to ``vp_wedges`` by Lemma 3
* ``vp_count_wedge`` -- Algorithm 2's count_wedge map for one start vertex
* ``priorities``     -- Definition 3's priority as a rank in [0, n)
* ``caterpillars``   -- Section 1: the three-paths C_G, sum over edges (u, v) of
  (d_u - 1)(d_v - 1), the denominator of the clustering coefficient 4 B_G / C_G
* ``k_wing``         -- Section 1: the k-wing, the largest subgraph whose every edge
  lies in at least k butterflies, by the peeling the paper describes (remove the
  edge with the fewest butterflies while below k, updating the others' counts)

Vertices carry the global ids of Section 2: lower v -> v, upper u -> |L| + u.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build_library() -> str:
    """Compiles ``oracle.c`` with gcc + OpenMP into ``liboracle.so``."""
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-Wall", "-Wextra", "-o", _LIB_PATH + ".tmp", _SRC]
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
    i64, i32, vp = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
    lib.orc_vertex_counts.argtypes = [vp, i64, i64, i64, i32, vp, i32]
    lib.orc_vertex_counts.restype = i32
    lib.orc_total.argtypes = [vp, i64, i64, i64, i32, i32, vp, vp]
    lib.orc_total.restype = i32
    lib.orc_edge_counts.argtypes = [vp, i64, i64, i64, i32, i32, vp]
    lib.orc_edge_counts.restype = i32
    lib.orc_vertex_counts_subset.argtypes = [vp, i64, i64, i64, i32, vp, i64, vp, i32]
    lib.orc_vertex_counts_subset.restype = i32
    lib.orc_open.argtypes = [vp, i64, i64, i64, vp]
    lib.orc_open.restype = vp
    lib.orc_close.argtypes = [vp]
    lib.orc_close.restype = None
    lib.orc_vertex_one.argtypes = [vp, i32, i64]
    lib.orc_vertex_one.restype = i64
    lib.orc_edge_one.argtypes = [vp, i64, i64]
    lib.orc_edge_one.restype = i64
    lib.orc_priorities.argtypes = [vp, i64, i64, i64, vp]
    lib.orc_priorities.restype = i32
    lib.orc_vp_wedges.argtypes = [vp, i64, i64, i64, i32, vp, vp]
    lib.orc_vp_wedges.restype = i32
    lib.orc_vpp_wedges.argtypes = [vp, i64, i64, i64, i32, vp, vp]
    lib.orc_vpp_wedges.restype = i32
    lib.orc_vp_count_wedge.argtypes = [vp, i64, i64, i64, i64, vp, vp, i64]
    lib.orc_vp_count_wedge.restype = i64
    lib.orc_caterpillars.argtypes = [vp, i64, i64, i64, vp]
    lib.orc_caterpillars.restype = i32
    lib.orc_k_wing.argtypes = [vp, i64, i64, i64, i64, i32, vp, vp, vp]
    lib.orc_k_wing.restype = i32
    lib.orc_max_threads.argtypes = []
    lib.orc_max_threads.restype = i32
    _lib = lib
    return lib


class OracleError(RuntimeError):
    pass


def _edges(g):
    e = np.ascontiguousarray(g.edges, dtype=np.int32).reshape(-1, 2)
    return e, e.ctypes.data if e.size else None


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise OracleError(f"{what} failed with code {rc}")


def threads(n: int | None = None) -> int:
    return int(n) if n else int(_load().orc_max_threads())


def total(g, side: int = -1, nthreads: int | None = None) -> int:
    """B_G (Eq. 2) from the layer picked by the sum-of-squared-degrees rule, or ``side``."""
    e, p = _edges(g)
    out = ctypes.c_int64(0)
    used = ctypes.c_int(0)
    _check(_load().orc_total(p, e.shape[0], g.n_upper, g.n_lower, side, threads(nthreads),
                             ctypes.addressof(out), ctypes.addressof(used)), "total")
    return int(out.value)


def vertex_counts(g, nthreads: int | None = None) -> tuple[np.ndarray, np.ndarray]:
    """(B_u for u in U, B_v for v in L), Eq. 1, each layer from its own walk."""
    e, p = _edges(g)
    up = np.zeros(g.n_upper, dtype=np.int64)
    lo = np.zeros(g.n_lower, dtype=np.int64)
    lib = _load()
    _check(lib.orc_vertex_counts(p, e.shape[0], g.n_upper, g.n_lower, 0, up.ctypes.data, threads(nthreads)), "vertex U")
    _check(lib.orc_vertex_counts(p, e.shape[0], g.n_upper, g.n_lower, 1, lo.ctypes.data, threads(nthreads)), "vertex L")
    return up, lo


def vertex_counts_side(g, side: int, nthreads: int | None = None) -> np.ndarray:
    e, p = _edges(g)
    out = np.zeros(g.n_upper if side == 0 else g.n_lower, dtype=np.int64)
    _check(_load().orc_vertex_counts(p, e.shape[0], g.n_upper, g.n_lower, side, out.ctypes.data, threads(nthreads)),
           "vertex")
    return out


def vertex_counts_subset(g, side: int, xs, nthreads: int | None = None) -> np.ndarray:
    """Eq. 1 for the listed vertices of one layer only."""
    e, p = _edges(g)
    xs = np.ascontiguousarray(xs, dtype=np.int64)
    out = np.zeros(len(xs), dtype=np.int64)
    _check(_load().orc_vertex_counts_subset(p, e.shape[0], g.n_upper, g.n_lower, side, xs.ctypes.data, len(xs),
                                            out.ctypes.data, threads(nthreads)), "vertex subset")
    return out


def cheaper_side(g) -> int:
    """The start layer of the sum-of-squared-degrees rule (0 upper, 1 lower)."""
    du = np.bincount(g.edges[:, 0], minlength=g.n_upper).astype(np.int64)
    dl = np.bincount(g.edges[:, 1], minlength=g.n_lower).astype(np.int64)
    return 1 if int((du * du).sum()) < int((dl * dl).sum()) else 0


def edge_counts(g, side: int = -1, nthreads: int | None = None) -> np.ndarray:
    """B_e for every edge in input order (Eq. 8)."""
    e, p = _edges(g)
    out = np.zeros(e.shape[0], dtype=np.int64)
    _check(_load().orc_edge_counts(p, e.shape[0], g.n_upper, g.n_lower, side, threads(nthreads), out.ctypes.data),
           "edge")
    return out


class Single:
    """Repeated single-vertex (Eq. 1) and single-edge (Eq. 8) queries on one graph."""

    def __init__(self, g):
        self._e, p = _edges(g)
        rc = ctypes.c_int(0)
        self._h = _load().orc_open(p, self._e.shape[0], g.n_upper, g.n_lower, ctypes.addressof(rc))
        _check(rc.value, "open")

    def vertex(self, side: int, x: int) -> int:
        r = _load().orc_vertex_one(self._h, side, x)
        if r < 0:
            raise OracleError(f"vertex_one failed with code {r}")
        return int(r)

    def edge(self, u: int, v: int) -> int:
        r = _load().orc_edge_one(self._h, u, v)
        if r < 0:
            raise OracleError(f"edge_one failed with code {r}")
        return int(r)

    def close(self):
        if self._h:
            _load().orc_close(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def priorities(g) -> np.ndarray:
    """Definition 3's priority of each global id as a rank in [0, n)."""
    e, p = _edges(g)
    out = np.zeros(g.n_upper + g.n_lower, dtype=np.int64)
    _check(_load().orc_priorities(p, e.shape[0], g.n_upper, g.n_lower, out.ctypes.data), "priorities")
    return out


def caterpillars(g) -> int:
    """C_G: three-paths, sum over edges (u, v) of (d_u - 1)(d_v - 1) (Section 1)."""
    e, p = _edges(g)
    out = ctypes.c_int64(0)
    _check(_load().orc_caterpillars(p, e.shape[0], g.n_upper, g.n_lower, ctypes.byref(out)), "caterpillars")
    return int(out.value)


def k_wing(g, k: int, nthreads: int | None = None) -> tuple[np.ndarray, np.ndarray, int]:
    """The k-wing of Section 1 by sequential peeling.

    Returns (in_wing bool [m], butterflies of each edge within the k-wing
    (0 outside it) int64 [m], number of edges removed)."""
    e, p = _edges(g)
    m = e.shape[0]
    mask = np.zeros(m, dtype=np.uint8)
    cnt = np.zeros(m, dtype=np.int64)
    removed = ctypes.c_int64(0)
    _check(_load().orc_k_wing(p, m, g.n_upper, g.n_lower, int(k), threads(nthreads),
                              mask.ctypes.data if m else None, cnt.ctypes.data if m else None,
                              ctypes.byref(removed)), "k_wing")
    return mask.astype(bool), cnt, int(removed.value)


def clustering_coefficient(g) -> float:
    """Bipartite clustering coefficient 4 B_G / C_G (Section 1); 0 without three-paths."""
    c = caterpillars(g)
    return 4.0 * total(g) / c if c else 0.0


def vp_wedges(g, per_start: bool = False, nthreads: int | None = None):
    """|W|: wedges processed by Algorithm 2; optionally per start (by global id)."""
    e, p = _edges(g)
    out = ctypes.c_int64(0)
    per = np.zeros(g.n_upper + g.n_lower, dtype=np.int64) if per_start else None
    _check(_load().orc_vp_wedges(p, e.shape[0], g.n_upper, g.n_lower, threads(nthreads), ctypes.addressof(out),
                                 per.ctypes.data if per is not None else None), "vp_wedges")
    return (int(out.value), per) if per_start else int(out.value)


def vpp_wedges(g, per_start: bool = False, nthreads: int | None = None):
    """Wedges Algorithm 3 (BFC-VP++) processes: end above both start and middle.
    With per_start, also each start's count by global id (lower v -> v, upper u -> |L| + u)."""
    e, p = _edges(g)
    out = ctypes.c_int64(0)
    per = np.zeros(g.n_upper + g.n_lower, dtype=np.int64) if per_start else None
    _check(_load().orc_vpp_wedges(p, e.shape[0], g.n_upper, g.n_lower, threads(nthreads), ctypes.byref(out),
                                  per.ctypes.data if per_start and per.size else None), "vpp_wedges")
    return (int(out.value), per) if per_start else int(out.value)


def vp_count_wedge(g, start_gid: int) -> dict[int, int]:
    """Algorithm 2's count_wedge map for one start, keyed by global id."""
    e, p = _edges(g)
    cap = g.n_upper + g.n_lower
    ends = np.zeros(max(cap, 1), dtype=np.int64)
    counts = np.zeros(max(cap, 1), dtype=np.int64)
    k = _load().orc_vp_count_wedge(p, e.shape[0], g.n_upper, g.n_lower, start_gid, ends.ctypes.data,
                                   counts.ctypes.data, cap)
    if k < 0:
        raise OracleError(f"vp_count_wedge failed with code {k}")
    return {int(a): int(b) for a, b in zip(ends[:k], counts[:k])}
