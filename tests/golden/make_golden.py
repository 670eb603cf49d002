"""Writes ``workloads.json``: oracle results for the benchmark workloads.

Run from the repository root:  ``python tests/golden/make_golden.py [names...]``

Calls only ``graphgen`` (the inputs) and ``oracle`` (the CPU definitions of
Lemma 1 and Eq. 8).  For each workload it stores the SHA-256 of the edge
list, the total, the number of wedges Algorithm 2 processes, SHA-256 digests
of the per-vertex and per-edge int64 arrays (little-endian), and a seeded
sample of individual values for readable failures.

With the single argument ``batch-4096`` it writes ``batch.json`` instead: each
graph's total and |W| for the 4,096-graph batch.

For the 200M-edge workload the lower layer's per-vertex counts are taken from
the per-edge counts by the identity 2 B_v = sum of B_e over the edges at v
(each butterfly through v uses two of its edges); a walk started from that
layer would cost the sum of squared upper degrees (about 1.3e12 steps).
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "workloads.json")
OUT_BATCH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch.json")
SAMPLES = 64


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i8").tobytes()).hexdigest()


def log(msg: str) -> None:
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def one(name: str) -> dict:
    g = gg.workload(name)
    log(f"{name}: generated m={g.m}")
    rec = {"edges_sha256": g.sha256(), "n_upper": g.n_upper, "n_lower": g.n_lower, "m": g.m}
    t = time.time()
    rec["vp_wedges"] = oracle.vp_wedges(g)
    log(f"  |W| = {rec['vp_wedges']} ({time.time() - t:.1f}s)")
    t = time.time()
    up = oracle.vertex_counts_side(g, 0)
    log(f"  vertex U ({time.time() - t:.1f}s)")
    t = time.time()
    be = oracle.edge_counts(g)
    log(f"  edges ({time.time() - t:.1f}s)")
    big = g.m > 50_000_000
    if big:
        sl = np.zeros(g.n_lower, np.int64)
        np.add.at(sl, g.edges[:, 1], be)
        assert not (sl & 1).any()
        lo = sl // 2
        rec["total"] = int(up.sum() // 2)
        rec["total_how"] = "half the upper layer's per-vertex sum (Eq. 2)"
        rec["lower_vertex_how"] = "half the per-edge sum at each lower vertex"
    else:
        t = time.time()
        lo = oracle.vertex_counts_side(g, 1)
        log(f"  vertex L ({time.time() - t:.1f}s)")
        t = time.time()
        rec["total"] = oracle.total(g)
        log(f"  total ({time.time() - t:.1f}s)")
        assert int(lo.sum()) == 2 * rec["total"]
    assert int(up.sum()) == 2 * rec["total"]
    assert int(be.sum()) == 4 * rec["total"]
    rec["vertex_upper_sha256"] = digest(up)
    rec["vertex_lower_sha256"] = digest(lo)
    rec["edge_sha256"] = digest(be)
    rng = np.random.default_rng(12345)
    iu = np.sort(rng.choice(g.n_upper, SAMPLES, replace=False))
    il = np.sort(rng.choice(g.n_lower, SAMPLES, replace=False))
    ie = np.sort(rng.choice(g.m, SAMPLES, replace=False))
    rec["sample_upper"] = {str(int(i)): int(up[i]) for i in iu}
    rec["sample_lower"] = {str(int(i)): int(lo[i]) for i in il}
    rec["sample_edges"] = {str(int(i)): int(be[i]) for i in ie}
    rec["max_vertex_upper"] = int(up.max()) if up.size else 0
    rec["max_edge"] = int(be.max()) if be.size else 0
    log(f"  total = {rec['total']}")
    return rec


def batch(name: str = "batch-4096") -> dict:
    """Per-graph totals and |W| of the 4,096-graph batch (seed 3), each graph
    counted on its own by the oracle (threads over graphs, one OpenMP thread each)."""
    from concurrent.futures import ThreadPoolExecutor

    b = gg.batch_workload()
    log(f"{name}: generated {b.count} graphs, {int(b.offsets[-1])} edges")
    graphs = [b.graph(i) for i in range(b.count)]
    order = sorted(range(b.count), key=lambda i: -graphs[i].m)
    totals = [0] * b.count
    wedges = [0] * b.count

    def one_graph(i):
        totals[i] = oracle.total(graphs[i], nthreads=1)
        wedges[i] = oracle.vp_wedges(graphs[i], nthreads=1)

    with ThreadPoolExecutor(max_workers=oracle.threads()) as ex:
        for k, _ in enumerate(ex.map(one_graph, order)):
            if k % 256 == 0:
                log(f"  {k}/{b.count} graphs")
    return {"sha256": b.sha256(), "graphs": b.count, "edges": int(b.offsets[-1]), "totals": totals,
            "vp_wedges": wedges}


def main(names: list[str]) -> None:
    if names == ["batch-4096"]:
        rec = batch("batch-4096")
        with open(OUT_BATCH, "w") as f:
            json.dump({"_about": "Oracle per-graph totals and |W| for the 4,096-graph batch, written by "
                                 "tests/golden/make_golden.py", "batch-4096": rec}, f)
            f.write("\n")
        return
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    data["_about"] = ("Oracle results (Lemma 1 Eq. 1/2, Eq. 8, and the wedge count of Algorithm 2) for the "
                      "seeded benchmark workloads, written by tests/golden/make_golden.py")
    for name in names or list(gg.WORKLOADS):
        data[name] = one(name)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
            f.write("\n")


if __name__ == "__main__":
    main(sys.argv[1:])
