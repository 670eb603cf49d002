"""Writes tests/golden/serve_10s.json: the oracle's answers for the served
workload's checked requests.

The served trace (graphgen.serve_schedule, seed 4, 200 requests/s) is
replayed for its first 10 s by ``bench.py --workload serve``.  Every request
whose graph has at most 1e6 edges is checked, plus a seeded 2% sample of the
larger ones.  The answer has the server's result form: the total for a
"total" request, else (sha256 of the int64 little-endian output arrays, their
sum) -- upper then lower per-vertex counts, or the per-edge counts in input
order.  Calls only graphgen/ and oracle/.

Usage: python tests/golden/make_serve_golden.py [threads]
"""
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

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "serve_10s.json")
DURATION_S = 10.0
SMALL_EDGES = 1_000_000
SAMPLE_FRACTION = 0.02
SAMPLE_SEED = 2024


def checked_requests(reqs):
    """Indices of the checked requests: graphs of at most SMALL_EDGES edges,
    plus a seeded SAMPLE_FRACTION of the others."""
    large = [r.index for r in reqs if r.graph.m > SMALL_EDGES]
    rng = np.random.default_rng(SAMPLE_SEED)
    k = int(round(SAMPLE_FRACTION * len(large)))
    sample = set(int(i) for i in rng.choice(large, size=k, replace=False)) if k else set()
    return sorted([r.index for r in reqs if r.graph.m <= SMALL_EDGES] + list(sample))


def answer(g, kind, threads):
    if kind == "total":
        return oracle.total(g, nthreads=threads)
    arrays = oracle.vertex_counts(g, threads) if kind == "vertex" else (oracle.edge_counts(g, nthreads=threads),)
    h = hashlib.sha256()
    s = 0
    for a in arrays:
        x = np.ascontiguousarray(a, dtype="<i8")
        h.update(x.tobytes())
        s += int(x.sum())
    return [h.hexdigest(), s]


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else None
    reqs = gg.serve_schedule(duration_s=DURATION_S)
    by_index = {r.index: r for r in reqs}
    want = checked_requests(reqs)
    # group by graph (follow-ups share their root's graph); big graphs last
    roots = {}
    for i in want:
        r = by_index[i]
        root = r.follow_up_of if r.follow_up_of >= 0 else r.index
        roots.setdefault(root, []).append(r)
    done = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            done = json.load(f).get("answers", {})
    t0 = time.time()
    order = sorted(roots, key=lambda k: by_index[k].graph.m)
    for n, root in enumerate(order):
        todo = [r for r in roots[root] if str(r.index) not in done]
        if not todo:
            continue
        g = gg.spec_graphs([by_index[root].graph], threads=1)[0]
        cache = {}
        for r in todo:
            if r.kind not in cache:
                cache[r.kind] = answer(g, r.kind, threads)
            done[str(r.index)] = cache[r.kind]
        if n % 50 == 0 or g.m > SMALL_EDGES:
            print(f"{n + 1}/{len(order)} graphs, m={g.m}, {time.time() - t0:.0f}s", flush=True)
            write(reqs, want, done)
    write(reqs, want, done)


def write(reqs, want, done):
    rec = {"trace": {"seed": gg.SERVE_SEED, "duration_s": DURATION_S, "requests": len(reqs),
                     "small_edges": SMALL_EDGES, "sample_fraction": SAMPLE_FRACTION, "sample_seed": SAMPLE_SEED,
                     "checked": len(want)},
           "answers": {k: done[k] for k in sorted(done, key=int)}}
    with open(OUT + ".tmp", "w") as f:
        json.dump(rec, f, separators=(",", ":"))
    os.replace(OUT + ".tmp", OUT)


if __name__ == "__main__":
    main()
