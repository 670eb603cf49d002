"""Writes ``caterpillars.json``: the oracle's caterpillar counts (three-paths,
the denominator of the bipartite clustering coefficient of Section 1) for
the benchmark workloads.

Run from the repository root:  ``python tests/golden/make_caterpillars.py``

Calls only ``graphgen`` (the inputs) and ``oracle`` (C_G = sum over edges
(u, v) of (d_u - 1)(d_v - 1)); stores each edge list's SHA-256 beside the
count so a changed generator is caught.
"""
from __future__ import annotations

import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "caterpillars.json")
NAMES = ["uniform-2k-3k-20k", "chunglu-1m-500k-20m", "chunglu-16m-4m-200m-planted"]


def main() -> None:
    out = {}
    for name in NAMES:
        g = gg.workload(name)
        out[name] = {"edges_sha256": g.sha256(), "caterpillars": oracle.caterpillars(g)}
        print(name, out[name], flush=True)
        del g
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
