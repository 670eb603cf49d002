"""Autotuner: picks kernel settings by measuring counts on the GPU.

None of the settings changes a count (they choose which kernel path handles
each start and which wedges each layer's starts take, Algorithm 2's or
Algorithm 3's); the tuner only times them.  All counting runs in libbfc.

* ``pick_direction``: the per-layer wedge direction (``vpp`` mask) for one
  built graph, by timing one total count per mask.
* ``tune_batch``: per (size bucket, skew bucket) of a batch's graphs, the
  light / heavy cutoff, hash window size, dense-window ratio and window mode,
  by timing the count of a sample of that bucket's graphs; the result is a
  JSON-serialisable table that ``apply_table`` installs on a batch handle
  (``bfc_set_graph_tuning``: one setting per graph, used by the one set of
  counting launches).
"""
from __future__ import annotations

import json
import math
import time

import numpy as np
import torch

from . import bfc


def time_count(h: bfc.Graph, reps: int = 2, stream=None) -> float:
    """Milliseconds of the fastest of `reps` total counts (after one warm count)."""
    h.count_total(stream)
    best = float("inf")
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h.count_total(stream)
        best = min(best, time.perf_counter() - t0)
    return 1e3 * best


def pick_direction(h: bfc.Graph, masks=(0, 1, 2, 3), reps: int = 2) -> tuple[dict, dict]:
    """Times the total count with each per-layer direction mask on the built
    handle; leaves the handle on the fastest and returns ({"vpp": mask}, ms per mask)."""
    ms = {}
    for mk in masks:
        h.set_tuning(vpp=mk)
        ms[mk] = time_count(h, reps)
    best = min(ms, key=ms.get)
    h.set_tuning(vpp=best)
    return {"vpp": best}, ms


# ---------------------------------------------------------------- batches
# candidate settings searched per bucket (fields of bfc_set_tuning)
BATCH_CANDIDATES = {
    "light_max_wedges": (256, 1024, 2048),
    "hash_window_wedges": (2048, 8192, 32768),
    "dense_min_ratio": (2, 4, 8),
    "window_mode": (1, 3),
}


def bucket_of(m: int, max_deg: int, mean_deg: float) -> str:
    """(size bucket, skew bucket): log4 of the edge count, and whether the
    largest degree exceeds 16x the mean (skewed) or not."""
    size = int(math.floor(math.log(max(m, 1), 4)))
    skew = "skewed" if max_deg > 16.0 * max(mean_deg, 1.0) else "flat"
    return f"m4^{size}-{skew}"


def graph_buckets(edges: np.ndarray, offsets, n_upper, n_lower) -> list[str]:
    out = []
    for g in range(len(n_upper)):
        e = edges[offsets[g]:offsets[g + 1]]
        m = len(e)
        if m == 0:
            out.append("empty")
            continue
        du = np.bincount(e[:, 0], minlength=int(n_upper[g]))
        dl = np.bincount(e[:, 1], minlength=int(n_lower[g]))
        mx = int(max(du.max(), dl.max()))
        mean = 2.0 * m / max(int(n_upper[g]) + int(n_lower[g]), 1)
        out.append(bucket_of(m, mx, mean))
    return out


def tune_batch(edges: np.ndarray, offsets, n_upper, n_lower, sample_edges: int = 20_000_000,
               candidates: dict | None = None, seed: int = 0, log=None, min_gain: float = 0.03) -> dict:
    """Per bucket, the candidate setting with the fastest total count of a
    seeded sample of the bucket's graphs (one batch handle per sample).
    Coordinate search: one field at a time, in the order of `candidates`; a
    value replaces the setting kept so far only when it counts at least
    `min_gain` faster (timing noise does not install per-graph settings,
    which cost a schedule rebuild).  A bucket whose defaults win keeps an
    empty setting.  Returns {bucket: {"tuning": {field: value}, ...}}."""
    cand = candidates or BATCH_CANDIDATES
    offsets = np.asarray(offsets, dtype=np.int64)
    buckets = graph_buckets(edges, offsets, n_upper, n_lower)
    rng = np.random.default_rng(seed)
    table = {}
    for b in sorted(set(buckets)):
        if b == "empty":
            continue
        idx = [i for i, x in enumerate(buckets) if x == b]
        rng.shuffle(idx)
        pick, tot = [], 0
        for i in idx:
            m = int(offsets[i + 1] - offsets[i])
            if pick and tot + m > sample_edges:
                break
            pick.append(i)
            tot += m
        pick.sort()
        e = np.concatenate([edges[offsets[i]:offsets[i + 1]] for i in pick])
        off = np.zeros(len(pick) + 1, np.int64)
        off[1:] = np.cumsum([offsets[i + 1] - offsets[i] for i in pick])
        dev = torch.from_numpy(np.ascontiguousarray(e)).cuda()
        with bfc.build_batch(dev, off, [int(n_upper[i]) for i in pick], [int(n_lower[i]) for i in pick]) as h:
            defaults = h.get_tuning()
            best = {}
            base_ms = best_ms = time_count(h, reps=3)
            for field, values in cand.items():
                for v in values:
                    if v == best.get(field, defaults[field]):
                        continue
                    h.set_tuning(**{**defaults, **best, field: v})
                    ms = time_count(h, reps=3)
                    if ms < best_ms * (1.0 - min_gain):
                        best[field] = v
                        best_ms = ms
            h.set_tuning(**{**defaults, **best})
            tuned_ms = time_count(h, reps=3)
        # the saving scaled from the sample to the bucket's graphs
        saving = max(base_ms - tuned_ms, 0.0) * len(idx) / len(pick) if best else 0.0
        table[b] = {"tuning": best, "graphs": len(idx), "sample_graphs": len(pick), "sample_edges": tot,
                    "default_ms": base_ms, "tuned_ms": tuned_ms, "est_saving_ms": saving}
        if log:
            log(f"tune {b}: {len(pick)} of {len(idx)} graphs, {tot} edges: default {base_ms:.2f} ms, "
                f"tuned {tuned_ms:.2f} ms with {best}")
    return table


def apply_table(h: bfc.Graph, table: dict, buckets: list[str], min_saving_ms: float = 10.0) -> bool:
    """Installs each graph's bucket setting on a batch handle when the
    buckets' estimated savings add up to at least `min_saving_ms` per count
    (installing rebuilds the schedule: about 8 ms on the 4,096-graph batch of
    5.9e8 edges); otherwise installs nothing and returns False."""
    if sum(v.get("est_saving_ms", 0.0) for v in table.values()) < min_saving_ms:
        return False
    per_graph = [table.get(b, {}).get("tuning", {}) for b in buckets]
    if not any(per_graph):
        return False
    h.set_graph_tuning(per_graph)
    return True


def save(table: dict, path: str) -> None:
    with open(path, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)


def load_table(path: str) -> dict:
    with open(path) as f:
        return json.load(f)
