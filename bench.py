"""Benchmark: exact BFC-VP butterfly counting on one MI355X.

One step = the whole path for an exact total count on one graph already
resident in HBM: bfc_build (validation, priorities, relabelled CSR,
schedule) followed by bfc_count_total (wedge counting, C(c,2) reduction).
The metric is wedges/s: |W| (the wedges Algorithm 2 processes) divided by
the step time.  Every step's total must equal the first one, and the
oracle's stored value when one exists.

Prints one JSON line (see the end of main) with a roofline entry for the
heavy-start counting kernel (timed with HIP events on the stream it runs on)
and the CPU oracle timed on a bounded sample of the same graph.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak, GB/s
DEFAULT_WORKLOAD = "chunglu-1m-500k-20m"


def log(msg: str) -> None:
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def heavy_kernel_bytes(si: dict) -> int:
    """Algorithmic bytes of one heavy-kernel launch: 4 per wedge (end id),
    16 per middle arc (middle id, reverse slot, middle's offset, cursor/prefix
    bound) and 8 per start (offset and prefix length)."""
    return 4 * si["wedges_heavy"] + 16 * si["middles_heavy"] + 8 * si["starts_heavy"]


def golden_total(name: str):
    path = os.path.join(ROOT, "tests", "golden", "workloads.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    rec = d.get(name)
    return (rec["total"], rec["vp_wedges"], rec["edges_sha256"]) if rec else None


def cpu_baseline(g, wedges: int, target_s: float = 15.0) -> dict:
    """The oracle (Lemma 1 Eq. 1 from the layer of the sum-of-squares rule) on a
    random sample of its start vertices, scaled to the whole graph by the
    sample's share of the oracle's work (sum over sampled starts of the degrees
    of their neighbours)."""
    import oracle

    side = oracle.cheaper_side(g)
    col, other = (0, 1) if side == 0 else (1, 0)
    n_side = g.n_upper if side == 0 else g.n_lower
    n_other = g.n_lower if side == 0 else g.n_upper
    d_other = np.bincount(g.edges[:, other], minlength=n_other).astype(np.float64)
    cost = np.bincount(g.edges[:, col], weights=d_other[g.edges[:, other]], minlength=n_side)
    total_cost = float(cost.sum())
    order = np.random.default_rng(2024).permutation(n_side)
    csum = np.cumsum(cost[order])
    threads = oracle.threads()
    # calibrate on ~0.5% of the work, then size the sample for ~target_s seconds
    k0 = int(np.searchsorted(csum, 0.005 * total_cost)) + 1
    t = time.perf_counter()
    oracle.vertex_counts_subset(g, side, order[:k0], threads)
    t0 = time.perf_counter() - t
    rate = float(csum[k0 - 1]) / max(t0, 1e-6)
    want = min(total_cost, rate * target_s)
    k = min(n_side, int(np.searchsorted(csum, want)) + 1)
    t = time.perf_counter()
    oracle.vertex_counts_subset(g, side, order[:k], threads)
    ts = time.perf_counter() - t
    share = float(csum[k - 1]) / total_cost
    est_full = ts / share
    return {
        "value": wedges / est_full,
        "unit": "wedges/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"Eq. 1 walk from {k} of {n_side} {'upper' if side == 0 else 'lower'} starts "
                   f"(random, {100 * share:.1f}% of the oracle's {total_cost:.3g} counter steps) in {ts:.1f} s; "
                   f"whole-graph time estimated as {est_full:.1f} s; value = |W| of BFC-VP / that time"),
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of this many MiB (calibrates HBM counters)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch

        n = args.copy_probe * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_mib": args.copy_probe, "launches": 3}), flush=True)
        return 0
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the counting path is a "
              "single-GPU build and no multi-GPU figure is produced", file=sys.stderr)
        return 2

    import torch

    import graphgen as gg
    from paper_1812_00283_amd import bfc

    bfc.load()
    torch.cuda.set_device(0)
    t = time.perf_counter()
    g = gg.workload(args.workload)
    log(f"generated {args.workload}: m={g.m} in {time.perf_counter() - t:.1f}s")
    gold = golden_total(args.workload)
    if gold and gold[2] != g.sha256():
        log("warning: generated edges differ from the stored oracle record; exactness check skipped")
        gold = None
    edges = torch.from_numpy(np.ascontiguousarray(g.edges)).cuda()
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

    def step(timing: bool):
        h = bfc.Graph(edges, g.n_upper, g.n_lower, stream)
        if timing:
            h.set_kernel_timing(True)
        tb = time.perf_counter()
        tot, wed = h.count_total(stream)
        tc = time.perf_counter() - tb
        kt = h.kernel_times() if timing else None
        si = h.schedule_info()
        h.close()
        return tot, wed, tc, kt, si

    for i in range(args.warmup):
        tot0, wed0, _, _, si = step(False)
        log(f"warmup {i + 1}/{args.warmup}: total={tot0} wedges={wed0}")
    if args.warmup == 0:
        tot0, wed0, _, _, si = step(False)
    if gold:
        assert tot0 == gold[0] and wed0 == gold[1], (tot0, wed0, gold)

    totals, count_s, heavy_ms, light_ms = [], [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        tot, wed, tc, kt, si = step(True)
        totals.append(tot)
        count_s.append(tc)
        heavy_ms.append(kt["heavy_ms"] / max(kt["calls"], 1))
        light_ms.append(kt["light_ms"] / max(kt["calls"], 1))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    assert all(x == tot0 for x in totals), "totals differ between steps"
    log(f"timed {args.steps} steps in {elapsed:.3f}s")

    ms_step = 1000.0 * elapsed / args.steps
    wedges = wed0
    hk_ms = float(np.mean(heavy_ms))
    hk_bytes = heavy_kernel_bytes(si)
    achieved = hk_bytes / (hk_ms / 1000.0) / 1e9 if hk_ms > 0 else 0.0
    count_ms = 1000.0 * float(np.median(count_s))
    result = {
        "metric": "wedges/sec at exact counts",
        "value": wedges / (ms_step / 1000.0),
        "unit": "wedges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "n_upper": g.n_upper,
            "n_lower": g.n_lower,
            "m": g.m,
            "wedges": wedges,
            "butterflies": tot0,
            "step": "bfc_build + bfc_count_total on device-resident edges",
            "exact_vs_oracle": bool(gold),
        },
        "count_ms": count_ms,
        "build_ms": ms_step - count_ms,
        "count_only_wedges_per_s": wedges / (count_ms / 1000.0),
        "edges_per_s": g.m / (ms_step / 1000.0),
        "kernels_ms": {"heavy": hk_ms, "light": float(np.mean(light_ms))},
        "schedule": si,
        "roofline": {
            "bound": "hbm",
            "kernel": "heavy_kernel (workgroup per heavy start)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "algorithmic_bytes_per_launch": hk_bytes,
            "avg_launch_ms": hk_ms,
        },
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample")
        result["cpu_baseline"] = cpu_baseline(g, wedges)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
