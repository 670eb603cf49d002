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
import glob
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak, GB/s
DEFAULT_WORKLOAD = "chunglu-1m-500k-20m"

# HBM traffic of one heavy-kernel launch per workload, from rocprofv3 --pmc
# runs (mean over the profiled dispatches): TCC_EA0_RDREQ_sum read requests
# (none of them 32-byte requests, TCC_BUBBLE_sum a few hundred), each 128
# bytes -- a plain 1 GiB device-to-device copy issues 8,388,792 such
# requests, and FETCH_SIZE counts them as 64 bytes, hence its factor 2 --
# and, in a separate run, WRITE_SIZE (KiB, factor 1.0 on the same copy).
# Reported only while the heavy kernel's sources hash to the value they were
# measured with (any change voids the figures).
HEAVY_TRAFFIC = {
    "sources_sha256": "c3631527911edf7c7f5e62fdb51eb9018816b8b343099eb79060468548b7fffd",
    "bytes_per_read_request": 128.0,
    "write_factor": 1.0,
    "workloads": {
        DEFAULT_WORKLOAD: {"read_requests": 234124042.0, "write_kib": 946409.3},
        "chunglu-16m-4m-200m-planted": {"read_requests": 8317063922.5, "write_kib": 55845976.5},
    },
}


def log(msg: str) -> None:
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def heavy_kernel_bytes(si: dict) -> int:
    """Algorithmic bytes of one heavy-kernel launch: 4 per wedge (end id),
    16 per middle arc (middle id, reverse slot, middle's offset, cursor/prefix
    bound) and 8 per start (offset and prefix length)."""
    return 4 * si["wedges_heavy"] + 16 * si["middles_heavy"] + 8 * si["starts_heavy"]


# the heavy kernel's sources: its traffic counters stay valid while these are unchanged
HEAVY_SOURCES = ("count.hip", "device.hpp", "internal.hpp")


def sources_sha256() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1812_00283_amd", "csrc")
    for f in [os.path.join(csrc, n) for n in HEAVY_SOURCES]:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def heavy_traffic(workload: str, tuned: bool):
    """Measured HBM bytes per heavy-kernel launch (default settings), or None
    when they do not apply (other workload, tuning, or sources changed since
    the counters)."""
    t = HEAVY_TRAFFIC
    w = t["workloads"].get(workload)
    if tuned or w is None or sources_sha256() != t["sources_sha256"]:
        return None
    return w["read_requests"] * t["bytes_per_read_request"] + 1024.0 * w["write_kib"] * t["write_factor"]


def golden_caterpillars(name: str):
    path = os.path.join(ROOT, "tests", "golden", "caterpillars.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f).get(name)
    return rec["caterpillars"] if rec else None


def golden_total(name: str):
    path = os.path.join(ROOT, "tests", "golden", "workloads.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    rec = d.get(name)
    return (rec["total"], rec["vp_wedges"], rec["edges_sha256"]) if rec else None


def measured_copy_gbs(gib: int = 4, reps: int = 5) -> float:
    """Device-to-device copy bandwidth on this GPU (bytes read + written per
    second, best of `reps` copies of `gib` GiB), reported beside the published
    HBM peak."""
    import torch

    n = gib * (1 << 30) // 4
    src = torch.ones(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1000.0)
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * gib * (1 << 30) / best / 1e9


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


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
    # the calibration can underestimate the rate: add further slices of the
    # same random order until the sample has taken about target_s seconds
    while ts < 0.8 * target_s and k < n_side:
        rate = float(csum[k - 1]) / max(ts, 1e-6)
        k2 = min(n_side, int(np.searchsorted(csum, csum[k - 1] + rate * (target_s - ts))) + 1)
        if k2 <= k:
            break
        t = time.perf_counter()
        oracle.vertex_counts_subset(g, side, order[k:k2], threads)
        ts += time.perf_counter() - t
        k = k2
    share = float(csum[k - 1]) / total_cost
    est_full = ts / share
    # the same walk on one thread, over a slice of about 3 s of one thread's work
    k1 = min(n_side, int(np.searchsorted(csum, rate / threads * 3.0)) + 1)
    t = time.perf_counter()
    oracle.vertex_counts_subset(g, side, order[:k1], 1)
    t1 = time.perf_counter() - t
    share1 = float(csum[k1 - 1]) / total_cost
    return {
        "value": wedges / est_full,
        "unit": "wedges/s",
        "cores": threads,
        "cpu_model": cpu_model(),
        "host_cpus": os.cpu_count(),
        "oracle_counter_steps": total_cost,
        "single_thread": {"value": wedges / (t1 / share1), "unit": "wedges/s",
                          "sample": f"{k1} starts, {100 * share1:.2f}% of the counter steps, in {t1:.1f} s"},
        "kind": "oracle",
        "sample": (f"Eq. 1 walk from {k} of {n_side} {'upper' if side == 0 else 'lower'} starts "
                   f"(random, {100 * share:.1f}% of the oracle's {total_cost:.3g} counter steps) in {ts:.1f} s; "
                   f"whole-graph time estimated as {est_full:.1f} s; value = |W| of BFC-VP / that time"),
    }


SECONDARY_WORKLOAD = "chunglu-16m-4m-200m-planted"


def secondary_record(name: str, steps: int, warmup: int) -> dict:
    """The 200M-edge graph beside the headline: steps of bfc_build +
    bfc_count_total with the default settings and with the per-layer wedge
    direction the tuner picks on this graph (picked once, before the timed
    steps; the step then includes the schedule rebuild that applies it), each
    with the heavy kernel's roofline entry (HIP events on its stream)."""
    import torch

    import graphgen as gg
    from paper_1812_00283_amd import bfc, tune

    t = time.perf_counter()
    g = gg.workload(name)
    log(f"generated {name}: m={g.m} in {time.perf_counter() - t:.1f}s")
    gold = golden_total(name)
    if gold and gold[2] != g.sha256():
        gold = None
    edges = torch.from_numpy(np.ascontiguousarray(g.edges)).cuda()
    with bfc.Graph(edges, g.n_upper, g.n_lower) as h:
        choice, ms = tune.pick_direction(h)
    log(f"{name}: direction masks (count ms) {ms}: tuner picks {choice}")
    rec = {"workload": name, "m": g.m, "n_upper": g.n_upper, "n_lower": g.n_lower,
           "tuner_direction_count_ms": {str(k): v for k, v in ms.items()}}
    for label, tun in (("default", None), ("tuned", choice)):
        steps_s, count_s, heavy_ms, tots = [], [], [], set()
        si = None
        for i in range(warmup + steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h = bfc.Graph(edges, g.n_upper, g.n_lower)
            if tun:
                h.set_tuning(**tun)
            h.set_kernel_timing(True)
            tb = time.perf_counter()
            tot, wed = h.count_total()
            tc = time.perf_counter() - tb
            kt = h.kernel_times()
            si = h.schedule_info()
            h.close()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            tots.add((tot, wed))
            if i >= warmup:
                steps_s.append(dt)
                count_s.append(tc)
                heavy_ms.append(kt["heavy_ms"] / max(kt["calls"], 1))
            log(f"{name} {label} step {i}: {1e3 * dt:.1f} ms (count {1e3 * tc:.1f} ms, heavy {heavy_ms[-1] if heavy_ms else 0:.1f} ms)")
        assert len(tots) == 1, "totals differ between steps"
        tot, wed = tots.pop()
        hk = float(np.mean(heavy_ms))
        hb = heavy_kernel_bytes(si)
        ms_step = 1e3 * float(np.mean(steps_s))
        rec[label] = {
            "tuning": tun or "default", "ms_per_step": ms_step, "wedges_per_s": wed / (ms_step / 1e3),
            "count_ms": 1e3 * float(np.median(count_s)), "heavy_ms": hk,
            "heavy_roofline": {"achieved": hb / (hk / 1e3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": hb / (hk / 1e3) / 1e9 / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": hb,
                               "traffic": heavy_traffic(name, bool(tun and any(tun.values())))},
            "butterflies": tot, "wedges": wed, "exact_vs_oracle": bool(gold and gold[0] == tot and gold[1] == wed),
        }
    return rec


def bench_batch(args) -> int:
    """Batched form: all graphs in one handle (one build, one set of count
    launches replayed from a captured HIP graph) against a loop of
    bfc_build + bfc_count_total, one graph per handle, on the same GPU."""
    import torch

    import graphgen as gg
    from paper_1812_00283_amd import bfc

    from paper_1812_00283_amd import tune

    bfc.load()
    t = time.perf_counter()
    b = gg.batch_workload(count=args.graphs)
    log(f"generated {b.count} graphs, {int(b.offsets[-1])} edges in {time.perf_counter() - t:.1f}s")
    edges = torch.from_numpy(b.edges).cuda()
    stream = torch.cuda.Stream()  # capture needs a created stream
    torch.cuda.synchronize()
    totals = torch.zeros(b.count, dtype=torch.int64, device="cuda")
    # the tuner: per (size, skew) bucket, the fastest setting on a sample of
    # the bucket's graphs (before and outside the timed steps)
    t = time.perf_counter()
    buckets = tune.graph_buckets(b.edges, b.offsets, b.n_upper, b.n_lower)
    table = tune.tune_batch(b.edges, b.offsets, b.n_upper, b.n_lower, log=log)
    tune_s = time.perf_counter() - t
    log(f"tuned {len(table)} buckets in {tune_s:.1f}s")

    installed = []

    def batched(tuned: bool):
        """Steps of batched build (+ per-graph settings) + captured count,
        replayed; returns (build s, count s, totals, wedges)."""
        ref = None
        times_build, times_count = [], []
        for i in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h = bfc.build_batch(edges, b.offsets, b.n_upper, b.n_lower, stream)
            if tuned:
                installed.append(tune.apply_table(h, table, buckets))
            t1 = time.perf_counter()
            h.capture_total(totals, stream)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            h.replay(stream)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            got = totals.cpu().numpy().copy()
            ref = got if ref is None else ref
            assert (got == ref).all()
            if i >= args.warmup:
                times_build.append(t1 - t0)
                times_count.append(t3 - t2)
            wed = h.batch_wedges()
            h.close()
            log(f"batched{' tuned' if tuned else ''} step {i}: build {1e3 * (t1 - t0):.1f} ms, "
                f"replayed count {1e3 * (t3 - t2):.1f} ms")
        return float(np.median(times_build)), float(np.median(times_count)), ref, wed

    d_build, d_count, ref, wed = batched(False)
    t_build, t_count, ref_t, _ = batched(True)
    assert (ref_t == ref).all(), "tuned and default per-graph totals differ"
    batched_s = t_build + t_count
    # plain: one graph per handle
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain = np.zeros(b.count, np.int64)
    for g in range(b.count):
        lo, hi = int(b.offsets[g]), int(b.offsets[g + 1])
        if hi == lo:
            continue
        with bfc.Graph(edges[lo:hi], int(b.n_upper[g]), int(b.n_lower[g]), stream) as h:
            plain[g] = h.count_total(stream)[0]
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    assert (plain == ref).all(), "batched and plain totals differ"
    exact = None
    gold = os.path.join(ROOT, "tests", "golden", "batch.json")
    if os.path.exists(gold) and args.graphs == 4096:
        with open(gold) as f:
            rec = json.load(f)["batch-4096"]
        exact = bool(rec["sha256"] == b.sha256() and (np.array(rec["totals"]) == ref).all())
    print(json.dumps({
        "metric": "batched graphs/s (tuned)", "value": b.count / batched_s, "unit": "graphs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * batched_s, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": f"batch-{b.count}", "edges": int(b.offsets[-1]), "wedges": int(wed.sum()),
                   "exact_vs_oracle": exact},
        "batched_build_ms": 1e3 * t_build,
        "batched_count_ms": 1e3 * t_count,
        "default_tuning": {"graphs_per_s": b.count / (d_build + d_count), "build_ms": 1e3 * d_build,
                           "count_ms": 1e3 * d_count},
        "tuner": {"seconds": tune_s, "installed": bool(installed and installed[-1]),
                  "buckets": {k: {kk: v[kk] for kk in ("tuning", "graphs", "default_ms", "tuned_ms", "est_saving_ms")}
                              for k, v in table.items()}},
        "plain_graphs_per_s": b.count / plain_s, "plain_ms": 1e3 * plain_s,
        "speedup_vs_plain": plain_s / batched_s,
        "capture": "count only: the build waits on the device twice (degree check, schedule sizes), so it is "
                   "not capturable",
    }), flush=True)
    return 0


def bench_serve(args) -> int:
    """Served form: a prefix of the arrival trace replayed in real time against
    the continuous-batching server, then against the plain FIFO server."""
    import torch

    import graphgen as gg
    from paper_1812_00283_amd import bfc, serve

    bfc.load()
    reqs = gg.serve_schedule(duration_s=args.serve_seconds, m_hi=args.serve_max_edges)
    roots = {r.index: r.graph for r in reqs if r.follow_up_of < 0}
    t = time.perf_counter()
    built = dict(zip(roots, gg.spec_graphs(list(roots.values()))))
    offered_edges = sum(built[r.follow_up_of if r.follow_up_of >= 0 else r.index].m for r in reqs)
    log(f"trace: {len(reqs)} requests over {args.serve_seconds}s, {len(roots)} graphs, "
        f"{offered_edges} request edges; generated in {time.perf_counter() - t:.1f}s")
    arrivals = [r.arrival_s for r in reqs]

    def jobs():
        return [serve.Job(r.index, r.kind, r.follow_up_of if r.follow_up_of >= 0 else r.index,
                          built[r.follow_up_of if r.follow_up_of >= 0 else r.index].edges,
                          r.graph.n_upper, r.graph.n_lower) for r in reqs]

    free, total = torch.cuda.mem_get_info()
    budget = int(args.serve_budget_gb * (1 << 30)) if args.serve_budget_gb else int(0.6 * free)
    out = {}
    for name, srv in (("batched", serve.Server(budget, slots=4)), ("plain", serve.Server(budget, plain=True))):
        js = jobs()
        wall = serve.replay(js, arrivals, srv)
        st = serve.latency_stats(js)
        st.update({"wall_s": wall, "requests_per_s": len(js) / wall, "edges_per_s": offered_edges / wall,
                   "cache_hits": sum(j.cache_hit for j in js), "batched_requests": sum(j.batched for j in js),
                   "peak_admitted_gb": srv.peak / (1 << 30)})
        out[name] = (st, [j.result for j in js])
        log(f"{name}: p50 {st['p50_ms']:.1f} ms p99 {st['p99_ms']:.1f} ms, {st['requests_per_s']:.1f} req/s")
    assert out["batched"][1] == out["plain"][1], "served results differ between the mix and the plain server"
    bst, pst = out["batched"][0], out["plain"][0]
    # the oracle's answers for the checked requests (every request of at most
    # 1e6 edges and a seeded 2% of the larger ones), stored by
    # tests/golden/make_serve_golden.py
    oracle_check = None
    gold = os.path.join(ROOT, "tests", "golden", "serve_10s.json")
    if os.path.exists(gold):
        with open(gold) as f:
            grec = json.load(f)
        if (grec["trace"]["duration_s"] == args.serve_seconds and args.serve_max_edges == 50_000_000):
            results = {r.index: res for r, res in zip(reqs, out["batched"][1])}
            bad = []
            for k, v in grec["answers"].items():
                got = results[int(k)]
                got = list(got) if isinstance(got, tuple) else got
                if got != v:
                    bad.append(int(k))
            oracle_check = {"checked": len(grec["answers"]), "of_requests": len(reqs), "mismatches": len(bad),
                            "first_mismatches": bad[:10],
                            "rule": "every request with m <= 1e6 and a seeded 2% of the larger ones"}
            log(f"oracle check: {oracle_check['checked']} requests, {len(bad)} mismatches")
            assert not bad, f"served results differ from the oracle for requests {bad[:10]}"
    print(json.dumps({
        "metric": "served p99 latency", "value": bst["p99_ms"], "unit": "ms", "n_gpus": 1, "steps": 1,
        "warmup": 0, "ms_per_step": 1e3 * bst["wall_s"], "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": f"serve-{args.serve_seconds}s", "requests": len(reqs),
                   "offered_requests_per_s": len(reqs) / args.serve_seconds,
                   "offered_edges_per_s": offered_edges / args.serve_seconds, "budget_gb": budget / (1 << 30),
                   "max_edges_per_request": args.serve_max_edges},
        "batched": bst, "plain": pst, "results_identical": True, "oracle_check": oracle_check,
        "offered_vs_achieved": {"offered_requests_per_s": len(reqs) / args.serve_seconds,
                                "achieved_requests_per_s": bst["requests_per_s"],
                                "offered_edges_per_s": offered_edges / args.serve_seconds,
                                "achieved_edges_per_s": bst["edges_per_s"]},
    }), flush=True)
    return 0


def bench_kwing(args) -> int:
    """k-wing (Section 1) of the default workload: each step is one
    bfc_k_wing call (rounds of exact per-edge counting, removal of the edges
    below k and rebuild) on edges already in HBM."""
    import torch

    import graphgen as gg
    from paper_1812_00283_amd import bfc

    bfc.load()
    t = time.perf_counter()
    g = gg.workload(DEFAULT_WORKLOAD)
    log(f"generated {DEFAULT_WORKLOAD}: m={g.m} in {time.perf_counter() - t:.1f}s")
    edges = torch.from_numpy(np.ascontiguousarray(g.edges)).cuda()
    stream = torch.cuda.current_stream()
    times, ref = [], None
    for i in range(args.warmup + args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mask, cnt, w, r = bfc.k_wing(edges, g.n_upper, g.n_lower, args.k, stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        key = (w, r, int(cnt.sum().item()))
        ref = key if ref is None else ref
        assert key == ref, "k-wing results differ between steps"
        if i >= args.warmup:
            times.append(dt)
        log(f"k-wing step {i}: {1e3 * dt:.1f} ms, {w} of {g.m} edges in the {args.k}-wing after {r} rounds")
    ok = bool((cnt[mask] >= args.k).all().item()) and not bool(cnt[~mask].any().item())
    s = float(np.mean(times))
    print(json.dumps({
        "metric": "k-wing input edges/s", "value": g.m / s, "unit": "edges/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * s, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": f"kwing-{DEFAULT_WORKLOAD}", "k": args.k, "m": g.m, "wing_edges": ref[0],
                   "rounds": ref[1], "wing_butterfly_edge_sum": ref[2], "threshold_property": ok},
    }), flush=True)
    return 0


def bench_sorted(args) -> int:
    """Sort-based total count (Algorithm 6, pairs sorted in device memory) of
    the default workload on a built graph: each step is one
    bfc_count_total_sorted call over the wedges of Algorithm 2 (the reported
    value), then one over those of Algorithm 3 (BFC-VP++) and one hash-based
    bfc_count_total of the same handle, for comparison."""
    import torch

    import graphgen as gg
    from paper_1812_00283_amd import bfc

    bfc.load()
    g = gg.workload(DEFAULT_WORKLOAD)
    edges = torch.from_numpy(np.ascontiguousarray(g.edges)).cuda()
    gold = golden_total(DEFAULT_WORKLOAD)
    with bfc.Graph(edges, g.n_upper, g.n_lower) as h:
        wedges = h.info()["wedges"]
        ref = h.count_total()[0]
        times = {0: [], 1: [], "hash": []}
        chunks = {}
        for i in range(args.warmup + args.steps):
            got = {}
            for d in (0, 1):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                t, pairs, chunks[d] = h.count_total_sorted(args.max_pairs, direction=d)
                got[d] = time.perf_counter() - t0
                assert t == ref and pairs == wedges, "sorted count differs from the hash count"
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            h.count_total()
            got["hash"] = time.perf_counter() - t1
            if i >= args.warmup:
                for k, v in got.items():
                    times[k].append(v)
            log(f"sorted step {i}: Algorithm 2 wedges {1e3 * got[0]:.1f} ms ({chunks[0]} chunks), "
                f"Algorithm 3 wedges {1e3 * got[1]:.1f} ms ({chunks[1]} chunks), hash count {1e3 * got['hash']:.2f} ms")
    ms = {k: 1e3 * float(np.mean(v)) for k, v in times.items()}
    print(json.dumps({
        "metric": "wedges/sec at exact counts (sort-based)", "value": wedges / (ms[0] / 1e3), "unit": "wedges/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms[0], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": f"sorted-{DEFAULT_WORKLOAD}", "wedges": wedges, "chunks": chunks[0],
                   "max_pairs": args.max_pairs, "butterflies": ref,
                   "exact_vs_oracle": gold is not None and gold[0] == ref and gold[1] == wedges},
        "vpp_direction": {"ms": ms[1], "wedges_per_s": wedges / (ms[1] / 1e3), "chunks": chunks[1]},
        "hash_count_ms": ms["hash"],
    }), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the 200M-edge graph's record that follows the headline")
    ap.add_argument("--steps-only", action="store_true",
                    help="time the steps only: no per-vertex / per-edge counts and no copy measurement afterwards "
                         "(for profiler runs whose kernels should all be steps)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of this many MiB (calibrates HBM counters)")
    ap.add_argument("--tuning", default="", help='JSON dict of bfc_set_tuning fields, e.g. {"window_mode": 3}')
    ap.add_argument("--graphs", type=int, default=4096, help="graphs in the batched workload")
    ap.add_argument("--serve-seconds", type=float, default=10.0, help="prefix of the arrival trace to serve")
    ap.add_argument("--serve-max-edges", type=int, default=50_000_000)
    ap.add_argument("--serve-budget-gb", type=float, default=0.0)
    ap.add_argument("--k", type=int, default=10000, help="threshold of the k-wing workload")
    ap.add_argument("--max-pairs", type=int, default=0, help="pairs per chunk of the sort-based count (0: 2^31)")
    args = ap.parse_args()
    if args.workload == "batch" and args.gpus == 1:
        return bench_batch(args)
    if args.workload == "serve" and args.gpus == 1:
        return bench_serve(args)
    if args.workload == "kwing" and args.gpus == 1:
        return bench_kwing(args)
    if args.workload == "sorted" and args.gpus == 1:
        return bench_sorted(args)
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

    tuning = json.loads(args.tuning) if args.tuning else None

    def step(timing: bool):
        h = bfc.Graph(edges, g.n_upper, g.n_lower, stream)
        if tuning:
            h.set_tuning(**tuning)
        if timing:
            h.set_kernel_timing(True)
        tb = time.perf_counter()
        tot, wed = h.count_total(stream)
        tc = time.perf_counter() - tb
        kt = h.kernel_times() if timing else None
        si = h.schedule_info()
        si["caterpillars"] = h.caterpillars()
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
        log(f"step {i}: count {1e3 * tc:.2f} ms (heavy kernel {heavy_ms[-1]:.2f} ms, light {light_ms[-1]:.2f} ms)")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    assert all(x == tot0 for x in totals), "totals differ between steps"
    log(f"timed {args.steps} steps in {elapsed:.3f}s")

    ms_step = 1000.0 * elapsed / args.steps
    wedges = wed0

    # per-vertex and per-edge counts (Lemma 1, Algorithm 4) on one more
    # handle, after the timed steps: median of three calls each
    def timed_calls(fn, n=3):
        ts = []
        for _ in range(n):
            torch.cuda.synchronize()
            tb = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - tb)
        return 1000.0 * float(np.median(ts))

    vertex_ms = edge_ms = None
    if not args.steps_only:
        with bfc.Graph(edges, g.n_upper, g.n_lower, stream) as h:
            if tuning:
                h.set_tuning(**tuning)
            vertex_ms = timed_calls(lambda: h.count_per_vertex(stream))
            edge_ms = timed_calls(lambda: h.count_per_edge(stream))
    # algorithmic bytes of a whole total count (4 per wedge, 16 per arc, 8 per
    # vertex) twice (two walks) plus 40 per edge (accumulators and output)
    per_edge_bytes = 2 * (4 * wedges + 16 * g.m + 8 * (g.n_upper + g.n_lower)) + 40 * g.m
    hk_ms = float(np.mean(heavy_ms))
    hk_bytes = heavy_kernel_bytes(si)
    achieved = hk_bytes / (hk_ms / 1000.0) / 1e9 if hk_ms > 0 else 0.0
    count_ms = 1000.0 * float(np.median(count_s))
    traffic = heavy_traffic(args.workload, bool(tuning))
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
            "tuning": tuning or "default",
            "caterpillars": si["caterpillars"],
            "clustering_coefficient": 4.0 * tot0 / si["caterpillars"] if si["caterpillars"] else 0.0,
            "caterpillars_exact_vs_oracle": golden_caterpillars(args.workload) == si["caterpillars"],
        },
        "count_ms": count_ms,
        "build_ms": ms_step - count_ms,
        "library_built_from_current_sources": bfc.library_matches_sources(),
        "count_only_wedges_per_s": wedges / (count_ms / 1000.0),
        "count_phase_roofline": {
            "algorithmic_bytes": 4 * wedges + 16 * g.m + 8 * (g.n_upper + g.n_lower),
            "achieved_GBps": (4 * wedges + 16 * g.m + 8 * (g.n_upper + g.n_lower)) / count_ms / 1e6,
            "frac": (4 * wedges + 16 * g.m + 8 * (g.n_upper + g.n_lower)) / count_ms / 1e6 / HBM_PEAK_GBS,
            "note": "whole count phase (light + heavy kernels), 4|W| + 16m + 8n over bfc_count_total's time"},
        "per_vertex_count_ms": vertex_ms,
        "per_edge_count_ms": edge_ms,
        "per_edge_roofline": None if edge_ms is None else {
            "algorithmic_bytes": per_edge_bytes, "achieved_GBps": per_edge_bytes / edge_ms / 1e6,
            "frac": per_edge_bytes / edge_ms / 1e6 / HBM_PEAK_GBS},
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
            "traffic": traffic,
            "traffic_unit": "bytes per launch (rocprofv3 TCC_EA0_RDREQ x 128 B + WRITE_SIZE, copy-calibrated)",
            "algorithmic_bytes_per_launch": hk_bytes,
            "avg_launch_ms": hk_ms,
            "copy_measured": None if args.steps_only else measured_copy_gbs(),
            "copy_measured_unit": "GB/s, best device-to-device copy of 4 GiB (read + write bytes), after the timed steps",
        },
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample")
        result["cpu_baseline"] = cpu_baseline(g, wedges)
    if args.workload == DEFAULT_WORKLOAD and not args.steps_only and not args.no_secondary:
        del edges, g
        torch.cuda.empty_cache()
        result["secondary"] = secondary_record(SECONDARY_WORKLOAD, steps=3, warmup=1)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
