"""Serving loop for butterfly-count requests over the C ABI.

Requests (total, per-vertex or per-edge counts of one bipartite graph) arrive
over time.  The server

* admits work while its estimated device footprint fits the HBM budget
  (``bfc_estimate_device_bytes`` plus the uploaded edges and the outputs;
  a follow-up on a resident graph reserves its outputs only, since the
  graph's own reservation covers its count accumulators), counting the
  library's idle cached blocks against the budget and trimming them when a
  job does not fit, and evicting idle cached graphs least-recently-used
  first.  A job larger than the whole budget can never fit beside others:
  it is admitted alone once the server is idle (nothing admitted), so it
  runs rather than waiting forever;
* keeps built graphs device-resident so that follow-up queries on the same
  graph skip the build;
* runs admitted work on several HIP streams ("slots") at once, so jobs that
  arrive while others are on the GPU overlap with them;
* merges pending small total-count requests into one batched build and one
  set of counting launches (``bfc_build_batch`` / ``bfc_count_total_batch``).

All counting happens in libbfc; this module only schedules.  ``plain=True``
serves the same trace first-in first-out, one request at a time, with no
cache and no batching (the baseline the batched server is compared with).
"""
from __future__ import annotations

import hashlib
import threading
import time
from collections import OrderedDict, deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import bfc


@dataclass
class Job:
    index: int
    kind: str                 # "total" | "vertex" | "edge"
    key: int                  # graph identity (requests with the same key share a graph)
    edges: object             # int32 [m, 2] host edge list: numpy array, or a pinned CPU tensor (copied asynchronously)
    n_upper: int
    n_lower: int
    arrival: float = 0.0      # monotonic seconds when submitted
    started: float = 0.0
    done: float = 0.0
    result: object = None     # int (total) or (sha256 hex, sum) of the output arrays
    cache_hit: bool = False
    batched: bool = False
    event: threading.Event = field(default_factory=threading.Event)

    @property
    def m(self) -> int:
        return int(self.edges.shape[0])


def digest(*arrays: torch.Tensor) -> tuple[str, int]:
    h = hashlib.sha256()
    total = 0
    for a in arrays:
        x = a.cpu().numpy().astype("<i8")
        h.update(x.tobytes())
        total += int(x.sum())
    return h.hexdigest(), total


def _host_tensor(edges) -> torch.Tensor:
    """A request's edge list as a CPU tensor: pinned tensors are copied to the
    device asynchronously on the worker's stream (DMA, no staging); numpy
    arrays go through a pageable copy."""
    if isinstance(edges, torch.Tensor):
        return edges
    return torch.from_numpy(np.ascontiguousarray(edges))


def out_bytes(m: int, nu: int, nl: int, kind: str) -> int:
    """Device bytes of a request's outputs."""
    if kind == "vertex":
        return 8 * (nu + nl)
    if kind == "edge":
        return 8 * m
    return 0


def job_bytes(m: int, nu: int, nl: int, kind: str) -> int:
    """A request that builds its graph: graph (build peak and count
    accumulators), uploaded edges and outputs."""
    return bfc.estimate_device_bytes(m, nu, nl) + 8 * m + out_bytes(m, nu, nl, kind)


class _Resident:
    def __init__(self, graph: bfc.Graph, nbytes: int):
        self.graph = graph
        self.bytes = nbytes
        self.users = 0


class Server:
    def __init__(self, budget_bytes: int, slots: int = 4, batch_max_edges: int = 4_000_000,
                 batch_small_edges: int = 200_000, batch_max_graphs: int = 512, cache: bool = True,
                 batching: bool = True, plain: bool = False):
        self.budget = int(budget_bytes)
        self.plain = plain
        self.slots = 1 if plain else max(1, slots)
        self.cache_on = cache and not plain
        self.batching = batching and not plain
        self.batch_max_edges = batch_max_edges
        self.batch_small_edges = batch_small_edges
        self.batch_max_graphs = batch_max_graphs
        self.used = 0
        self.peak = 0
        self.cache: OrderedDict[int, _Resident] = OrderedDict()
        self.pending: deque[Job] = deque()
        self.lock = threading.Condition()
        self.units: deque = deque()
        self.stop_flag = False
        self.errors: list[BaseException] = []
        self.completed: list[Job] = []
        self.inflight_keys: set[int] = set()
        self.threads = [threading.Thread(target=self._dispatch, daemon=True)]
        self.threads += [threading.Thread(target=self._worker, args=(i,), daemon=True) for i in range(self.slots)]

    # ---------------------------------------------------------------- api
    def start(self):
        for t in self.threads:
            t.start()
        return self

    def submit(self, job: Job) -> None:
        job.arrival = time.monotonic()
        with self.lock:
            self.pending.append(job)
            self.lock.notify_all()

    def close(self):
        with self.lock:
            self.stop_flag = True
            self.lock.notify_all()
        for t in self.threads:
            t.join()
        for r in self.cache.values():
            r.graph.close()
        self.cache.clear()
        if self.errors:
            raise self.errors[0]

    # ---------------------------------------------------------------- dispatcher
    def _in_use(self) -> int:
        """Admitted bytes plus the library's idle cached blocks."""
        return self.used + bfc.cached_bytes()

    def _evict_for(self, need: int, keep: int | None = None) -> bool:
        """Makes room for `need` more bytes: first returns the library's idle
        cached blocks, then frees idle resident graphs (LRU first, never
        `keep`)."""
        if self._in_use() + need > self.budget:
            bfc.trim_cache()
        while self._in_use() + need > self.budget:
            victim = next((k for k, r in self.cache.items() if r.users == 0 and k != keep), None)
            if victim is None:
                return False
            r = self.cache.pop(victim)
            r.graph.close()
            self.used -= r.bytes
            bfc.trim_cache()
        return True

    def _next_unit(self):
        """Picks the next unit of work from `pending` that fits the budget, or None."""
        if not self.pending:
            return None
        job = self.pending[0]
        if self.plain:
            need = job_bytes(job.m, job.n_upper, job.n_lower, job.kind)
            if not self._evict_for(need) and self.used > 0:
                return None
            self.pending.popleft()
            self.used += need
            return ("single", [job], need)
        # follow-up on a resident graph: no build
        for i, jb in enumerate(self.pending):
            if jb.key in self.cache and jb.key not in self.inflight_keys:
                r = self.cache[jb.key]
                need = out_bytes(jb.m, jb.n_upper, jb.n_lower, jb.kind)
                if not self._evict_for(need, keep=jb.key):
                    continue
                del self.pending[i]
                r.users += 1
                self.cache.move_to_end(jb.key)
                self.used += need
                jb.cache_hit = True
                return ("resident", [jb], need)
        # small total-count jobs arriving together share one batched build
        if self.batching:
            group, edges = [], 0
            for jb in list(self.pending):
                if (jb.kind == "total" and jb.m <= self.batch_small_edges and jb.key not in self.cache
                        and jb.key not in self.inflight_keys and edges + jb.m <= self.batch_max_edges
                        and len(group) < self.batch_max_graphs):
                    group.append(jb)
                    edges += jb.m
            if len(group) > 1:
                need = sum(job_bytes(j.m, j.n_upper, j.n_lower, "total") for j in group)
                if self._evict_for(need) or self.used == 0:
                    for jb in group:
                        self.pending.remove(jb)
                        jb.batched = True
                    self.used += need
                    return ("batch", group, need)
        # otherwise the oldest job that is not waiting for its graph, built on its own
        for i, jb in enumerate(self.pending):
            if jb.key in self.inflight_keys:
                continue  # its graph is being built: it will be served from the cache
            need = job_bytes(jb.m, jb.n_upper, jb.n_lower, jb.kind)
            if not self._evict_for(need) and self.used > 0:
                return None
            del self.pending[i]
            self.used += need
            self.inflight_keys.add(jb.key)
            return ("single", [jb], need)
        return None

    def _dispatch(self):
        try:
            while True:
                with self.lock:
                    while True:
                        if self.stop_flag and not self.pending:
                            for _ in range(self.slots):
                                self.units.append(None)
                            self.lock.notify_all()
                            return
                        busy = sum(1 for u in self.units if u is not None)
                        unit = self._next_unit() if busy < self.slots else None
                        if unit is not None:
                            self.peak = max(self.peak, self.used)
                            self.units.append(unit)
                            self.lock.notify_all()
                            continue
                        self.lock.wait(0.002)
        except BaseException as e:  # pragma: no cover - surfaced by close()
            self.errors.append(e)
            with self.lock:
                for _ in range(self.slots):
                    self.units.append(None)
                self.lock.notify_all()

    # ---------------------------------------------------------------- workers
    def _worker(self, slot: int):
        stream = torch.cuda.Stream()
        while True:
            with self.lock:
                while not self.units:
                    self.lock.wait(0.01)
                unit = self.units.popleft()
                self.lock.notify_all()
            if unit is None:
                return
            kind, jobs, need = unit
            try:
                with torch.cuda.stream(stream):
                    self._run(kind, jobs, stream)
            except BaseException as e:
                self.errors.append(e)
            finally:
                with self.lock:
                    self.used -= need
                    for jb in jobs:
                        self.inflight_keys.discard(jb.key)
                    self.lock.notify_all()
                for jb in jobs:
                    jb.event.set()

    def _answer(self, g: bfc.Graph, job: Job, stream) -> None:
        if job.kind == "total":
            job.result = g.count_total(stream)[0]
        elif job.kind == "vertex":
            up, lo = g.count_per_vertex(stream)
            stream.synchronize()
            job.result = digest(up, lo)
        else:
            be = g.count_per_edge(stream)
            stream.synchronize()
            job.result = digest(be)

    def _run(self, kind: str, jobs: list[Job], stream) -> None:
        t0 = time.monotonic()
        for jb in jobs:
            jb.started = t0
        if kind == "resident":
            jb = jobs[0]
            with self.lock:
                r = self.cache[jb.key]
            try:
                self._answer(r.graph, jb, stream)
            finally:
                with self.lock:
                    r.users -= 1
            jb.done = time.monotonic()
            self.completed.append(jb)
            return
        if kind == "batch":
            offs = np.zeros(len(jobs) + 1, np.int64)
            offs[1:] = np.cumsum([jb.m for jb in jobs])
            dev = torch.empty((int(offs[-1]), 2), dtype=torch.int32, device="cuda")
            for jb, o in zip(jobs, offs):
                if jb.m:
                    dev[int(o):int(o) + jb.m].copy_(_host_tensor(jb.edges), non_blocking=True)
            with bfc.build_batch(dev, offs, [jb.n_upper for jb in jobs], [jb.n_lower for jb in jobs], stream) as g:
                totals = g.count_total_batch(stream=stream).cpu().numpy()
            now = time.monotonic()
            for jb, t in zip(jobs, totals):
                jb.result = int(t)
                jb.done = now
                self.completed.append(jb)
            return
        jb = jobs[0]
        dev = _host_tensor(jb.edges).to("cuda", non_blocking=True)
        g = bfc.Graph(dev, jb.n_upper, jb.n_lower, stream)
        del dev
        try:
            self._answer(g, jb, stream)
        finally:
            keep = False
            if self.cache_on:
                # the larger of the estimate and what the handle holds (its
                # scratch depends on the graph's largest degrees)
                nbytes = max(bfc.estimate_device_bytes(jb.m, jb.n_upper, jb.n_lower), g.info()["device_bytes"])
                with self.lock:
                    if jb.key not in self.cache and self._in_use() + nbytes <= self.budget:
                        self.cache[jb.key] = _Resident(g, nbytes)
                        self.used += nbytes
                        keep = True
            if not keep:
                g.close()
        jb.done = time.monotonic()
        self.completed.append(jb)


def replay(jobs: list[Job], arrivals: list[float], server: Server, time_scale: float = 1.0) -> float:
    """Submits jobs at their arrival offsets (seconds) and waits for all; returns wall seconds."""
    server.start()
    t0 = time.monotonic()
    for jb, a in zip(jobs, arrivals):
        delay = t0 + a * time_scale - time.monotonic()
        if delay > 0:
            time.sleep(delay)
        server.submit(jb)
    for jb in jobs:
        jb.event.wait()
    wall = time.monotonic() - t0
    server.close()
    return wall


def latency_stats(jobs: list[Job]) -> dict:
    lat = np.array([jb.done - jb.arrival for jb in jobs])
    return {
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "max_ms": float(lat.max() * 1e3),
        "mean_ms": float(lat.mean() * 1e3),
    }
