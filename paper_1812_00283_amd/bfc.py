"""Python binding of libbfc (ctypes).  Argument marshalling only.

Every step of the counting path runs in the HIP library: this module passes
device pointers of torch tensors and the current HIP stream to the C entry
points of ``include/bfc.h`` and turns status codes into exceptions.  If the
library has not been built, ``load()`` raises; there is no fallback.
"""
from __future__ import annotations

import ctypes
import sys
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libbfc.so")
_lib = None

OK = 0
STATUS = {
    0: "BFC_OK",
    1: "BFC_ERR_INVALID_ARGUMENT",
    2: "BFC_ERR_VERTEX_OUT_OF_RANGE",
    3: "BFC_ERR_DUPLICATE_EDGE",
    4: "BFC_ERR_TOO_LARGE",
    5: "BFC_ERR_OUT_OF_MEMORY",
    6: "BFC_ERR_DEVICE",
}

EXPORTS = [
    "bfc_build", "bfc_count_total", "bfc_count_total_async", "bfc_count_per_vertex", "bfc_count_per_edge",
    "bfc_graph_info", "bfc_estimate_device_bytes", "bfc_destroy", "bfc_set_tuning", "bfc_get_tuning",
    "bfc_last_error", "bfc_version", "bfc_get_schedule_info", "bfc_set_kernel_timing", "bfc_get_kernel_times",
    "bfc_build_batch", "bfc_count_total_batch", "bfc_batch_wedges", "bfc_graph_capture_total", "bfc_graph_replay",
    "bfc_graph_count", "bfc_caterpillars", "bfc_clustering_coefficient", "bfc_k_wing",
    "bfc_count_total_sorted", "bfc_sync", "bfc_set_allocator", "bfc_trim_cache", "bfc_cached_bytes",
    "bfc_count_total_static", "bfc_static_scratch_bytes", "bfc_set_graph_tuning",
]

# Signatures of the allocator functions bfc_set_allocator takes.
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)
_installed = None  # keeps the installed callbacks alive


class BfcError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class Tuning(ctypes.Structure):
    _fields_ = [("light_max_wedges", ctypes.c_int32), ("dense_min_ratio", ctypes.c_int32),
                ("window_mode", ctypes.c_int32), ("hash_window_wedges", ctypes.c_int32),
                ("dense_block", ctypes.c_int32), ("dense_min_wedges", ctypes.c_int32),
                ("medium_max_wedges", ctypes.c_int32), ("vpp", ctypes.c_int32),
                ("top_band", ctypes.c_int32)]


class ScheduleInfo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("wedges", "starts_light", "starts_heavy", "wedges_light",
                                               "wedges_heavy", "middles_light", "middles_heavy",
                                               "max_start_wedges", "starts_medium", "starts_small")]


class KernelTimes(ctypes.Structure):
    _fields_ = [("calls", ctypes.c_int64), ("light_ms", ctypes.c_double), ("heavy_ms", ctypes.c_double),
                ("other_ms", ctypes.c_double)]


def library_matches_sources() -> bool:
    """Whether the in-tree libbfc.so was built from the sources now in the
    tree (the digest its build recorded beside it)."""
    from . import build as _build

    try:
        with open(LIB_PATH + ".sources") as f:
            return f.read().strip() == _build.sources_digest()
    except OSError:
        return False


def load(path: str | None = None, torch_memory: bool = True):
    """Loads libbfc.so; raises if it has not been built.  With torch_memory
    (the default) the library takes its device memory from PyTorch's caching
    allocator (``bfc_set_allocator``)."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is missing: build it with `python -m paper_1812_00283_amd.build`")
    if path is None and not library_matches_sources():
        print(f"warning: {p} was not built from the current sources (rebuild with "
              "`python -m paper_1812_00283_amd.build`)", file=sys.stderr, flush=True)
    lib = ctypes.CDLL(p)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    pi64, pi32 = ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)
    sig = {
        "bfc_build": ([vp, i64, i32, i32, vp, ctypes.POINTER(vp)], i32),
        "bfc_count_total": ([vp, vp, pi64, pi64], i32),
        "bfc_count_total_async": ([vp, vp, vp], i32),
        "bfc_count_per_vertex": ([vp, vp, vp, vp], i32),
        "bfc_count_per_edge": ([vp, vp, vp], i32),
        "bfc_graph_info": ([vp, pi64, pi32, pi32, pi64, pi64], i32),
        "bfc_estimate_device_bytes": ([i64, i32, i32], i64),
        "bfc_destroy": ([vp], i32),
        "bfc_set_tuning": ([vp, ctypes.POINTER(Tuning)], i32),
        "bfc_get_tuning": ([vp, ctypes.POINTER(Tuning)], i32),
        "bfc_get_schedule_info": ([vp, ctypes.POINTER(ScheduleInfo)], i32),
        "bfc_set_kernel_timing": ([vp, i32], i32),
        "bfc_get_kernel_times": ([vp, ctypes.POINTER(KernelTimes)], i32),
        "bfc_build_batch": ([vp, vp, vp, vp, i32, vp, ctypes.POINTER(vp)], i32),
        "bfc_count_total_batch": ([vp, vp, vp], i32),
        "bfc_batch_wedges": ([vp, vp], i32),
        "bfc_graph_capture_total": ([vp, vp, vp], i32),
        "bfc_graph_replay": ([vp, vp], i32),
        "bfc_graph_count": ([vp, pi32], i32),
        "bfc_caterpillars": ([vp, pi64], i32),
        "bfc_clustering_coefficient": ([vp, vp, ctypes.POINTER(ctypes.c_double)], i32),
        "bfc_k_wing": ([vp, i64, i32, i32, i64, vp, vp, vp, pi64, pi32], i32),
        "bfc_count_total_sorted": ([vp, vp, i32, i64, pi64, pi64, pi64], i32),
        "bfc_sync": ([vp, vp], i32),
        "bfc_count_total_static": ([vp, vp, vp], i32),
        "bfc_static_scratch_bytes": ([], i64),
        "bfc_set_graph_tuning": ([vp, vp, i32], i32),
        "bfc_set_allocator": ([ALLOC_FN, FREE_FN, vp], i32),
        "bfc_trim_cache": ([], i64),
        "bfc_cached_bytes": ([], i64),
        "bfc_last_error": ([], ctypes.c_char_p),
        "bfc_version": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    if torch_memory:
        use_torch_allocator()
    return lib


def _torch_alloc(nbytes, stream, _ctx):
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(), int(stream or 0))
    except Exception:  # out of memory (or no device): the library reports BFC_ERR_OUT_OF_MEMORY
        return None


def _torch_free(ptr, _stream, _ctx):
    torch.cuda.caching_allocator_delete(int(ptr))


def set_allocator(alloc=None, free=None) -> None:
    """Installs Python functions alloc(bytes, stream) -> int pointer or None and
    free(ptr, stream) as the library's source of device memory
    (``bfc_set_allocator``); both None restores hipMalloc / hipFree."""
    global _installed
    if (alloc is None) != (free is None):
        raise ValueError("alloc and free must both be given or both be None")
    if alloc is None:
        pair = (ALLOC_FN(), FREE_FN())
    else:
        pair = (ALLOC_FN(lambda n, st, c: alloc(int(n), int(st or 0))),
                FREE_FN(lambda ptr, st, c: free(int(ptr), int(st or 0))))
    _check(load(torch_memory=False).bfc_set_allocator(pair[0], pair[1], None))
    _installed = pair


def use_torch_allocator() -> None:
    """Device memory from torch.cuda's caching allocator (counted in
    torch.cuda.memory_allocated while the library holds it)."""
    global _installed
    pair = (ALLOC_FN(_torch_alloc), FREE_FN(_torch_free))
    _check(load(torch_memory=False).bfc_set_allocator(pair[0], pair[1], None))
    _installed = pair


def trim_cache() -> int:
    """Returns the library's idle cached device blocks to their allocator (bytes)."""
    return int(load().bfc_trim_cache())


def cached_bytes() -> int:
    return int(load().bfc_cached_bytes())


def _check(status: int) -> None:
    if status != OK:
        raise BfcError(status, load().bfc_last_error().decode())


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _ptr(t: torch.Tensor | None) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr() if t is not None and t.numel() else None)


def version() -> str:
    return load().bfc_version().decode()


def estimate_device_bytes(m: int, n_upper: int, n_lower: int) -> int:
    return int(load().bfc_estimate_device_bytes(m, n_upper, n_lower))


class Graph:
    """A graph built on the GPU (``bfc_build``) and its count calls."""

    def __init__(self, edges: torch.Tensor, n_upper: int, n_lower: int, stream=None, _batch=None):
        lib = load()
        self.graphs = 1
        if not isinstance(edges, torch.Tensor) or edges.dtype != torch.int32 or not edges.is_cuda:
            raise TypeError("edges must be an int32 CUDA tensor of shape [m, 2]")
        if edges.dim() != 2 or edges.shape[1] != 2:
            raise ValueError("edges must have shape [m, 2]")
        edges = edges.contiguous()
        self.m = int(edges.shape[0])
        self.n_upper = int(n_upper)
        self.n_lower = int(n_lower)
        self.device = edges.device
        h = ctypes.c_void_p()
        if _batch is None:
            _check(lib.bfc_build(_ptr(edges), self.m, self.n_upper, self.n_lower, _stream(stream), ctypes.byref(h)))
        else:
            import numpy as np

            eoff, nus, nls = _batch
            eoff = np.ascontiguousarray(eoff, dtype=np.int64)
            nus = np.ascontiguousarray(nus, dtype=np.int32)
            nls = np.ascontiguousarray(nls, dtype=np.int32)
            if eoff[-1] != self.m:
                raise ValueError("edge offsets must end at the number of edges")
            self.graphs = len(nus)
            _check(lib.bfc_build_batch(_ptr(edges), eoff.ctypes.data, nus.ctypes.data, nls.ctypes.data,
                                       self.graphs, _stream(stream), ctypes.byref(h)))
        self._h = h

    # -- counts -------------------------------------------------------
    def count_total(self, stream=None) -> tuple[int, int]:
        """(B_G, |W|): the butterfly count and the wedges Algorithm 2 processes."""
        t = ctypes.c_int64(0)
        w = ctypes.c_int64(0)
        _check(load().bfc_count_total(self._h, _stream(stream), ctypes.byref(t), ctypes.byref(w)))
        return int(t.value), int(w.value)

    def count_total_async(self, out: torch.Tensor, stream=None) -> torch.Tensor:
        """Writes B_G into ``out`` (int64 CUDA tensor with one element) without synchronising."""
        if out.dtype != torch.int64 or not out.is_cuda or out.numel() < 1:
            raise TypeError("out must be an int64 CUDA tensor")
        _check(load().bfc_count_total_async(self._h, _stream(stream), _ptr(out)))
        return out

    def count_total_static(self, out: torch.Tensor, stream=None) -> torch.Tensor:
        """As count_total_async, with the kernels' scratch in the library's fixed
        device array (``bfc_count_total_static``: no allocation)."""
        if out.dtype != torch.int64 or not out.is_cuda or out.numel() < 1:
            raise TypeError("out must be an int64 CUDA tensor")
        _check(load().bfc_count_total_static(self._h, _stream(stream), _ptr(out)))
        return out

    def count_per_vertex(self, stream=None, sync: bool = True) -> tuple[torch.Tensor, torch.Tensor]:
        """(B_u by upper id, B_v by lower id), int64 CUDA tensors.  With sync
        (the default) waits for the count and raises if its kernels failed
        (``bfc_sync``); otherwise the call is asynchronous."""
        up = torch.empty(self.n_upper, dtype=torch.int64, device=self.device)
        lo = torch.empty(self.n_lower, dtype=torch.int64, device=self.device)
        _check(load().bfc_count_per_vertex(self._h, _stream(stream), _ptr(up), _ptr(lo)))
        if sync:
            self.sync(stream)
        return up, lo

    def count_per_edge(self, stream=None, sync: bool = True) -> torch.Tensor:
        """B_e in input edge order (int64 CUDA tensor [m]); sync as in count_per_vertex."""
        out = torch.empty(self.m, dtype=torch.int64, device=self.device)
        _check(load().bfc_count_per_edge(self._h, _stream(stream), _ptr(out)))
        if sync:
            self.sync(stream)
        return out

    def sync(self, stream=None) -> None:
        """Waits for the handle's counts; raises if any failed (``bfc_sync``)."""
        _check(load().bfc_sync(self._h, _stream(stream)))

    def count_total_sorted(self, max_pairs: int = 0, stream=None, direction: int = 0) -> tuple[int, int, int]:
        """(B_G, pairs, chunks) by Algorithm 6's pair sort (``bfc_count_total_sorted``)
        over the wedges of Algorithm 2 (direction 0) or Algorithm 3 (direction 1)."""
        t, p, c = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
        _check(load().bfc_count_total_sorted(self._h, _stream(stream), int(direction), int(max_pairs),
                                             ctypes.byref(t), ctypes.byref(p), ctypes.byref(c)))
        return int(t.value), int(p.value), int(c.value)

    def caterpillars(self) -> int:
        """C_G: the graph's three-paths, computed by the build."""
        c = ctypes.c_int64(0)
        _check(load().bfc_caterpillars(self._h, ctypes.byref(c)))
        return int(c.value)

    def clustering_coefficient(self, stream=None) -> float:
        """4 B_G / C_G (runs the total count)."""
        c = ctypes.c_double(0.0)
        _check(load().bfc_clustering_coefficient(self._h, _stream(stream), ctypes.byref(c)))
        return float(c.value)

    def count_total_batch(self, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """Per-graph totals (int64 CUDA tensor [graphs]); asynchronous."""
        if out is None:
            out = torch.empty(self.graphs, dtype=torch.int64, device=self.device)
        _check(load().bfc_count_total_batch(self._h, _stream(stream), _ptr(out)))
        return out

    def batch_wedges(self):
        import numpy as np

        w = np.zeros(self.graphs, dtype=np.int64)
        _check(load().bfc_batch_wedges(self._h, w.ctypes.data))
        return w

    def capture_total(self, out: torch.Tensor, stream=None) -> None:
        """Captures the per-graph total count into a HIP graph held by the handle."""
        self._captured_out = out
        _check(load().bfc_graph_capture_total(self._h, _stream(stream), _ptr(out)))

    def replay(self, stream=None) -> None:
        _check(load().bfc_graph_replay(self._h, _stream(stream)))

    # -- info and tuning ------------------------------------------------
    def info(self) -> dict:
        m, nu, nl, w, b = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
        _check(load().bfc_graph_info(self._h, ctypes.byref(m), ctypes.byref(nu), ctypes.byref(nl), ctypes.byref(w),
                                     ctypes.byref(b)))
        return {"m": m.value, "n_upper": nu.value, "n_lower": nl.value, "wedges": w.value, "device_bytes": b.value}

    def set_tuning(self, light_max_wedges: int = 0, dense_min_ratio: int = 0, window_mode: int = 0,
                   hash_window_wedges: int = 0, dense_block: int = -1, dense_min_wedges: int = 0,
                   medium_max_wedges: int = -1, vpp: int = -1, top_band: int = -1) -> None:
        """Changes which kernel path handles each start; no count changes.
        window_mode: 1 automatic, 2 dense windows only, 3 hash windows only.
        vpp: 1 counts Algorithm 3's wedges (BFC-VP++), 0 Algorithm 2's.
        top_band: width of each layer's top band of ranks (0: none)."""
        t = Tuning(light_max_wedges, dense_min_ratio, window_mode, hash_window_wedges, dense_block, dense_min_wedges,
                   medium_max_wedges, vpp, top_band)
        _check(load().bfc_set_tuning(self._h, ctypes.byref(t)))

    def set_graph_tuning(self, per_graph) -> None:
        """Per-graph settings of a batch handle (``bfc_set_graph_tuning``):
        one dict of bfc_set_tuning fields per graph (missing fields take the
        handle's); an empty list clears them."""
        fields = [f for f, _ in Tuning._fields_]
        if not per_graph:
            _check(load().bfc_set_graph_tuning(self._h, None, 0))
            return
        arr = (Tuning * len(per_graph))()
        for i, d in enumerate(per_graph):
            for f in fields:
                setattr(arr[i], f, int(d.get(f, -1 if f in ("dense_block", "medium_max_wedges", "vpp", "top_band") else 0)))
        _check(load().bfc_set_graph_tuning(self._h, ctypes.cast(arr, ctypes.c_void_p), len(per_graph)))

    def get_tuning(self) -> dict:
        t = Tuning()
        _check(load().bfc_get_tuning(self._h, ctypes.byref(t)))
        return {"light_max_wedges": t.light_max_wedges, "dense_min_ratio": t.dense_min_ratio,
                "window_mode": t.window_mode, "hash_window_wedges": t.hash_window_wedges,
                "dense_block": t.dense_block, "dense_min_wedges": t.dense_min_wedges,
                "medium_max_wedges": t.medium_max_wedges, "vpp": t.vpp, "top_band": t.top_band}

    def schedule_info(self) -> dict:
        si = ScheduleInfo()
        _check(load().bfc_get_schedule_info(self._h, ctypes.byref(si)))
        return {n: int(getattr(si, n)) for n, _ in ScheduleInfo._fields_}

    def set_kernel_timing(self, enable: bool) -> None:
        """Records HIP events around the count kernels of later calls (resets the sums)."""
        _check(load().bfc_set_kernel_timing(self._h, 1 if enable else 0))

    def kernel_times(self) -> dict:
        kt = KernelTimes()
        _check(load().bfc_get_kernel_times(self._h, ctypes.byref(kt)))
        return {"calls": int(kt.calls), "light_ms": kt.light_ms, "heavy_ms": kt.heavy_ms, "other_ms": kt.other_ms}

    # -- lifetime --------------------------------------------------------
    def close(self) -> None:
        if getattr(self, "_h", None):
            _check(load().bfc_destroy(self._h))
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


# Module-level names matching the C entry points.
def build(edges: torch.Tensor, n_upper: int, n_lower: int, stream=None) -> Graph:
    return Graph(edges, n_upper, n_lower, stream)


def build_batch(edges: torch.Tensor, edge_offsets, n_upper, n_lower, stream=None) -> Graph:
    """Batched build: graph g owns edge rows [edge_offsets[g], edge_offsets[g+1])."""
    return Graph(edges, int(sum(int(x) for x in n_upper)), int(sum(int(x) for x in n_lower)), stream,
                 _batch=(edge_offsets, n_upper, n_lower))


def k_wing(edges: torch.Tensor, n_upper: int, n_lower: int, k: int, stream=None, counts: bool = True):
    """The k-wing (``bfc_k_wing``): (in_wing bool [m], butterflies of each edge
    within the k-wing int64 [m] or None, wing edges, count rounds)."""
    if not isinstance(edges, torch.Tensor) or edges.dtype != torch.int32 or not edges.is_cuda:
        raise TypeError("edges must be an int32 CUDA tensor of shape [m, 2]")
    if edges.dim() != 2 or edges.shape[1] != 2:
        raise ValueError("edges must have shape [m, 2]")
    edges = edges.contiguous()
    m = int(edges.shape[0])
    mask = torch.empty(m, dtype=torch.uint8, device=edges.device)
    cnt = torch.empty(m, dtype=torch.int64, device=edges.device) if counts else None
    w, r = ctypes.c_int64(0), ctypes.c_int32(0)
    _check(load().bfc_k_wing(_ptr(edges), m, int(n_upper), int(n_lower), int(k), _stream(stream), _ptr(mask),
                             _ptr(cnt), ctypes.byref(w), ctypes.byref(r)))
    return mask.bool(), cnt, int(w.value), int(r.value)


def count_total(g: Graph, stream=None) -> tuple[int, int]:
    return g.count_total(stream)


def count_per_vertex(g: Graph, stream=None) -> tuple[torch.Tensor, torch.Tensor]:
    return g.count_per_vertex(stream)


def count_per_edge(g: Graph, stream=None) -> torch.Tensor:
    return g.count_per_edge(stream)
