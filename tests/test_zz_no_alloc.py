"""bfc_count_total_static: the total count with its scratch in the library's
fixed device array, for callers that cannot allocate.  Checked against
bfc_count_total_async on the same handle (and the oracle), on two calls in a
row, the second on a smaller graph, with an allocator installed that records
every request: the static calls must make none."""
import ctypes

import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
from gpu_util import to_dev

pytestmark = pytest.mark.gpu


def _call_static(lib, h, out, stream):
    return lib.bfc_count_total_static(h._h, ctypes.c_void_p(stream.cuda_stream), ctypes.c_void_p(out.data_ptr()))


def test_static_equals_async_twice_and_allocates_nothing(gpu_lib):
    bfc = gpu_lib
    lib = bfc.load()
    assert lib.bfc_static_scratch_bytes() == 64 << 20
    big = gg.workload("chunglu-1m-500k-20m")
    small = gg.chung_lu(11, 30_000, 20_000, 400_000, 2.1, 2.1, 5000.0)
    s = torch.cuda.Stream()
    handles = [bfc.Graph(to_dev(g), g.n_upper, g.n_lower, stream=s) for g in (big, small)]
    ref = []
    for h in handles:
        o = torch.zeros(1, dtype=torch.int64, device="cuda")
        h.count_total_async(o, stream=s)
        s.synchronize()
        ref.append(int(o.item()))
    assert ref[1] == oracle.total(small)
    # from here on every device allocation the library makes is recorded
    torch.cuda.synchronize()
    bfc.trim_cache()
    asked = []

    def alloc(n, st):
        asked.append(n)
        return torch.cuda.caching_allocator_alloc(n, torch.cuda.current_device(), st)

    bfc.set_allocator(alloc, lambda p, st: torch.cuda.caching_allocator_delete(p))
    try:
        outs = [torch.full((1,), -1, dtype=torch.int64, device="cuda") for _ in handles]
        for h, o in zip(handles, outs):  # big graph, then the smaller one
            assert _call_static(lib, h, o, s) == 0, lib.bfc_last_error()
            s.synchronize()
        assert [int(o.item()) for o in outs] == ref
        # again in the same order: the array keeps the last call's contents
        for h, o in zip(handles, outs):
            o.fill_(-1)
            assert _call_static(lib, h, o, s) == 0, lib.bfc_last_error()
            h.sync(s)
        assert [int(o.item()) for o in outs] == ref
        assert asked == [], f"static calls allocated {asked}"
    finally:
        bfc.use_torch_allocator()
        for h in handles:
            h.close()


def test_static_is_capturable(gpu_lib):
    bfc = gpu_lib
    g = gg.chung_lu(12, 20_000, 15_000, 300_000, 2.1, 2.1, 4000.0)
    ref = oracle.total(g)
    s = torch.cuda.Stream()
    with bfc.Graph(to_dev(g), g.n_upper, g.n_lower, stream=s) as h:
        out = torch.zeros(1, dtype=torch.int64, device="cuda")
        h.count_total_static(out, stream=s)  # warm: first use looks up the array's address
        s.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=s):
            h.count_total_static(out, stream=s)
        for _ in range(3):
            out.fill_(-1)
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            assert int(out.item()) == ref


def test_static_rejects_a_start_beyond_the_array(gpu_lib):
    """Two upper vertices sharing 6M lower neighbours: the second has 6M
    lower-priority middles, whose cursors (28 bytes each) exceed 64 MiB."""
    bfc = gpu_lib
    lib = bfc.load()
    n = 6_000_000
    e = np.empty((2 * n, 2), np.int32)
    e[:n, 0], e[n:, 0] = 0, 1
    e[:n, 1] = e[n:, 1] = np.arange(n, dtype=np.int32)
    with bfc.Graph(torch.from_numpy(e).cuda(), 2, n) as h:
        assert h.schedule_info()["starts_heavy"] == 1
        out = torch.full((1,), -7, dtype=torch.int64, device="cuda")
        st = _call_static(lib, h, out, torch.cuda.current_stream())
        assert st == 4, lib.bfc_last_error()  # BFC_ERR_TOO_LARGE
        assert b"static buffer" in lib.bfc_last_error()
        torch.cuda.synchronize()
        assert int(out.item()) == -7  # nothing written
