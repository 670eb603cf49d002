"""The C-ABI boundary beyond the counts: where device memory comes from
(bfc_set_allocator, bfc_trim_cache), running out of it, the status check of
the asynchronous counts (bfc_sync) and a captured count after a retune."""
import ctypes

import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
from gpu_util import to_dev

pytestmark = pytest.mark.gpu


def _fresh_pool(bfc):
    """Idle cached blocks back to their allocator, with no work pending on them."""
    torch.cuda.synchronize()
    bfc.trim_cache()
    assert bfc.cached_bytes() == 0


def test_memory_comes_from_torch(gpu_lib):
    bfc = gpu_lib
    bfc.use_torch_allocator()
    g = gg.workload("uniform-2k-3k-20k")
    e = to_dev(g)
    _fresh_pool(bfc)
    before = torch.cuda.memory_allocated()
    with bfc.Graph(e, g.n_upper, g.n_lower) as h:
        held = h.info()["device_bytes"]
        assert torch.cuda.memory_allocated() - before >= held > 0
        assert h.count_total()[0] == oracle.total(g)
    # freed blocks stay in the library's cache (still torch memory) until trimmed
    torch.cuda.synchronize()
    assert bfc.trim_cache() > 0
    assert torch.cuda.memory_allocated() == before


def test_null_allocator_gives_out_of_memory(gpu_lib):
    bfc = gpu_lib
    lib = bfc.load()
    g = gg.workload("uniform-2k-3k-20k")
    e = to_dev(g)
    calls = []
    _fresh_pool(bfc)
    try:
        bfc.set_allocator(lambda n, s: calls.append(n) or None, lambda p, s: None)
        out = ctypes.c_void_p(12345)
        st = lib.bfc_build(ctypes.c_void_p(e.data_ptr()), g.m, g.n_upper, g.n_lower, None, ctypes.byref(out))
        assert st == 5, lib.bfc_last_error()  # BFC_ERR_OUT_OF_MEMORY
        assert out.value is None
        assert b"allocat" in lib.bfc_last_error()
        assert len(calls) >= 2  # the failed request is retried once after trimming
        with pytest.raises(bfc.BfcError) as ei:
            bfc.Graph(e, g.n_upper, g.n_lower)
        assert ei.value.status == 5
    finally:
        bfc.use_torch_allocator()
    # the library works again with memory available
    with bfc.Graph(e, g.n_upper, g.n_lower) as h:
        assert h.count_total()[0] == oracle.total(g)


def test_allocator_that_fails_midway(gpu_lib):
    """A build whose k-th allocation fails returns OUT_OF_MEMORY, leaks nothing
    it allocated before (every block returns to the allocator) and leaves the
    library usable."""
    bfc = gpu_lib
    g = gg.chung_lu(5, 3000, 2000, 40000, 2.1, 2.1, 1000.0)
    e = to_dev(g)
    ref = oracle.total(g)
    for k in (0, 3, 17, 40):
        live = {}
        _fresh_pool(bfc)

        def alloc(n, s):
            if len(live) >= k:
                return None
            p = torch.cuda.caching_allocator_alloc(n, torch.cuda.current_device(), s)
            live[p] = n
            return p

        def free(p, s):
            live.pop(p)
            torch.cuda.caching_allocator_delete(p)

        try:
            bfc.set_allocator(alloc, free)
            try:
                with bfc.Graph(e, g.n_upper, g.n_lower) as h:
                    got = h.count_total()[0]
                assert got == ref
            except bfc.BfcError as err:
                assert err.status == 5
            torch.cuda.synchronize()
            bfc.trim_cache()
            assert not live, f"k={k}: {len(live)} blocks not returned"
        finally:
            bfc.use_torch_allocator()


def test_sync_reports_ok_and_counts_are_exact(gpu_lib):
    bfc = gpu_lib
    g = gg.chung_lu(6, 4000, 3000, 60000, 2.1, 2.1, 1500.0)
    with bfc.Graph(to_dev(g), g.n_upper, g.n_lower) as h:
        s = torch.cuda.Stream()
        up, lo = h.count_per_vertex(stream=s, sync=False)
        be = h.count_per_edge(stream=s, sync=False)
        h.sync(s)
        o_up, o_lo = oracle.vertex_counts(g)
        np.testing.assert_array_equal(up.cpu().numpy(), o_up)
        np.testing.assert_array_equal(lo.cpu().numpy(), o_lo)
        np.testing.assert_array_equal(be.cpu().numpy(), oracle.edge_counts(g))


def test_retune_discards_capture(gpu_lib):
    bfc = gpu_lib
    g = gg.chung_lu(7, 3000, 2500, 50000, 2.1, 2.1, 1200.0)
    ref = oracle.total(g)
    s = torch.cuda.Stream()
    with bfc.Graph(to_dev(g), g.n_upper, g.n_lower, stream=s) as h:
        out = torch.zeros(1, dtype=torch.int64, device="cuda")
        h.capture_total(out, stream=s)
        h.replay(stream=s)
        s.synchronize()
        assert int(out.item()) == ref
        h.set_tuning(light_max_wedges=256)
        with pytest.raises(bfc.BfcError) as ei:
            h.replay(stream=s)
        assert ei.value.status == 1
        h.capture_total(out, stream=s)
        out.zero_()
        h.replay(stream=s)
        s.synchronize()
        assert int(out.item()) == ref
