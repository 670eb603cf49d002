"""The C-ABI library loads and exports what include/bfc.h declares (no GPU needed).

Only host-side entry points are called here: argument validation happens
before any HIP call, so these run without a device.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bfc.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bfc_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1812_00283_amd import bfc, build

    if not os.path.exists(bfc.LIB_PATH):
        build.build()
    return bfc.load()


def test_header_declares_the_four_calls():
    names = header_functions()
    for required in ("bfc_build", "bfc_count_total", "bfc_count_per_vertex", "bfc_count_per_edge"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    raw = ctypes.CDLL(lib._name)
    for name in header_functions():
        assert hasattr(raw, name), name


def test_binding_covers_the_header():
    from paper_1812_00283_amd import bfc

    assert sorted(bfc.EXPORTS) == header_functions()


def test_host_side_calls(lib):
    from paper_1812_00283_amd import bfc

    assert "gfx950" in bfc.version()
    assert bfc.estimate_device_bytes(1000, 10, 20) > 1000 * 20
    assert bfc.estimate_device_bytes(-1, 1, 1) == 0


def test_argument_errors_need_no_device(lib):
    from paper_1812_00283_amd import bfc

    vp = ctypes.c_void_p
    out = vp()
    t = ctypes.c_int64()
    assert lib.bfc_count_total(None, None, ctypes.byref(t), None) == 1
    assert lib.bfc_count_per_edge(None, None, None) == 1
    assert lib.bfc_count_per_vertex(None, None, None, None) == 1
    assert lib.bfc_destroy(None) == 0
    assert lib.bfc_build(None, 10, 5, 5, None, None) == 1          # out is null
    assert lib.bfc_build(None, -1, 5, 5, None, ctypes.byref(out)) == 1
    assert lib.bfc_build(None, 10, 5, 5, None, ctypes.byref(out)) == 1   # null edges
    assert lib.bfc_build(vp(8), 1 << 30, 1 << 20, 1 << 20, None, ctypes.byref(out)) == 4
    assert lib.bfc_build(vp(8), 26, 5, 5, None, ctypes.byref(out)) == 3  # more edges than pairs
    assert out.value is None
    assert b"pairs" in lib.bfc_last_error()
    tun = bfc.Tuning()
    assert lib.bfc_set_tuning(None, ctypes.byref(tun)) == 1
    # the later entry points check their arguments before any device work
    c = ctypes.c_int64()
    d = ctypes.c_double()
    assert lib.bfc_caterpillars(None, ctypes.byref(c)) == 1
    assert lib.bfc_clustering_coefficient(None, None, ctypes.byref(d)) == 1
    assert lib.bfc_count_total_sorted(None, None, 0, 0, ctypes.byref(t), None, None) == 1
    w, r = ctypes.c_int64(), ctypes.c_int32()
    assert lib.bfc_k_wing(vp(8), 10, 5, 5, 1, None, None, None, ctypes.byref(w), ctypes.byref(r)) == 1  # null mask
    assert lib.bfc_k_wing(vp(8), 1 << 30, 1 << 20, 1 << 20, 1, None, vp(8), None, ctypes.byref(w), ctypes.byref(r)) == 4
    assert lib.bfc_k_wing(vp(8), 26, 5, 5, 1, None, vp(8), None, ctypes.byref(w), ctypes.byref(r)) == 3
