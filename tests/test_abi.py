"""The C-ABI library loads and exports every symbol include/fmt.h declares
(no compute calls here: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fmt.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fmt_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("fmt_fit", "fmt_fit_batch", "fmt_eval", "fmt_tree_wait", "fmt_tree_get_info",
              "fmt_tree_export_nodes", "fmt_tree_export_points", "fmt_tree_import", "fmt_refit",
              "fmt_tree_destroy", "fmt_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1511_01353_amd as m
    if not os.path.exists(m.LIB_PATH):
        pytest.skip("libfmt.so not built")
    lib = ctypes.CDLL(m.LIB_PATH)
    for n in declared_functions():
        assert hasattr(lib, n), n
    assert set(declared_functions()) == set(m.EXPORTED)


def test_host_side_calls_without_gpu():
    import paper_1511_01353_amd as m
    if not os.path.exists(m.LIB_PATH):
        pytest.skip("libfmt.so not built")
    o = m.fmt_default_opts()
    assert (o.p, o.max_depth, o.path, o.refine_steps) == (4, 6, 0, 1)
    assert list(o.box_lo) == [0.0, 0.0, 0.0] and list(o.box_hi) == [1.0, 1.0, 1.0]
    assert "gfx950" in m.fmt_version()
    lib = m.load_library()
    # argument validation happens before any device work
    st = lib.fmt_fit(None, None, None, None, None, 0, 0, None, None)
    assert st == m.FMT_E_INVALID_ARG
    assert "NULL" in m.fmt_last_error()
    bad = m.fmt_default_opts(p=99)
    h = ctypes.c_void_p()
    st = lib.fmt_fit(ctypes.byref(bad), None, None, None, None, 100, 0, None, ctypes.byref(h))
    assert st == m.FMT_E_INVALID_ARG and not h.value
    bad = m.fmt_default_opts(tol=-1.0)
    assert lib.fmt_fit(ctypes.byref(bad), None, None, None, None, 100, 0, None, ctypes.byref(h)) == m.FMT_E_INVALID_ARG
    bad = m.fmt_default_opts(box_lo=(0, 0, 1), box_hi=(1, 1, 1))
    assert lib.fmt_fit(ctypes.byref(bad), None, None, None, None, 100, 0, None, ctypes.byref(h)) == m.FMT_E_INVALID_ARG
    ok = m.fmt_default_opts()
    assert lib.fmt_fit(ctypes.byref(ok), None, None, None, None, 100, 7, None, ctypes.byref(h)) == m.FMT_E_INVALID_ARG
    out = (ctypes.c_void_p * 2)()
    assert lib.fmt_refit(None, None, None, None, None, 100, 2, 0, None, out) == m.FMT_E_INVALID_ARG
    assert not out[0] and not out[1]
    lib.fmt_tree_destroy(None)
