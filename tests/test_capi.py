"""The C-ABI library loads and exports every symbol include/duplexgs.h declares
(no device calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "duplexgs.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dgs_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("dgs_create", "dgs_destroy", "dgs_reserve", "dgs_render", "dgs_sync", "dgs_get_stats",
                 "dgs_sort_pairs", "dgs_read_lists", "dgs_read_prims"):
        assert want in names


def test_library_exports_every_declared_symbol():
    from paper_2508_03180_amd import _capi
    if not os.path.exists(_capi.LIB_PATH):
        pytest.fail("libduplexgs.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(_capi.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), f"{name} not exported"
    # the binding wraps exactly the declared functions
    assert sorted(_capi.exported_names()) == declared_functions()


def test_struct_layouts_match_header_sizes():
    from paper_2508_03180_amd import _capi
    assert ctypes.sizeof(_capi.dgs_camera) == 16 * 4 + 4 * 4 + 2 * 4 + 4
    assert ctypes.sizeof(_capi.dgs_render_opts) == 4 + 4 + 5 * 4 + 3 * 4 + 4
    assert ctypes.sizeof(_capi.dgs_image) == 4 * 8
    assert ctypes.sizeof(_capi.dgs_grads) == 8 * 8 + 8  # eight pointers, overwrite flag, padding


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2508_03180_amd import _capi
    monkeypatch.setattr(_capi, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_capi, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        _capi.lib()
