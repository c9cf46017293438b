"""The C ABI library loads and exports every function include/gts.h declares
(no compute call: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gts.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gts_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("gts_build_index", "gts_range_query", "gts_knn_query", "gts_search", "gts_insert",
                     "gts_delete", "gts_result_free", "gts_destroy", "gts_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2404_00966_amd import gts

    if not os.path.exists(gts.LIB_PATH):
        pytest.skip("libgts.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(gts.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(gts.EXPORTS) == set(declared_functions())


def test_last_error_is_empty_string_initially():
    from paper_2404_00966_amd import gts

    if not os.path.exists(gts.LIB_PATH):
        pytest.skip("libgts.so not built")
    lib = gts.library()
    assert lib.gts_last_error() == b""


def test_struct_layouts_match_header_sizes():
    from paper_2404_00966_amd import gts

    # sizes follow from the header's field lists (natural alignment, x86-64)
    assert ctypes.sizeof(gts._Objects) == 40
    assert ctypes.sizeof(gts._BuildOpts) == 32
    assert ctypes.sizeof(gts._QueryOpts) == 16
    assert ctypes.sizeof(gts._Result) == 64
    assert ctypes.sizeof(gts._Stats) == 7 * 8 + 8 + 64 + 8
