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
    assert ctypes.sizeof(gts._BuildOpts) == 48
    assert ctypes.sizeof(gts._QueryOpts) == 24
    assert ctypes.sizeof(gts._Result) == 64
    assert ctypes.sizeof(gts._Stats) == 7 * 8 + 8 + 64 + 11 * 8


def test_struct_layouts_match_the_c_compiler(tmp_path):
    """Every ctypes mirror has the size and field offsets that a C compiler
    gives the header's struct (gcc on the header itself)."""
    import shutil
    import subprocess

    from paper_2404_00966_amd import gts

    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    structs = {"gts_objects": gts._Objects, "gts_build_opts": gts._BuildOpts, "gts_query_opts": gts._QueryOpts,
               "gts_result": gts._Result, "gts_stats": gts._Stats, "gts_index_info": gts._Info,
               "gts_request": gts._Request, "gts_completion": gts._Completion,
               "gts_server_opts": gts._ServerOpts, "gts_server_stats": gts._ServerStats,
               "gts_plan_io": gts._PlanIO}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "gts.h"', "int main(void) {"]
    expect = []
    for cname, cls in structs.items():
        lines.append(f'printf("%zu\\n", sizeof({cname}));')
        expect.append(ctypes.sizeof(cls))
        for f, _ in cls._fields_:
            lines.append(f'printf("%zu\\n", offsetof({cname}, {f}));')
            expect.append(getattr(cls, f).offset)
    lines += ["return 0; }"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert got == expect
