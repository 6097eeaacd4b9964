"""The C ABI library loads and exports every entry point declared in
include/tr.h (no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_2011_05427_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "tr.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|size_t|const char \*)\s*(tr_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_entry_points():
    names = declared_symbols()
    assert set(binding.EXPORTS) == set(names), names


@pytest.mark.skipif(not os.path.exists(binding.LIB_PATH), reason="libtr.so not built (run __graft_entry__.build())")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(binding.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(lib, name), name
    lib.tr_error_string.restype = ctypes.c_char_p
    assert lib.tr_error_string(-4).startswith(b"transport iterations")


def test_structs_match_header_field_order():
    src = open(os.path.join(ROOT, "include", "tr.h")).read()
    body = src[src.index("typedef struct tr_state"):]
    body = body[:body.index("} tr_state;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"\*\s*(\w+)", body)
    assert [f for f, _ in binding.TrState._fields_] == fields
