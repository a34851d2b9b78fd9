"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every entry point declared in include/fmm.h, and the host-built operator
tables are consistent with the oracle (checked through the oracle only on the
host side of the test)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fmm.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fmm_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_three_calls():
    names = declared_functions()
    for n in ("fmm_build_tree", "fmm_traverse", "fmm_evaluate", "fmm_create", "fmm_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1108_5815_amd.binding import library_path
    path = library_path()
    if not os.path.exists(path):
        pytest.fail(f"{path} not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    from paper_1108_5815_amd import binding
    src = open(binding.__file__).read()
    for n in declared_functions():
        assert f'"{n}"' in src, n
