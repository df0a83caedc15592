"""The C-ABI library loads and exports every entry point its header declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bs32.h")
LIB = os.path.join(ROOT, "paper_2605_23727_amd", "libbs32.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bs32_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def built_lib():
    if not os.path.exists(LIB):
        from paper_2605_23727_amd.build import build
        build()
    return ctypes.CDLL(LIB)


def test_header_declares_core_calls():
    names = declared()
    for core in ("bs32_create", "bs32_set_system", "bs32_solve", "bs32_stats", "bs32_destroy"):
        assert core in names


def test_every_declared_symbol_is_exported(built_lib):
    for name in declared():
        assert hasattr(built_lib, name), name


def test_binding_covers_header():
    import paper_2605_23727_amd as b
    assert sorted(b.exported_symbols()) == declared()
