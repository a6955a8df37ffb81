"""CPU checks of the C ABI: the built library loads and exports every symbol
that include/stau.h declares; the ctypes declarations match the header."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stau.h")
LIB = os.path.join(ROOT, "paper_1905_10388_amd", "libstau.so")


def header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(stau_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = header_functions()
    for required in ("stau_create_domain", "stau_build_pencils", "stau_factor", "stau_step"):
        assert required in names


LIB_CHECK = os.path.join(ROOT, "paper_1905_10388_amd", "libstau_check.so")


@pytest.mark.parametrize("path", [LIB, LIB_CHECK], ids=["libstau", "libstau_check"])
def test_library_exports_every_declared_symbol(path):
    if not os.path.exists(path):
        pytest.skip(f"{os.path.basename(path)} not built")
    lib = ctypes.CDLL(path)
    missing = [n for n in header_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_ctypes_binding_covers_header():
    from paper_1905_10388_amd import _lib

    assert sorted(_lib.EXPORTS) == header_functions()


def test_struct_layouts_match_header():
    from paper_1905_10388_amd import _lib

    # field order and sizes of the C structs (natural alignment, LP64)
    assert ctypes.sizeof(_lib.DomainDesc) == 4 + 4 + 8 * 3 + 8 * 3 + 4 + 4 + 4 + 4
    assert ctypes.sizeof(_lib.RBParamsC) == 5 * 8 + 8 + 4 * 8
    assert ctypes.sizeof(_lib.StateC) == 8 + 8 + 8 + 8 + 4 + 4
    assert ctypes.sizeof(_lib.InfoC) == 17 * 8
    src = open(HEADER).read()
    info_fields = re.search(r"typedef struct stau_info \{(.*?)\} stau_info;", src, re.S).group(1)
    names = re.findall(r"\b([A-Za-z_][A-Za-z_0-9]*)\s*[,;]", re.sub(r"/\*.*?\*/", "", info_fields))
    assert [f for f, _ in _lib.InfoC._fields_] == [n for n in names if n != "int64_t"]
