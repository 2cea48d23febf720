"""The C-ABI library loads on a machine without a GPU and exports every
function declared in include/yeerom.h (no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "yeerom.h")
LIB = os.path.join(ROOT, "paper_1406_7042_amd", "_lib", "libyeerom.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^(?:int|void|const char\*)\s+(\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1406_7042_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("fdtd_step", "mor_reduce", "rom_perturb", "rom_step", "rom_lift", "fdtd_adjoint",
              "rom_adjoint",
              "yr_operator_create", "yr_last_error"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_error_path_without_device(lib):
    """A null argument is rejected before any device work, with a message."""
    lib.yr_operator_create.restype = ctypes.c_int
    lib.yr_last_error.restype = ctypes.c_char_p
    st = lib.yr_operator_create(None, None, None)
    assert st == -1
    assert b"null" in lib.yr_last_error()
