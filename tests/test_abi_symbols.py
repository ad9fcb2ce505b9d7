"""CPU-side checks of the built library: it loads without a GPU and exports
every function include/fdas.h declares (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fdas.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fdas_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1805_12280_amd import fdas
    if not os.path.exists(fdas.LIB_PATH):
        from paper_1805_12280_amd import build
        build.build()
    return ctypes.CDLL(fdas.LIB_PATH)


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("fdas_plan_create", "fdas_convolve", "fdas_tdfir", "fdas_plan_info",
              "fdas_plan_destroy", "fdas_strerror", "fdas_last_error"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    from paper_1805_12280_amd import fdas
    names = declared_functions()
    assert set(names) == set(fdas.EXPORTED)
    for n in names:
        assert hasattr(lib, n), n


def test_strerror_is_host_only(lib):
    lib.fdas_strerror.restype = ctypes.c_char_p
    assert lib.fdas_strerror(0) == b"ok"
    assert lib.fdas_strerror(1) == b"invalid argument"
    assert lib.fdas_strerror(99) == b"unknown status"


def test_missing_library_fails_loudly(tmp_path):
    from paper_1805_12280_amd import fdas
    with pytest.raises(fdas.FdasError):
        fdas.load_library(str(tmp_path / "libfdas.so"))
