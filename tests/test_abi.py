"""The C-ABI library loads and exports every entry point that include/spmv.h
declares (CPU only: no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spmv.h")
LIB = os.path.join(ROOT, "paper_1805_11938_amd", "libspmv.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(spmv_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1805_11938_amd import build
        build.build_spmv()
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert len(names) >= 30
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_1805_11938_amd import spmv
    assert sorted(spmv.EXPORTED) == declared()


def test_status_strings(lib):
    lib.spmv_status_str.restype = ctypes.c_char_p
    lib.spmv_status_str.argtypes = [ctypes.c_int]
    assert lib.spmv_status_str(0) == b"ok"
    assert lib.spmv_status_str(-4) == b"too large"
    assert lib.spmv_status_str(-7) == b"model error"


def test_no_oracle_in_product():
    """The product package never imports or links the oracle."""
    pkg = os.path.join(ROOT, "paper_1805_11938_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h", ".c")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src and "liboracle" not in src, f
