"""The C-ABI library loads and exports every entry point include/dbfft.h
declares (no GPU needed; no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dbfft.h")
LIB = os.path.join(ROOT, "paper_1905_12725_amd", "libdbfft.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dbfft_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("dbfft_setup", "dbfft_apply", "dbfft_solve", "dbfft_homogenize", "dbfft_adjoint",
                     "dbfft_destroy", "dbfft_last_error"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdbfft.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdbfft.so not built")
def test_binding_names_match_header():
    from paper_1905_12725_amd import _native
    assert sorted(_native.EXPORTED) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdbfft.so not built")
def test_default_opts_and_error_string_without_gpu():
    from paper_1905_12725_amd import _native
    o = _native.default_opts()
    assert o.tol == 1e-8 and o.tol_load == 1e-10 and o.max_iter == 10000
    assert o.newton_tol == 1e-6
    lib = _native.lib()
    assert isinstance(lib.dbfft_last_error(), bytes)
