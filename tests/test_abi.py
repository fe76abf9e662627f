"""The C-ABI library loads on a machine without a GPU and exports every
function that include/mhdc.h declares; the binding covers them all.  No
compute call is made here."""
import ctypes
import os
import re

import pytest

from tests.conftest import ROOT

HEADER = os.path.join(ROOT, "include", "mhdc.h")
LIB = os.path.join(ROOT, "paper_2105_04937_amd", "libmhdc.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_ ]*?[\s\*]+([a-z_][a-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while", "for", "return")))


def test_header_parses():
    names = declared_functions()
    for must in ("mhdc_from_csr", "mhdc_spmv", "mhdc_spmm", "hdc_from_csr", "hdc_spmv",
                 "csr_from_csr", "csr_spmv", "mhdc_destroy", "mhdc_get_info"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmhdc.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_2105_04937_amd import mhdc
    assert sorted(mhdc.SIGNATURES) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmhdc.so not built")
def test_error_strings_without_gpu():
    from paper_2105_04937_amd import mhdc
    L = mhdc.lib()
    assert L.mhdc_error_string(-2) == b"MHDC_ERR_BAD_CSR"
    assert L.mhdc_last_error() == 0
