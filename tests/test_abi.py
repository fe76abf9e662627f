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


def header_structs():
    """{typedef name: [(field, C type), ...]} of the plain structs the
    header declares (comments stripped, 'int32_t a, b;' expanded)."""
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    out = {}
    for body, name in re.findall(r"typedef struct \{(.*?)\}\s*(\w+)\s*;", src, flags=re.S):
        fields = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            ctype, names = decl.split(None, 1)
            fields += [(f.strip(), ctype) for f in names.split(",")]
        out[name] = fields
    return out


def test_binding_structs_match_header():
    """The ctypes structures of the binding have the header's fields, in
    its order and with the same types, so no layout can drift apart."""
    from paper_2105_04937_amd import mhdc
    ctypes_of = {"int32_t": ctypes.c_int32, "int64_t": ctypes.c_int64,
                 "double": ctypes.c_double, "float": ctypes.c_float,
                 "mhdc_launch": mhdc.Launch}
    pairs = {"mhdc_info": mhdc.Info, "mhdc_launch": mhdc.Launch,
             "mhdc_batch_info": mhdc.BatchInfo, "mhdc_tune_result": mhdc.TuneResult,
             "mhdc_select_result": mhdc.SelectResult}
    structs = header_structs()
    assert set(pairs) <= set(structs), sorted(structs)
    for cname, py in pairs.items():
        want = [(f, ctypes_of[t]) for f, t in structs[cname]]
        assert list(py._fields_) == want, cname


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU; asked for more it says so and exits
    before touching a device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
