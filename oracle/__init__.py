"""CPU oracle for M-HDC SpMV (arXiv:2105.04937) -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never calls it and
shares no code with it; if the HIP library is missing the product raises
instead of falling back here.

The arithmetic lives in ``oracle.c`` (plain C, FP64, built with
``-ffp-contract=off``); this module only marshals numpy arrays through ctypes.
Each wrapper names the passage of the paper it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc into liboracle.so (no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call([
            "gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
            "-shared", "-fPIC", "-std=c11", "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        vp = ctypes.c_void_p
        lib.orc_csr_spmv.argtypes = [_i32, _i32p, _i32p, _f64p, _f64p, _f64p, _i32]
        lib.orc_csr_spmm.argtypes = [_i32, _i32p, _i32p, _f64p, _i32, _f64p, _i64,
                                     _f64p, _i64, _i32]
        lib.orc_csr_absmv.argtypes = [_i32, _i32p, _i32p, _f64p, _f64p, _f64p]
        lib.orc_dense_matvec.argtypes = [_i32, _f64p, _f64p, _f64p]
        lib.orc_mhdc_convert.argtypes = [_i32, _i32p, _i32p, _f64p, _i32, ctypes.c_double,
                                         vp, vp, vp, vp, vp, vp,
                                         ctypes.POINTER(_i64), ctypes.POINTER(_i64)]
        lib.orc_mhdc_convert.restype = ctypes.c_int
        lib.orc_hdc_convert.argtypes = [_i32, _i32p, _i32p, _f64p, ctypes.c_double,
                                        vp, vp, vp, vp, vp,
                                        ctypes.POINTER(_i64), ctypes.POINTER(_i64)]
        lib.orc_hdc_convert.restype = ctypes.c_int
        lib.orc_mhdc_spmv.argtypes = [_i32, _i32, _i32p, _i32p, _f64p, _i32p, _i32p,
                                      _f64p, _f64p, _f64p]
        lib.orc_hdc_spmv.argtypes = [_i32, _i32, _i32p, _f64p, _i32p, _i32p, _f64p,
                                     _f64p, _f64p]
        lib.orc_mhdc_to_csr.argtypes = [_i32, _i32, _i32p, _i32p, _f64p, _i32p, _i32p,
                                        _f64p, _i32p, _i32p, _f64p]
        lib.orc_mhdc_to_csr.restype = ctypes.c_int
        lib.orc_stream_direct.argtypes = [_i64, _f64p, _f64p, _f64p]
        lib.orc_stream_indirect.argtypes = [_i64, _f64p, _f64p, _i32p, _f64p]
        _lib = lib
    return _lib


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


# --------------------------------------------------------------------------
# SpMV definitions
# --------------------------------------------------------------------------
def csr_spmv(rowptr, colind, val, x, nthreads: int = 1) -> np.ndarray:
    """y = A x by the CSR kernel of Sec. 3.2 (Fig. 3): per row, ascending k."""
    rowptr, colind, val, x = _c(rowptr, np.int32), _c(colind, np.int32), _c(val, np.float64), _c(x, np.float64)
    n = rowptr.size - 1
    y = np.empty(n, np.float64)
    _load().orc_csr_spmv(n, rowptr, colind, val, x, y, nthreads)
    return y


def csr_spmm(rowptr, colind, val, X, nthreads: int = 1) -> np.ndarray:
    """Y = A X for an (n, k) block of right-hand sides; each column by Fig. 3."""
    rowptr, colind, val = _c(rowptr, np.int32), _c(colind, np.int32), _c(val, np.float64)
    n = rowptr.size - 1
    Xf = np.asfortranarray(X, dtype=np.float64)
    k = Xf.shape[1]
    Y = np.empty((n, k), np.float64, order="F")
    xf = Xf.reshape(-1, order="F")
    yf = Y.reshape(-1, order="F")
    _load().orc_csr_spmm(n, rowptr, colind, val, k, xf, n, yf, n, nthreads)
    return Y


def csr_absmv(rowptr, colind, val, x) -> np.ndarray:
    """(|A| |x|)_i, the scale of the summation-order error bound."""
    rowptr, colind, val, x = _c(rowptr, np.int32), _c(colind, np.int32), _c(val, np.float64), _c(x, np.float64)
    n = rowptr.size - 1
    y = np.empty(n, np.float64)
    _load().orc_csr_absmv(n, rowptr, colind, val, x, y)
    return y


def dense_matvec(A, x) -> np.ndarray:
    """Brute-force y = A x (Sec. 3.1), ascending column order."""
    A = _c(A, np.float64)
    n = A.shape[0]
    y = np.empty(n, np.float64)
    _load().orc_dense_matvec(n, A.reshape(-1), _c(x, np.float64), y)
    return y


# --------------------------------------------------------------------------
# Formats
# --------------------------------------------------------------------------
@dataclass
class MHDC:
    """Arrays of the M-HDC format (Sec. 4.3, Fig. 15); HDC is the case
    bl = n with a single block (Sec. 3.4, Fig. 7)."""
    n: int
    bl: int
    dia_ptr: np.ndarray
    dia_off: np.ndarray
    dia_val: np.ndarray
    rem_ptr: np.ndarray
    rem_col: np.ndarray
    rem_val: np.ndarray

    @property
    def K(self) -> int:
        return int(self.dia_off.size)

    @property
    def R(self) -> int:
        return int(self.rem_col.size)

    @property
    def n_blk(self) -> int:
        return int(self.dia_ptr.size - 1)


def mhdc_from_csr(rowptr, colind, val, bl: int, theta: float) -> MHDC:
    """Reference M-HDC converter (Sec. 4.3): per block keep partial diagonals
    with N~(d,ib)/rows_ib >= theta, ascending; the rest goes to the remainder."""
    rowptr, colind, val = _c(rowptr, np.int32), _c(colind, np.int32), _c(val, np.float64)
    n = rowptr.size - 1
    lib = _load()
    K, R = _i64(0), _i64(0)
    rc = lib.orc_mhdc_convert(n, rowptr, colind, val, bl, theta,
                              None, None, None, None, None, None,
                              ctypes.byref(K), ctypes.byref(R))
    if rc != 0:
        raise ValueError("oracle mhdc_from_csr failed: %d" % rc)
    n_blk = 0 if n == 0 else (n + bl - 1) // bl
    dia_ptr = np.zeros(n_blk + 1, np.int32)
    dia_off = np.zeros(K.value, np.int32)
    dia_val = np.zeros(K.value * bl, np.float64)
    rem_ptr = np.zeros(n + 1, np.int32)
    rem_col = np.zeros(R.value, np.int32)
    rem_val = np.zeros(R.value, np.float64)
    rc = lib.orc_mhdc_convert(n, rowptr, colind, val, bl, theta,
                              _ptr(dia_ptr), _ptr(dia_off), _ptr(dia_val),
                              _ptr(rem_ptr), _ptr(rem_col), _ptr(rem_val),
                              ctypes.byref(K), ctypes.byref(R))
    if rc != 0:
        raise ValueError("oracle mhdc_from_csr failed: %d" % rc)
    return MHDC(n, bl, dia_ptr, dia_off, dia_val, rem_ptr, rem_col, rem_val)


def hdc_from_csr(rowptr, colind, val, theta: float) -> MHDC:
    """Reference HDC converter (Sec. 3.4): keep diagonal d iff N(d)/n >= theta;
    global DIA dia_val[k*n + i] plus a CSR part.  Returned as an MHDC with one
    block of n rows (dia_ptr = [0, K])."""
    rowptr, colind, val = _c(rowptr, np.int32), _c(colind, np.int32), _c(val, np.float64)
    n = rowptr.size - 1
    lib = _load()
    K, R = _i64(0), _i64(0)
    rc = lib.orc_hdc_convert(n, rowptr, colind, val, theta, None, None, None, None, None,
                             ctypes.byref(K), ctypes.byref(R))
    if rc != 0:
        raise ValueError("oracle hdc_from_csr failed: %d" % rc)
    dia_off = np.zeros(K.value, np.int32)
    dia_val = np.zeros(K.value * n, np.float64)
    rem_ptr = np.zeros(n + 1, np.int32)
    rem_col = np.zeros(R.value, np.int32)
    rem_val = np.zeros(R.value, np.float64)
    rc = lib.orc_hdc_convert(n, rowptr, colind, val, theta, _ptr(dia_off), _ptr(dia_val),
                             _ptr(rem_ptr), _ptr(rem_col), _ptr(rem_val),
                             ctypes.byref(K), ctypes.byref(R))
    if rc != 0:
        raise ValueError("oracle hdc_from_csr failed: %d" % rc)
    dia_ptr = np.array([0, K.value] if n > 0 else [0], np.int32)
    return MHDC(n, max(n, 1), dia_ptr, dia_off, dia_val, rem_ptr, rem_col, rem_val)


def mhdc_spmv(m: MHDC, x) -> np.ndarray:
    """y = A x by the M-HDC kernel of Fig. 16 (remainder first, then the
    block's partial diagonals in ascending k)."""
    y = np.empty(m.n, np.float64)
    _load().orc_mhdc_spmv(m.n, m.bl, m.dia_ptr, m.dia_off, m.dia_val, m.rem_ptr,
                          m.rem_col, m.rem_val, _c(x, np.float64), y)
    return y


def hdc_spmv(m: MHDC, x) -> np.ndarray:
    """y = A x by the HDC kernel of Fig. 8 on a one-block (global DIA) MHDC."""
    y = np.empty(m.n, np.float64)
    _load().orc_hdc_spmv(m.n, m.K, m.dia_off, m.dia_val, m.rem_ptr, m.rem_col,
                         m.rem_val, _c(x, np.float64), y)
    return y


def mhdc_to_csr(m: MHDC):
    """Decode M-HDC back to CSR (merge of nonzero DIA slots and remainder)."""
    nnz = int(np.count_nonzero(m.dia_val)) + m.R
    ptr = np.zeros(m.n + 1, np.int32)
    col = np.zeros(nnz, np.int32)
    val = np.zeros(nnz, np.float64)
    rc = _load().orc_mhdc_to_csr(m.n, m.bl, m.dia_ptr, m.dia_off, m.dia_val, m.rem_ptr,
                                 m.rem_col, m.rem_val, ptr, col, val)
    if rc != 0:
        raise ValueError("oracle mhdc_to_csr failed: %d" % rc)
    e = int(ptr[-1])
    return ptr, col[:e], val[:e]


def stream_direct(A, B, C) -> np.ndarray:
    """C[i] += A[i] * B[i] (Sec. 6.2, Fig. 19)."""
    C = np.array(C, np.float64)
    _load().orc_stream_direct(C.size, _c(A, np.float64), _c(B, np.float64), C)
    return C


def stream_indirect(A, B, I, C) -> np.ndarray:
    """C[i] += A[i] * B[I[i]] (Sec. 6.2, Fig. 20)."""
    C = np.array(C, np.float64)
    _load().orc_stream_indirect(C.size, _c(A, np.float64), _c(B, np.float64),
                                _c(I, np.int32), C)
    return C
