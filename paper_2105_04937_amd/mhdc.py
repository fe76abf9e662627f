"""Thin ctypes binding of libmhdc.so (the C-ABI of include/mhdc.h).

Argument marshalling only: every step of conversion and SpMV runs in the HIP
kernels of the library.  torch tensors provide device memory and streams.
If the library has not been built, loading raises RuntimeError; there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmhdc.so")

KIND_MHDC, KIND_HDC, KIND_CSR = 0, 1, 2
ERRORS = {0: "MHDC_OK", -1: "MHDC_ERR_INVALID_ARG", -2: "MHDC_ERR_BAD_CSR", -3: "MHDC_ERR_OOM",
          -4: "MHDC_ERR_HIP", -5: "MHDC_ERR_SIZE", -6: "MHDC_ERR_NOT_SUPPORTED"}


class MhdcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s: %s" % (ERRORS.get(code, code), msg))
        self.code = code
        self.name = ERRORS.get(code, str(code))


class Info(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("n_b", ctypes.c_int32), ("theta", ctypes.c_double), ("n_blk", ctypes.c_int64),
                ("K", ctypes.c_int64), ("S", ctypes.c_int64), ("R", ctypes.c_int64),
                ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
                ("bytes_alg", ctypes.c_double), ("bytes_paper", ctypes.c_double),
                ("rp_est", ctypes.c_double), ("rows_per_lane", ctypes.c_int32),
                ("wg_size", ctypes.c_int32), ("xcd_remap", ctypes.c_int32),
                ("csr_mode", ctypes.c_int32), ("rhs_group", ctypes.c_int32),
                ("row_repeat", ctypes.c_double), ("lone_per_row", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Launch(ctypes.Structure):
    _fields_ = [("rows_per_lane", ctypes.c_int32), ("wg_size", ctypes.c_int32),
                ("xcd_remap", ctypes.c_int32), ("csr_mode", ctypes.c_int32),
                ("rhs_group", ctypes.c_int32)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("wg_size", ctypes.c_int32),
                ("total_tiles", ctypes.c_int64), ("grid", ctypes.c_int32),
                ("flops", ctypes.c_double), ("bytes_alg", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class TuneResult(ctypes.Structure):
    _fields_ = [("n_b", ctypes.c_int32), ("launch", Launch), ("us", ctypes.c_float),
                ("tried", ctypes.c_int32)]


class SelectResult(ctypes.Structure):
    _fields_ = [("theta", ctypes.c_double), ("n_b", ctypes.c_int32),
                ("used_rule", ctypes.c_int32), ("theta_net", ctypes.c_double),
                ("n_b_net", ctypes.c_int32), ("net_ok", ctypes.c_int32),
                ("bytes_net", ctypes.c_double), ("bytes_rule", ctypes.c_double),
                ("rp_est", ctypes.c_double), ("alpha", ctypes.c_double),
                ("beta", ctypes.c_double), ("csr_cheaper", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


MLP_PARAMS = 25346
MLP_SCORER_PARAMS = 30248  # the 40-output scorer (one output per grid point)
MLP_IN = 66
GRID_POINTS = 40  # theta 0.5 .. 0.9 x n_b 32 .. 4096


_lib = None
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_f64 = ctypes.c_double

# name -> (restype, argtypes); every exported symbol of include/mhdc.h
SIGNATURES = {
    "mhdc_last_error": (ctypes.c_int, []),
    "mhdc_last_error_message": (ctypes.c_char_p, []),
    "mhdc_error_string": (ctypes.c_char_p, [ctypes.c_int]),
    "mhdc_from_csr": (_vp, [_i32, _vp, _vp, _vp, _i32, _f64]),
    "mhdc_spmv": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "mhdc_spmm": (ctypes.c_int, [_vp, _vp, _i64, _vp, _i64, _i32, _vp]),
    "mhdc_spmm_rowmajor": (ctypes.c_int, [_vp, _vp, _i64, _vp, _i64, _i32, _vp]),
    "mhdc_spmm_ws": (ctypes.c_int, [_vp, _vp, _i64, _vp, _i64, _i32, _i32, _vp, ctypes.c_size_t, _vp]),
    "mhdc_spmm_workspace_bytes": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(ctypes.c_size_t)]),
    "mhdc_spmm_ws_route": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(_i32)]),
    "mhdc_to_csr": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "mhdc_export": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "mhdc_get_info": (ctypes.c_int, [_vp, ctypes.POINTER(Info)]),
    "mhdc_set_launch": (ctypes.c_int, [_vp, ctypes.POINTER(Launch)]),
    "mhdc_destroy": (None, [_vp]),
    "hdc_from_csr": (_vp, [_i32, _vp, _vp, _vp, _f64]),
    "hdc_spmv": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "hdc_spmv_unblocked": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "hdc_spmm": (ctypes.c_int, [_vp, _vp, _i64, _vp, _i64, _i32, _vp]),
    "hdc_spmm_rowmajor": (ctypes.c_int, [_vp, _vp, _i64, _vp, _i64, _i32, _vp]),
    "hdc_spmm_ws": (ctypes.c_int, [_vp, _vp, _i64, _vp, _i64, _i32, _i32, _vp, ctypes.c_size_t, _vp]),
    "hdc_spmm_workspace_bytes": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(ctypes.c_size_t)]),
    "hdc_spmm_ws_route": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(_i32)]),
    "hdc_export": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "hdc_get_info": (ctypes.c_int, [_vp, ctypes.POINTER(Info)]),
    "hdc_set_launch": (ctypes.c_int, [_vp, ctypes.POINTER(Launch)]),
    "hdc_destroy": (None, [_vp]),
    "csr_from_csr": (_vp, [_i32, _vp, _vp, _vp]),
    "csr_spmv": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "csr_spmm": (ctypes.c_int, [_vp, _vp, _i64, _vp, _i64, _i32, _vp]),
    "csr_spmm_rowmajor": (ctypes.c_int, [_vp, _vp, _i64, _vp, _i64, _i32, _vp]),
    "csr_spmm_ws": (ctypes.c_int, [_vp, _vp, _i64, _vp, _i64, _i32, _i32, _vp, ctypes.c_size_t, _vp]),
    "csr_spmm_workspace_bytes": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(ctypes.c_size_t)]),
    "csr_spmm_ws_route": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(_i32)]),
    "csr_get_info": (ctypes.c_int, [_vp, ctypes.POINTER(Info)]),
    "csr_set_launch": (ctypes.c_int, [_vp, ctypes.POINTER(Launch)]),
    "csr_destroy": (None, [_vp]),
    "mhdc_stream_direct": (ctypes.c_int, [_i64, _vp, _vp, _vp, _vp]),
    "mhdc_stream_indirect": (ctypes.c_int, [_i64, _vp, _vp, _vp, _vp, _vp]),
    "mhdc_debug_fail_alloc": (ctypes.c_int, [_i32]),
    "mhdc_batch_create": (_vp, [_i32, _vp, _vp, _vp, _vp, _vp, _vp, _i32]),
    "mhdc_batch_create_rowmajor": (_vp, [_i32, _vp, _vp, _vp, _vp, _vp, _vp, _i32]),
    "mhdc_batch_bind": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "mhdc_batch_run": (ctypes.c_int, [_vp, _vp]),
    "mhdc_batch_graph_launch": (ctypes.c_int, [_vp, _vp]),
    "mhdc_batch_set_wg": (ctypes.c_int, [_vp, _i32]),
    "mhdc_batch_get_info": (ctypes.c_int, [_vp, ctypes.POINTER(BatchInfo)]),
    "mhdc_batch_destroy": (None, [_vp]),
    "mhdc_autotune": (_vp, [_i32, _vp, _vp, _vp, _f64, _i32, _vp, _i32, _vp,
                            ctypes.POINTER(TuneResult)]),
    "mhdc_batch_tune": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(_i32),
                                       ctypes.POINTER(ctypes.c_float)]),
    "mhdc_features": (ctypes.c_int, [_i32, _vp, _vp, _vp, _vp, _vp]),
    "mhdc_mlp_create": (_vp, [_vp]),
    "mhdc_mlp_create_scorer": (_vp, [_vp]),
    "mhdc_mlp_outputs": (_i32, [_vp]),
    "mhdc_mlp_get_params": (ctypes.c_int, [_vp, _vp]),
    "mhdc_mlp_forward": (ctypes.c_int, [_vp, _vp, _i32, _vp, _vp]),
    "mhdc_mlp_forward_noalloc": (ctypes.c_int, [_vp, _vp, _i32, _vp, _vp]),
    "mhdc_mlp_loss_grad": (ctypes.c_int, [_vp, _vp, _vp, _i32, ctypes.c_float, ctypes.c_float,
                                          _vp, _vp, _vp]),
    "mhdc_mlp_train": (ctypes.c_int, [_vp, _vp, _vp, _i32, _vp, _i64, _i32, ctypes.c_float,
                                      ctypes.c_float, ctypes.c_float, _vp, _vp]),
    "mhdc_mlp_grid_loss_grad": (ctypes.c_int, [_vp, _vp, _vp, _i32, _vp, _vp, _vp]),
    "mhdc_mlp_train_grid": (ctypes.c_int, [_vp, _vp, _vp, _i32, _vp, _i64, _i32,
                                           ctypes.c_float, _vp, _vp]),
    "mhdc_mlp_decide": (ctypes.c_int, [_vp, _vp, _i32, _vp, _vp, _vp, _vp]),
    "mhdc_mlp_destroy": (None, [_vp]),
    "mhdc_time_spmv": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.POINTER(ctypes.c_float)]),
    "mhdc_select": (_vp, [_i32, _vp, _vp, _vp, _vp, _f64, ctypes.POINTER(SelectResult)]),
    "mhdc_judge_keep": (ctypes.c_int, [_f64, _f64, _f64]),
    "mhdc_refine_candidates": (_i32, [_f64, _i32, _vp, _vp, _i32]),
    "mhdc_select_refine": (_vp, [_i32, _vp, _vp, _vp, _vp, _f64, _vp,
                                 ctypes.POINTER(SelectResult)]),
}


def lib():
    """Load libmhdc.so once; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmhdc.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _raise(code=None):
    L = lib()
    c = L.mhdc_last_error() if code is None else code
    raise MhdcError(c, (L.mhdc_last_error_message() or b"").decode())


def _check(rc):
    if rc != 0:
        _raise(rc)


def _dptr(t, dtype, name):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _rows_dense(t):
    """The k values of each row of an (n, k) view are adjacent (stride 1 along
    the row; any stride when k = 1) and rows are at least k apart."""
    k = t.shape[1]
    return (k == 1 or t.stride(1) == 1) and (t.shape[0] <= 1 or t.stride(0) >= k)


class _Matrix:
    _prefix = ""
    kind = -1

    def __init__(self, handle, n):
        self._h = handle
        self.n = n

    def _fn(self, suffix):
        return getattr(lib(), self._prefix + suffix)

    def info(self) -> dict:
        out = Info()
        _check(self._fn("get_info")(self._h, ctypes.byref(out)))
        return out.as_dict()

    def set_launch(self, rows_per_lane=2, wg_size=256, xcd_remap=0, csr_mode=0, rhs_group=0):
        cfg = Launch(rows_per_lane, wg_size, xcd_remap, csr_mode, rhs_group)
        _check(self._fn("set_launch")(self._h, ctypes.byref(cfg)))
        return self

    def spmv(self, x, y=None, stream=None):
        """y = A x (overwrites y); x, y float64 device vectors of length n."""
        if x.numel() != self.n:
            raise ValueError("x has %d entries, expected %d" % (x.numel(), self.n))
        if y is None:
            y = torch.empty(self.n, dtype=torch.float64, device=x.device)
        if y.numel() != self.n:
            raise ValueError("y has %d entries, expected %d" % (y.numel(), self.n))
        _check(self._fn("spmv")(self._h, _dptr(x, torch.float64, "x"),
                                _dptr(y, torch.float64, "y"), _stream(stream)))
        return y

    def time_spmv(self, x, y, stream=None):
        """Mean microseconds per spmv, timed from C with HIP events (M-HDC)."""
        if self.kind != KIND_MHDC:
            raise TypeError("time_spmv takes an M-HDC handle")
        if x.numel() != self.n or y.numel() != self.n:
            raise ValueError("x and y must hold %d entries" % self.n)
        us = ctypes.c_float(0)
        _check(lib().mhdc_time_spmv(self._h, _dptr(x, torch.float64, "x"),
                                    _dptr(y, torch.float64, "y"), _stream(stream), ctypes.byref(us)))
        return us.value

    def spmm(self, X, Y=None, stream=None):
        """Y = A X for k right-hand sides given as rows of X, shape (k, n)
        contiguous (column-major (n, k) in the C-ABI, ldx = n)."""
        if X.dim() != 2 or X.shape[1] != self.n:
            raise ValueError("X must have shape (k, n)")
        k = X.shape[0]
        if Y is None:
            Y = torch.empty((k, self.n), dtype=torch.float64, device=X.device)
        if tuple(Y.shape) != (k, self.n):
            raise ValueError("Y must have shape (%d, %d)" % (k, self.n))
        _check(self._fn("spmm")(self._h, _dptr(X, torch.float64, "X"), self.n,
                                _dptr(Y, torch.float64, "Y"), self.n, k, _stream(stream)))
        return Y

    def workspace_bytes(self, k):
        """Bytes of the workspace spmm_ws needs for k right-hand sides."""
        out = ctypes.c_size_t(0)
        _check(self._fn("spmm_workspace_bytes")(self._h, k, ctypes.byref(out)))
        return out.value

    def ws_route(self, k):
        """The route spmm_ws takes by default for k right-hand sides: 1 =
        the column-major kernel, 2 = through the row-major kernel."""
        out = _i32(0)
        _check(self._fn("spmm_ws_route")(self._h, k, ctypes.byref(out)))
        return out.value

    def spmm_ws(self, X, Y=None, route=0, ws=None, stream=None):
        """spmm with a workspace (C-ABI *_spmm_ws): same shapes and bits as
        spmm; route 0 = the library's choice, 1 = column-major kernel,
        2 = transposed through the row-major kernel.  ws: a device tensor of
        at least workspace_bytes(k) bytes (allocated here when None)."""
        if X.dim() != 2 or X.shape[1] != self.n:
            raise ValueError("X must have shape (k, n)")
        k = X.shape[0]
        if Y is None:
            Y = torch.empty((k, self.n), dtype=torch.float64, device=X.device)
        if tuple(Y.shape) != (k, self.n):
            raise ValueError("Y must have shape (%d, %d)" % (k, self.n))
        if ws is None:
            ws = torch.empty(self.workspace_bytes(k), dtype=torch.uint8, device=X.device)
        if not ws.is_cuda or not ws.is_contiguous():
            raise ValueError("ws must be a contiguous device tensor")
        _check(self._fn("spmm_ws")(self._h, _dptr(X, torch.float64, "X"), self.n,
                                   _dptr(Y, torch.float64, "Y"), self.n, k, route,
                                   ctypes.c_void_p(ws.data_ptr()),
                                   ws.numel() * ws.element_size(), _stream(stream)))
        return Y

    def spmm_rowmajor(self, X, Y=None, stream=None):
        """Y = A X for k right-hand sides stored row by row: X of shape
        (n, ldx) with the k columns first (ldx >= k; a view X[:, :k] of a
        wider row-major array is allowed), Y likewise (allocated (n, k) when
        None)."""
        if X.dim() != 2 or X.shape[0] != self.n or not _rows_dense(X):
            raise ValueError("X must be an (n, k) row-major view")
        k = X.shape[1]
        ldx = X.stride(0) if self.n > 1 else k
        if Y is None:
            Y = torch.empty((self.n, k), dtype=torch.float64, device=X.device)
        if tuple(Y.shape) != (self.n, k) or not _rows_dense(Y):
            raise ValueError("Y must be an (%d, %d) row-major view" % (self.n, k))
        ldy = Y.stride(0) if self.n > 1 else k
        for t, name in ((X, "X"), (Y, "Y")):
            if t.dtype != torch.float64 or not t.is_cuda:
                raise ValueError("%s must be a float64 device tensor" % name)
        _check(self._fn("spmm_rowmajor")(self._h, ctypes.c_void_p(X.data_ptr()), ldx,
                                         ctypes.c_void_p(Y.data_ptr()), ldy, k, _stream(stream)))
        return Y

    def close(self):
        if self._h:
            self._fn("destroy")(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def _csr_args(rowptr, colind, val):
    # conversion runs on the null stream; make torch's producers finish first
    torch.cuda.current_stream().synchronize()
    n = rowptr.numel() - 1
    return (n, _dptr(rowptr, torch.int32, "rowptr"), _dptr(colind, torch.int32, "colind"),
            _dptr(val, torch.float64, "val"))


class MHDCMatrix(_Matrix):
    """M-HDC handle (Sec. 4.3 of the paper): per-block partial diagonals with
    N~(d,ib)/rows_ib >= theta as n_b-long segments, the rest as CSR."""
    _prefix = "mhdc_"
    kind = KIND_MHDC

    @classmethod
    def from_csr(cls, rowptr, colind, val, n_b: int, theta: float):
        n, rp, ci, v = _csr_args(rowptr, colind, val)
        h = lib().mhdc_from_csr(n, rp, ci, v, int(n_b), float(theta))
        if not h:
            _raise()
        return cls(h, n)

    def export(self):
        """Device copies of dia_ptr, dia_off, dia_val, rem_ptr, rem_col, rem_val."""
        inf = self.info()
        dev = torch.device("cuda")
        t = dict(dia_ptr=torch.empty(inf["n_blk"] + 1, dtype=torch.int32, device=dev),
                 dia_off=torch.empty(inf["K"], dtype=torch.int32, device=dev),
                 dia_val=torch.empty(inf["S"], dtype=torch.float64, device=dev),
                 rem_ptr=torch.empty(inf["n"] + 1, dtype=torch.int32, device=dev),
                 rem_col=torch.empty(inf["R"], dtype=torch.int32, device=dev),
                 rem_val=torch.empty(inf["R"], dtype=torch.float64, device=dev))
        torch.cuda.synchronize()
        _check(lib().mhdc_export(self._h, *[_dptr(t[k], t[k].dtype, k) for k in
                                            ("dia_ptr", "dia_off", "dia_val", "rem_ptr",
                                             "rem_col", "rem_val")]))
        return t

    def to_csr(self):
        """Decode on the device back to (rowptr, colind, val)."""
        inf = self.info()
        dev = torch.device("cuda")
        rp = torch.empty(inf["n"] + 1, dtype=torch.int32, device=dev)
        ci = torch.empty(inf["nnz"], dtype=torch.int32, device=dev)
        v = torch.empty(inf["nnz"], dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        _check(lib().mhdc_to_csr(self._h, _dptr(rp, torch.int32, "rowptr"),
                                 _dptr(ci, torch.int32, "colind"), _dptr(v, torch.float64, "val")))
        return rp, ci, v


class HDCMatrix(_Matrix):
    """HDC handle (Sec. 3.4): global diagonals with N(d)/n >= theta plus CSR;
    its kernel is the cache-blocked B-HDC kernel (Sec. 4.2)."""
    _prefix = "hdc_"
    kind = KIND_HDC

    @classmethod
    def from_csr(cls, rowptr, colind, val, theta: float):
        n, rp, ci, v = _csr_args(rowptr, colind, val)
        h = lib().hdc_from_csr(n, rp, ci, v, float(theta))
        if not h:
            _raise()
        return cls(h, n)

    def spmv_unblocked(self, x, y=None, stream=None):
        """y = A x with the unblocked HDC kernel (Fig. 8): the CSR part, then
        one pass over y per diagonal.  Same bits as spmv()."""
        if x.numel() != self.n:
            raise ValueError("x has %d entries, expected %d" % (x.numel(), self.n))
        if y is None:
            y = torch.empty(self.n, dtype=torch.float64, device=x.device)
        if y.numel() != self.n:
            raise ValueError("y has %d entries, expected %d" % (y.numel(), self.n))
        _check(lib().hdc_spmv_unblocked(self._h, _dptr(x, torch.float64, "x"),
                                        _dptr(y, torch.float64, "y"), _stream(stream)))
        return y

    def export(self):
        inf = self.info()
        dev = torch.device("cuda")
        t = dict(dia_off=torch.empty(inf["K"], dtype=torch.int32, device=dev),
                 dia_val=torch.empty(inf["S"], dtype=torch.float64, device=dev),
                 rem_ptr=torch.empty(inf["n"] + 1, dtype=torch.int32, device=dev),
                 rem_col=torch.empty(inf["R"], dtype=torch.int32, device=dev),
                 rem_val=torch.empty(inf["R"], dtype=torch.float64, device=dev))
        torch.cuda.synchronize()
        _check(lib().hdc_export(self._h, *[_dptr(t[k], t[k].dtype, k) for k in
                                           ("dia_off", "dia_val", "rem_ptr", "rem_col",
                                            "rem_val")]))
        return t


class CSRMatrix(_Matrix):
    """Plain CSR baseline handle (Sec. 3.2)."""
    _prefix = "csr_"
    kind = KIND_CSR

    @classmethod
    def from_csr(cls, rowptr, colind, val):
        n, rp, ci, v = _csr_args(rowptr, colind, val)
        h = lib().csr_from_csr(n, rp, ci, v)
        if not h:
            _raise()
        return cls(h, n)


def autotune(rowptr, colind, val, theta: float, nrhs: int = 1,
             nb_candidates=(32, 64, 128, 256, 512), stream=None):
    """Convert for each candidate n_b, time every launch shape, return
    (fastest MHDCMatrix, result dict)."""
    n, rp, ci, v = _csr_args(rowptr, colind, val)
    cands = (ctypes.c_int32 * len(nb_candidates))(*nb_candidates)
    res = TuneResult()
    h = lib().mhdc_autotune(n, rp, ci, v, float(theta), int(nrhs), cands, len(nb_candidates),
                            _stream(stream), ctypes.byref(res))
    if not h:
        _raise()
    out = dict(n_b=res.n_b, us=res.us, tried=res.tried,
               launch=(res.launch.rows_per_lane, res.launch.wg_size, res.launch.xcd_remap,
                       res.launch.csr_mode, res.launch.rhs_group))
    return MHDCMatrix(h, n), out


class Batch:
    """Several M-HDC products Y_i = A_i X_i in one persistent launch.

    mats: MHDCMatrix list; Xs: per item a float64 device tensor of shape
    (k_i, n_i) (rows are right-hand sides; layout "colmajor") or (n_i, k_i)
    (right-hand sides stored row by row; layout "rowmajor"); Ys: outputs of
    the same shapes (allocated when None).  The tensors must stay alive
    while the batch is used."""

    def __init__(self, mats, Xs, Ys=None, wg_size=256, layout="colmajor"):
        if layout not in ("colmajor", "rowmajor"):
            raise ValueError("layout must be colmajor or rowmajor")
        self.rowmajor = layout == "rowmajor"
        self.mats = list(mats)
        self.Xs = list(Xs)
        self.Ys = list(Ys) if Ys is not None else [torch.empty_like(X) for X in self.Xs]
        cnt = len(self.mats)
        hs = (ctypes.c_void_p * cnt)(*[m._h for m in self.mats])
        k = (ctypes.c_int32 * cnt)(*[X.shape[1 if self.rowmajor else 0] for X in self.Xs])
        xp, yp, lx, ly = self._ptrs()
        torch.cuda.synchronize()
        create = lib().mhdc_batch_create_rowmajor if self.rowmajor else lib().mhdc_batch_create
        self._h = create(cnt, hs, k, xp, lx, yp, ly, int(wg_size))
        if not self._h:
            _raise()

    def _ptrs(self):
        cnt = len(self.mats)
        for m, X, Y in zip(self.mats, self.Xs, self.Ys):
            if self.rowmajor:
                if (X.dim() != 2 or X.shape[0] != m.n or Y.shape != X.shape
                        or not _rows_dense(X) or not _rows_dense(Y)):
                    raise ValueError("X_i, Y_i must be (n_i, k_i) row-major views")
                for t, name in ((X, "X"), (Y, "Y")):
                    if t.dtype != torch.float64 or not t.is_cuda:
                        raise ValueError("%s must be a float64 device tensor" % name)
            else:
                if X.dim() != 2 or X.shape[1] != m.n or Y.shape != X.shape:
                    raise ValueError("X_i, Y_i must have shape (k_i, n_i)")
                _dptr(X, torch.float64, "X")
                _dptr(Y, torch.float64, "Y")
        xp = (ctypes.c_void_p * cnt)(*[X.data_ptr() for X in self.Xs])
        yp = (ctypes.c_void_p * cnt)(*[Y.data_ptr() for Y in self.Ys])
        if self.rowmajor:
            lx = (ctypes.c_int64 * cnt)(*[X.stride(0) if m.n > 1 else X.shape[1]
                                          for m, X in zip(self.mats, self.Xs)])
            ly = (ctypes.c_int64 * cnt)(*[Y.stride(0) if m.n > 1 else Y.shape[1]
                                          for m, Y in zip(self.mats, self.Ys)])
        else:
            lx = (ctypes.c_int64 * cnt)(*[m.n for m in self.mats])
            ly = (ctypes.c_int64 * cnt)(*[m.n for m in self.mats])
        return xp, yp, lx, ly

    def bind(self, Xs, Ys):
        old = self.Xs, self.Ys
        self.Xs, self.Ys = list(Xs), list(Ys)
        try:
            xp, yp, lx, ly = self._ptrs()
            _check(lib().mhdc_batch_bind(self._h, xp, lx, yp, ly))
        except Exception:
            self.Xs, self.Ys = old  # the library keeps its previous binding too
            raise

    def run(self, stream=None):
        _check(lib().mhdc_batch_run(self._h, _stream(stream)))
        return self.Ys

    def graph_launch(self, stream=None):
        _check(lib().mhdc_batch_graph_launch(self._h, _stream(stream)))
        return self.Ys

    def set_wg(self, wg_size):
        _check(lib().mhdc_batch_set_wg(self._h, int(wg_size)))

    def tune(self, stream=None):
        wg, us = ctypes.c_int32(0), ctypes.c_float(0)
        _check(lib().mhdc_batch_tune(self._h, _stream(stream), ctypes.byref(wg), ctypes.byref(us)))
        return wg.value, us.value

    def info(self):
        out = BatchInfo()
        _check(lib().mhdc_batch_get_info(self._h, ctypes.byref(out)))
        return out.as_dict()

    def close(self):
        if self._h:
            lib().mhdc_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def features(rowptr, colind, val, stream=None):
    """66 selector features of a device CSR matrix (float32 device tensor)."""
    n, rp, ci, v = _csr_args(rowptr, colind, val)
    f = torch.empty(MLP_IN, dtype=torch.float32, device=rowptr.device)
    _check(lib().mhdc_features(n, rp, ci, v, ctypes.c_void_p(f.data_ptr()), _stream(stream)))
    return f


class MLP:
    """The 66 -> 128 -> 128 -> 2 selector network on the device, or the
    40-output scorer when given MLP_SCORER_PARAMS parameters."""

    def __init__(self, params):
        import numpy as np
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
        if p.size == MLP_PARAMS:
            self._h = lib().mhdc_mlp_create(p.ctypes.data_as(ctypes.c_void_p))
        elif p.size == MLP_SCORER_PARAMS:
            self._h = lib().mhdc_mlp_create_scorer(p.ctypes.data_as(ctypes.c_void_p))
        else:
            raise ValueError("expected %d or %d parameters" % (MLP_PARAMS, MLP_SCORER_PARAMS))
        if not self._h:
            _raise()
        self.outputs = lib().mhdc_mlp_outputs(self._h)
        self.n_params = p.size

    def params(self):
        import numpy as np
        p = np.empty(self.n_params, np.float32)
        _check(lib().mhdc_mlp_get_params(self._h, p.ctypes.data_as(ctypes.c_void_p)))
        return p

    @staticmethod
    def _rows(X):
        if X.dim() != 2 or X.shape[1] != MLP_IN:
            raise ValueError("X must have shape (B, %d)" % MLP_IN)
        return X.shape[0]

    def forward(self, X, stream=None):
        B = self._rows(X)
        out = torch.empty((B, self.outputs), dtype=torch.float32, device=X.device)
        _check(lib().mhdc_mlp_forward(self._h, _dptr(X, torch.float32, "X"), B,
                                      _dptr(out, torch.float32, "out"), _stream(stream)))
        return out

    def forward_noalloc(self, X, out, stream=None):
        """mhdc_mlp_forward_noalloc: the forward pass into a caller-provided
        (B, outputs) float32 output, with no device allocation in the library."""
        B = self._rows(X)
        if tuple(out.shape) != (B, self.outputs):
            raise ValueError("out must have shape (B, %d)" % self.outputs)
        _check(lib().mhdc_mlp_forward_noalloc(self._h, _dptr(X, torch.float32, "X"), B,
                                              _dptr(out, torch.float32, "out"), _stream(stream)))
        return out

    def loss_grad(self, X, T, w=(1.0, 1.0), stream=None):
        if tuple(T.shape) != (self._rows(X), 2):
            raise ValueError("T must have shape (B, 2)")
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
        grad = torch.empty(self.n_params, dtype=torch.float32, device=X.device)
        _check(lib().mhdc_mlp_loss_grad(self._h, _dptr(X, torch.float32, "X"),
                                        _dptr(T, torch.float32, "T"), X.shape[0], float(w[0]),
                                        float(w[1]), _dptr(loss, torch.float32, "loss"),
                                        _dptr(grad, torch.float32, "grad"), _stream(stream)))
        return loss, grad

    def train(self, X, T, order, steps, B, lr, w=(1.0, 1.0), stream=None):
        """Adam over minibatches order[s*B:(s+1)*B] (int32 device tensor)."""
        if tuple(T.shape) != (self._rows(X), 2):
            raise ValueError("T must have shape (N, 2)")
        if order.numel() < int(steps) * int(B):
            raise ValueError("order must hold steps * B row indices")
        hist = torch.empty(int(steps), dtype=torch.float32, device=X.device)
        _check(lib().mhdc_mlp_train(self._h, _dptr(X, torch.float32, "X"),
                                    _dptr(T, torch.float32, "T"), X.shape[0],
                                    _dptr(order, torch.int32, "order"), int(steps), int(B),
                                    float(lr), float(w[0]), float(w[1]),
                                    _dptr(hist, torch.float32, "loss_hist"), _stream(stream)))
        return hist

    def grid_loss_grad(self, X, G, stream=None):
        """mhdc_mlp_grid_loss_grad: G of shape (B, 40), the measured log time
        ratios on the theta x n_b sweep grid (row-major, theta outer)."""
        if tuple(G.shape) != (self._rows(X), GRID_POINTS):
            raise ValueError("G must have shape (B, %d)" % GRID_POINTS)
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
        grad = torch.empty(self.n_params, dtype=torch.float32, device=X.device)
        _check(lib().mhdc_mlp_grid_loss_grad(self._h, _dptr(X, torch.float32, "X"),
                                             _dptr(G, torch.float32, "G"), X.shape[0],
                                             _dptr(loss, torch.float32, "loss"),
                                             _dptr(grad, torch.float32, "grad"),
                                             _stream(stream)))
        return loss, grad

    def train_grid(self, X, G, order, steps, B, lr, stream=None):
        """Adam with the grid loss over minibatches order[s*B:(s+1)*B]."""
        if tuple(G.shape) != (self._rows(X), GRID_POINTS):
            raise ValueError("G must have shape (N, %d)" % GRID_POINTS)
        if order.numel() < int(steps) * int(B):
            raise ValueError("order must hold steps * B row indices")
        hist = torch.empty(int(steps), dtype=torch.float32, device=X.device)
        _check(lib().mhdc_mlp_train_grid(self._h, _dptr(X, torch.float32, "X"),
                                         _dptr(G, torch.float32, "G"), X.shape[0],
                                         _dptr(order, torch.int32, "order"), int(steps),
                                         int(B), float(lr),
                                         _dptr(hist, torch.float32, "loss_hist"),
                                         _stream(stream)))
        return hist

    def decide(self, X, stream=None):
        """(theta, n_b, ok) device tensors for B feature rows."""
        B = self._rows(X)
        th = torch.empty(B, dtype=torch.float64, device=X.device)
        nb = torch.empty(B, dtype=torch.int32, device=X.device)
        ok = torch.empty(B, dtype=torch.int32, device=X.device)
        _check(lib().mhdc_mlp_decide(self._h, _dptr(X, torch.float32, "X"), B,
                                     _dptr(th, torch.float64, "theta"), _dptr(nb, torch.int32, "n_b"),
                                     _dptr(ok, torch.int32, "ok"), _stream(stream)))
        return th, nb, ok

    def close(self):
        if self._h:
            lib().mhdc_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def select(rowptr, colind, val, model=None, tolerance=0.25):
    """Choose (theta, n_b) with the network (None: the policy 0.6 / 256),
    judged by the byte model; returns (MHDCMatrix, result dict)."""
    n, rp, ci, v = _csr_args(rowptr, colind, val)
    res = SelectResult()
    h = lib().mhdc_select(n, rp, ci, v, model._h if model is not None else None,
                          float(tolerance), ctypes.byref(res))
    if not h:
        _raise()
    return MHDCMatrix(h, n), res.as_dict()


def select_refine(rowptr, colind, val, model=None, tolerance=0.25, stream=None):
    """select() followed by timing its choice, the choice's grid neighbours
    and the policy on the device; returns the fastest (MHDCMatrix, dict)."""
    n, rp, ci, v = _csr_args(rowptr, colind, val)
    res = SelectResult()
    h = lib().mhdc_select_refine(n, rp, ci, v, model._h if model is not None else None,
                                 float(tolerance), _stream(stream), ctypes.byref(res))
    if not h:
        _raise()
    return MHDCMatrix(h, n), res.as_dict()


def stream_direct(A, B, C, stream=None):
    """C += A * B elementwise (memory benchmark, Sec. 6.2)."""
    if A.numel() != C.numel() or B.numel() != C.numel():
        raise ValueError("A, B and C must hold the same number of elements")
    _check(lib().mhdc_stream_direct(C.numel(), _dptr(A, torch.float64, "A"),
                                    _dptr(B, torch.float64, "B"), _dptr(C, torch.float64, "C"),
                                    _stream(stream)))
    return C


def stream_indirect(A, B, I, C, stream=None):
    """C += A * B[I] elementwise (memory benchmark, Sec. 6.2)."""
    if A.numel() != C.numel() or B.numel() != C.numel() or I.numel() != C.numel():
        raise ValueError("A, B, I and C must hold the same number of elements")
    _check(lib().mhdc_stream_indirect(C.numel(), _dptr(A, torch.float64, "A"),
                                      _dptr(B, torch.float64, "B"), _dptr(I, torch.int32, "I"),
                                      _dptr(C, torch.float64, "C"), _stream(stream)))
    return C


def to_device(m, device="cuda"):
    """Copy a synth.CSRMatrix to device tensors (rowptr, colind, val)."""
    return (torch.from_numpy(m.rowptr).to(device), torch.from_numpy(m.colind).to(device),
            torch.from_numpy(m.val).to(device))


def judge_keep(v_proposal, v_policy, tolerance):
    """mhdc_judge_keep: the rule by which mhdc_select keeps a proposal."""
    return bool(lib().mhdc_judge_keep(float(v_proposal), float(v_policy), float(tolerance)))


def refine_candidates(theta, n_b):
    """mhdc_refine_candidates: the (theta, n_b) pairs mhdc_select_refine
    times besides the decision."""
    th = (ctypes.c_double * 8)()
    nb = (ctypes.c_int32 * 8)()
    cnt = lib().mhdc_refine_candidates(float(theta), int(n_b), th, nb, 8)
    return [(round(th[i], 1), int(nb[i])) for i in range(cnt)]
