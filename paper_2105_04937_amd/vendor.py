"""rocSPARSE's CSR SpMV (rocsparse_dcsrmv, plain and after
rocsparse_dcsrmv_analysis) through ctypes: the vendor GPU CSR kernel that
stands beside this library's CSR baseline as a point of reference (the
paper compares its CSR kernel with Intel MKL's, Sec. 6.4.4).  It is not part
of the path; nothing in the library calls it."""
from __future__ import annotations

import ctypes
import os

OP_NONE = 111  # rocsparse_operation_none


def library_path() -> str:
    return os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib", "librocsparse.so")


def available() -> bool:
    return os.path.exists(library_path())


class RocSparse:
    """One rocSPARSE handle bound to a torch stream, with a general matrix
    descriptor (zero-based, FP64 values, INT32 indices)."""

    def __init__(self, stream):
        self.L = L = ctypes.CDLL(library_path())
        vp = ctypes.c_void_p
        for name, args in (("rocsparse_create_handle", [ctypes.POINTER(vp)]),
                           ("rocsparse_destroy_handle", [vp]),
                           ("rocsparse_set_stream", [vp, vp]),
                           ("rocsparse_create_mat_descr", [ctypes.POINTER(vp)]),
                           ("rocsparse_destroy_mat_descr", [vp]),
                           ("rocsparse_create_mat_info", [ctypes.POINTER(vp)]),
                           ("rocsparse_destroy_mat_info", [vp]),
                           ("rocsparse_dcsrmv_analysis",
                            [vp, ctypes.c_int, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp,
                             vp, vp, vp, vp]),
                           ("rocsparse_dcsrmv",
                            [vp, ctypes.c_int, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                             ctypes.POINTER(ctypes.c_double), vp, vp, vp, vp, vp, vp,
                             ctypes.POINTER(ctypes.c_double), vp])):
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        self.h = vp()
        self._ok(L.rocsparse_create_handle(ctypes.byref(self.h)), "create_handle")
        self._ok(L.rocsparse_set_stream(self.h, vp(stream.cuda_stream)), "set_stream")
        self.descr = vp()
        self._ok(L.rocsparse_create_mat_descr(ctypes.byref(self.descr)), "create_mat_descr")
        self.one, self.zero = ctypes.c_double(1.0), ctypes.c_double(0.0)

    @staticmethod
    def _ok(rc, what):
        if rc != 0:
            raise RuntimeError("rocsparse %s failed with status %d" % (what, rc))

    def analysis(self, n, nnz, rp, ci, v):
        """rocsparse_dcsrmv_analysis; returns the mat_info to pass to csrmv
        (free it with free_info)."""
        info = ctypes.c_void_p()
        self._ok(self.L.rocsparse_create_mat_info(ctypes.byref(info)), "create_mat_info")
        self._ok(self.L.rocsparse_dcsrmv_analysis(self.h, OP_NONE, n, n, nnz, self.descr,
                                                  v.data_ptr(), rp.data_ptr(), ci.data_ptr(),
                                                  info), "dcsrmv_analysis")
        return info

    def free_info(self, info):
        if info:
            self.L.rocsparse_destroy_mat_info(info)

    def csrmv(self, n, nnz, rp, ci, v, info, x, y):
        """y = A x (alpha 1, beta 0); info = None for the plain kernel."""
        self._ok(self.L.rocsparse_dcsrmv(self.h, OP_NONE, n, n, nnz, ctypes.byref(self.one),
                                         self.descr, v.data_ptr(), rp.data_ptr(), ci.data_ptr(),
                                         info if info else ctypes.c_void_p(None), x.data_ptr(),
                                         ctypes.byref(self.zero), y.data_ptr()), "dcsrmv")

    def close(self):
        if self.descr:
            self.L.rocsparse_destroy_mat_descr(self.descr)
            self.descr = ctypes.c_void_p()
        if self.h:
            self.L.rocsparse_destroy_handle(self.h)
            self.h = ctypes.c_void_p()
