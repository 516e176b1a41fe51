"""Binding of liboz_blas.so (include/oz_blas.h): the Fortran-ABI dgemm_ and
zgemm_ offload layer, with argument marshalling only.  Matrices are numpy
arrays (host memory, column-major storage is read through their buffer) or
device pointers given as integers (e.g. torch's data_ptr()); every product
runs on the GPU.  Raises ImportError when the library is not built."""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
BLAS_LIB_PATH = os.path.join(_HERE, "liboz_blas.so")
if not os.path.exists(BLAS_LIB_PATH):
    raise ImportError("liboz_blas.so is not built (%s); run __graft_entry__.build() first" % BLAS_LIB_PATH)
_lib = ctypes.CDLL(BLAS_LIB_PATH)

EXPORTS = ["dgemm_", "zgemm_", "oz_blas_set_mode", "oz_blas_stats", "oz_blas_finalize"]


class oz_blas_stats_t(ctypes.Structure):
    _fields_ = [("calls", ctypes.c_int64), ("bytes_to_device", ctypes.c_int64), ("bytes_to_host", ctypes.c_int64),
                ("copy_ms", ctypes.c_double), ("compute_ms", ctypes.c_double), ("last_info", ctypes.c_int32),
                ("last_slices", ctypes.c_int32), ("mode", ctypes.c_int32), ("slices", ctypes.c_int32),
                ("tol", ctypes.c_double)]


_P = ctypes.c_void_p
_I = ctypes.POINTER(ctypes.c_int32)
for _name in ("dgemm_", "zgemm_"):
    getattr(_lib, _name).argtypes = [ctypes.c_char_p, ctypes.c_char_p, _I, _I, _I, _P, _P, _I, _P, _I, _P, _P, _I]
    getattr(_lib, _name).restype = None
_lib.oz_blas_set_mode.argtypes = [ctypes.c_char_p]
_lib.oz_blas_set_mode.restype = ctypes.c_int
_lib.oz_blas_stats.argtypes = [ctypes.POINTER(oz_blas_stats_t)]
_lib.oz_blas_stats.restype = None
_lib.oz_blas_finalize.argtypes = []
_lib.oz_blas_finalize.restype = None


def _ptr(x):
    if isinstance(x, np.ndarray):
        return ctypes.c_void_p(x.ctypes.data)
    if x is None:
        return ctypes.c_void_p(0)
    if hasattr(x, "data_ptr"):
        return ctypes.c_void_p(x.data_ptr())
    return ctypes.c_void_p(int(x))


def _int(v):
    return ctypes.byref(ctypes.c_int32(int(v)))


def _gemm(fn, cplx, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc):
    dt = np.complex128 if cplx else np.float64
    al = np.array([alpha], dtype=dt)
    be = np.array([beta], dtype=dt)
    fn(transa.encode()[:1], transb.encode()[:1], _int(m), _int(n), _int(k), _ptr(al), _ptr(A), _int(lda), _ptr(B),
       _int(ldb), _ptr(be), _ptr(C), _int(ldc))


def dgemm_(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc):
    """C <- alpha op(A) op(B) + beta C in place (C a Fortran-ordered float64 array or a device pointer)."""
    _gemm(_lib.dgemm_, False, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc)


def zgemm_(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc):
    """The complex128 form of dgemm_."""
    _gemm(_lib.zgemm_, True, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc)


def oz_blas_set_mode(mode):
    """'fp64_int8_<s>', 'fp64_int8_bal<s>', 'fp64_int8_tol<tol>' or 'dgemm'; False when not a mode."""
    return _lib.oz_blas_set_mode(mode.encode()) == 0


def oz_blas_stats():
    st = oz_blas_stats_t()
    _lib.oz_blas_stats(ctypes.byref(st))
    return st


def oz_blas_finalize():
    _lib.oz_blas_finalize()
