"""Oracle: ctypes binding of qsw_oracle.c (built with gcc).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this file.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qsw_oracle.c")
_OUT_DIR = os.path.join(_HERE, "_build")
_LIB = os.path.join(_OUT_DIR, "liboracle.so")

_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile the oracle library with gcc (OpenMP over rows)."""
    os.makedirs(_OUT_DIR, exist_ok=True)
    if force or not os.path.exists(_LIB):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-std=c11", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        L.oracle_superop_csr.restype = ctypes.c_int64
        L.oracle_superop_csr.argtypes = [
            ctypes.c_int64, _i64p, _i32p, _f64p, _i64p, _i32p, _f64p,
            ctypes.c_double, _i64p, ctypes.c_void_p, ctypes.c_void_p]
        L.oracle_norm1.restype = ctypes.c_double
        L.oracle_norm1.argtypes = [ctypes.c_int64, _i64p, _i32p, _f64p]
        L.oracle_spmv.restype = None
        L.oracle_spmv.argtypes = [ctypes.c_int64, _i64p, _i32p, _f64p, _f64p, _f64p]
        L.oracle_taylor_expmv.restype = ctypes.c_int64
        L.oracle_taylor_expmv.argtypes = [
            ctypes.c_int64, _i64p, _i32p, _f64p, _f64p, ctypes.c_double,
            ctypes.c_int32, ctypes.c_int32, ctypes.c_double, _f64p]
        _lib = L
    return _lib


def _ri(z: np.ndarray) -> np.ndarray:
    """complex128 array -> contiguous float64 view (re, im interleaved)."""
    z = np.ascontiguousarray(z, dtype=np.complex128)
    return z.view(np.float64)


class CSR:
    """Row-major CSR with int64 row_ptr, int32 col, complex128 val."""

    def __init__(self, n, row_ptr, col, val):
        self.n = int(n)
        self.row_ptr = np.ascontiguousarray(row_ptr, np.int64)
        self.col = np.ascontiguousarray(col, np.int32)
        self.val = np.ascontiguousarray(val, np.complex128)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def matvec(self, x: np.ndarray) -> np.ndarray:
        y = np.empty(self.n, np.complex128)
        lib().oracle_spmv(self.n, self.row_ptr, self.col, _ri(self.val), _ri(x),
                          y.view(np.float64))
        return y

    def norm1(self) -> float:
        return float(lib().oracle_norm1(self.n, self.row_ptr, self.col, _ri(self.val)))

    def dense(self) -> np.ndarray:
        A = np.zeros((self.n, self.n), np.complex128)
        for r in range(self.n):
            lo, hi = self.row_ptr[r], self.row_ptr[r + 1]
            A[r, self.col[lo:hi]] = self.val[lo:hi]
        return A


def _dense_to_csr(M: np.ndarray, complex_vals: bool):
    N = M.shape[0]
    rows, cols = np.nonzero(M)
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    rp = np.zeros(N + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=N), out=rp[1:])
    v = M[rows, cols]
    v = v.astype(np.complex128) if complex_vals else v.astype(np.float64)
    return rp, cols.astype(np.int32), v


def superop_csr(H: np.ndarray, ML: np.ndarray, omega: float) -> CSR:
    """Row-major CSR of the generator for Hermitian H and Lindblad
    coefficient matrix ML (rates R = |ML|^2)."""
    N = H.shape[0]
    hp, hi, hv = _dense_to_csr(np.asarray(H), True)
    R = np.abs(np.asarray(ML)) ** 2
    rp, ri, rv = _dense_to_csr(R, False)
    n = N * N
    row_ptr = np.zeros(n + 1, np.int64)
    L = lib()
    nnz = L.oracle_superop_csr(N, hp, hi, _ri(hv), rp, ri, rv, float(omega),
                               row_ptr, None, None)
    if nnz < 0:
        raise MemoryError("oracle_superop_csr")
    col = np.empty(nnz, np.int32)
    val = np.empty(nnz, np.complex128)
    nnz2 = L.oracle_superop_csr(N, hp, hi, _ri(hv), rp, ri, rv, float(omega),
                                row_ptr, col.ctypes.data, val.ctypes.data)
    if nnz2 != nnz:
        raise RuntimeError("oracle_superop_csr: inconsistent passes")
    return CSR(n, row_ptr, col, val)


def taylor_expmv(A: CSR, b: np.ndarray, t: float, m: int, s: int, tol: float):
    """One application of the single-time Taylor algorithm with given (m, s).
    Returns (F, number of matrix-vector products)."""
    F = np.empty(A.n, np.complex128)
    k = lib().oracle_taylor_expmv(A.n, A.row_ptr, A.col, _ri(A.val), _ri(b),
                                  float(t), int(m), int(s), float(tol),
                                  F.view(np.float64))
    if k < 0:
        raise MemoryError("oracle_taylor_expmv")
    return F, int(k)
