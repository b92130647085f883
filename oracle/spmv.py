"""y = A x for CSR A, in float64 (test infrastructure; see package header).

The definition (paper Section 2.1 with Section 3: whatever format the tuner
picks, the product is that of the input CSR):

    y_i = sum over the stored entries p of row i of val[p] * x[col[p]].

float32 matrices and vectors are widened to float64 exactly before the call,
so the oracle always answers in float64.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import build as _build

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        lib = ctypes.CDLL(path)
        i64, p = ctypes.c_int64, ctypes.c_void_p
        lib.ref_spmv_accurate.argtypes = [i64, p, p, p, p, p, p]
        lib.ref_spmv_accurate.restype = None
        lib.ref_spmv_rows.argtypes = [i64, p, p, p, p, p, p, p]
        lib.ref_spmv_rows.restype = None
        lib.ref_spmv_plain.argtypes = [i64, p, p, p, p, p, ctypes.c_int]
        lib.ref_spmv_plain.restype = None
        lib.ref_spmv_plain_f32.argtypes = [i64, p, p, p, p, p, ctypes.c_int]
        lib.ref_spmv_plain_f32.restype = None
        lib.ref_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _prep(row_ptr, col, val, x):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    c = np.ascontiguousarray(col, dtype=np.int32)
    v = np.ascontiguousarray(val, dtype=np.float64)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    return rp, c, v, xx


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def spmv_accurate(row_ptr, col, val, x):
    """Return (y, absax) with absax_i = sum |val| |x| over row i."""
    rp, c, v, xx = _prep(row_ptr, col, val, x)
    m = rp.size - 1
    y = np.empty(m, dtype=np.float64)
    a = np.empty(m, dtype=np.float64)
    _load().ref_spmv_accurate(m, _ptr(rp), _ptr(c), _ptr(v), _ptr(xx), _ptr(y), _ptr(a))
    return y, a


def spmv_rows(row_ptr, col, val, x, rows):
    """Accurate y_i and absax_i for the listed rows only."""
    rp, c, v, xx = _prep(row_ptr, col, val, x)
    r = np.ascontiguousarray(rows, dtype=np.int64)
    y = np.empty(r.size, dtype=np.float64)
    a = np.empty(r.size, dtype=np.float64)
    _load().ref_spmv_rows(r.size, _ptr(r), _ptr(rp), _ptr(c), _ptr(v), _ptr(xx), _ptr(y), _ptr(a))
    return y, a


def spmv_plain(row_ptr, col, val, x, nthreads=None, out=None):
    """Naive float64 sum, nnz-balanced OpenMP row blocks (paper Section 6)."""
    rp, c, v, xx = _prep(row_ptr, col, val, x)
    m = rp.size - 1
    y = out if out is not None else np.empty(m, dtype=np.float64)
    if nthreads is None:
        nthreads = max_threads()
    _load().ref_spmv_plain(m, _ptr(rp), _ptr(c), _ptr(v), _ptr(xx), _ptr(y), int(nthreads))
    return y


def spmv_plain_f32(row_ptr, col, val, x, nthreads=None, out=None):
    """The plain mode on float32 values and x (float64 sums, rounded once
    per row to float32): the CPU timing of float32-stored matrices."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    c = np.ascontiguousarray(col, dtype=np.int32)
    v = np.ascontiguousarray(val, dtype=np.float32)
    xx = np.ascontiguousarray(x, dtype=np.float32)
    m = rp.size - 1
    y = out if out is not None else np.empty(m, dtype=np.float32)
    if nthreads is None:
        nthreads = max_threads()
    _load().ref_spmv_plain_f32(m, _ptr(rp), _ptr(c), _ptr(v), _ptr(xx), _ptr(y), int(nthreads))
    return y


def max_threads() -> int:
    return int(_load().ref_max_threads())


def spmv_dense_exact(row_ptr, col, val, x):
    """Exact rational y (fractions.Fraction) for tiny inputs, by brute force."""
    from fractions import Fraction

    m = len(row_ptr) - 1
    out = []
    for i in range(m):
        s = Fraction(0)
        for p in range(int(row_ptr[i]), int(row_ptr[i + 1])):
            s += Fraction(float(val[p])) * Fraction(float(x[int(col[p])]))
        out.append(s)
    return out
