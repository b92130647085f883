"""The allocation-free feature entry point against the allocating one.

spmv_features_compute_noalloc runs the same validation and feature kernels
as spmv_features_compute with its device buffers in a fixed device array;
its report must equal the allocating call's field for field (integers
exactly, ratios bit for bit: same kernels, same order), on calls in a row
whose sizes shrink, so that what one call leaves in the shared array never
reaches the next.  Oversized matrices are refused before any device work.
"""
import ctypes

import numpy as np
import pytest

from paper_1210_2536_amd import capi as C
from paper_1210_2536_amd import synth as S

from gpu_util import dev, note

pytestmark = pytest.mark.gpu


def _csr(A, dtype):
    rp, col, val = dev(A, dtype)
    c = C.spmv_csr(A.m, A.n, A.nnz, ctypes.c_void_p(rp.data_ptr()),
                   ctypes.c_void_p(col.data_ptr()), ctypes.c_void_p(val.data_ptr()),
                   C.SPMV_F64 if dtype == np.float64 else C.SPMV_F32)
    return c, (rp, col, val)


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _fields(F):
    return {k: getattr(F, k) for k, _ in F._fields_}


def _both(A, dtype):
    c, keep = _csr(A, dtype)
    Fa, Fn = C.spmv_features(), C.spmv_features()
    sa = C.lib().spmv_features_compute(ctypes.byref(c), ctypes.byref(Fa), _stream())
    sn = C.lib().spmv_features_compute_noalloc(ctypes.byref(c), ctypes.byref(Fn), _stream())
    del keep
    return sa, sn, _fields(Fa), _fields(Fn)


def _same(a, b):
    for k in a:
        va, vb = a[k], b[k]
        if isinstance(va, float):
            assert np.array_equal(np.float64(va), np.float64(vb), equal_nan=True), (k, va, vb)
        else:
            assert va == vb, (k, va, vb)


def test_noalloc_features_equal_allocating_features():
    big = S.stencil_7pt(140)          # census after the checks (m + n - 1 > 2^22)
    rng = np.random.default_rng([61, 0])
    zipf = S.zipf_g2(rng, 200_000)    # power-law fit over many degrees
    small = S.stencil_5pt(64)         # census together with the checks
    for A, dt in ((big, np.float64), (zipf, np.float32), (small, np.float64),
                  (S.stencil_5pt(8), np.float32)):
        note(f"[noalloc] {A.name} {np.dtype(dt).name} m={A.m} n={A.n} nnz={A.nnz}")
        sa, sn, fa, fn = _both(A, dt)
        assert sa == C.SPMV_OK and sn == C.SPMV_OK, (sa, sn, C.lib().spmv_last_error())
        _same(fa, fn)
        assert fn["m"] == A.m and fn["nnz"] == A.nnz and fn["max_rd"] >= 1
    # the census really ran on the stencils (DIA feasible there)
    assert _both(small, np.float64)[3]["ndiags"] == 5


def test_noalloc_features_errors():
    # invalid CSR: the same rejection as the allocating call
    A = S.stencil_5pt(16)
    bad_col = A.col.copy()
    bad_col[5], bad_col[6] = bad_col[6], bad_col[5]      # unsorted row
    B = S.CSR(A.m, A.n, A.row_ptr, bad_col, A.val, "unsorted")
    note("[noalloc] unsorted columns")
    sa, sn, _, _ = _both(B, np.float64)
    assert sa == C.SPMV_EINVAL and sn == C.SPMV_EINVAL
    # then a valid call on the same array still agrees
    sa, sn, fa, fn = _both(A, np.float64)
    assert sa == sn == C.SPMV_OK
    _same(fa, fn)
    # beyond the fixed array: refused before any device work
    F = C.spmv_features()
    huge = C.spmv_csr(10_000_000, 10_000_000, 0, None, None, None, C.SPMV_F64)
    assert C.lib().spmv_features_compute_noalloc(ctypes.byref(huge), ctypes.byref(F),
                                                 None) == C.SPMV_EUNSUPPORTED
    assert b"scratch" in C.lib().spmv_last_error()
