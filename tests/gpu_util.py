"""Helpers shared by the GPU parity tests (inputs, oracle comparison)."""
from __future__ import annotations

import sys

import numpy as np

from oracle import spmv as O

# Tolerances of the method's numerical contract: |y_gpu - y| <= tol * (|A||x|)_i
TOL = {np.float64: 1e-12, np.float32: 2e-6}


def dev(A, dtype):
    import torch
    rp = torch.from_numpy(A.row_ptr.astype(np.int32)).cuda()
    col = torch.from_numpy(np.ascontiguousarray(A.col, dtype=np.int32)).cuda()
    val = torch.from_numpy(np.ascontiguousarray(A.val).astype(dtype)).cuda()
    return rp, col, val


def vec(x, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x).astype(dtype)).cuda()


def note(msg):
    """Print (and flush) what the next GPU step is about to run."""
    print(msg, flush=True)
    sys.stdout.flush()


def assert_parity(y_gpu, A, x, dtype, rows=None, ref=None):
    """Compare GPU output with the float64 oracle on the same (rounded) data.

    ref: the oracle's (y, (|A||x|)) for these inputs when already computed
    (full vectors only)."""
    y = np.asarray(y_gpu, dtype=np.float64)
    if ref is not None:
        assert rows is None
        ref, absax = ref
    else:
        val = np.asarray(A.val).astype(dtype).astype(np.float64)
        xx = np.asarray(x).astype(dtype).astype(np.float64)
        if rows is None:
            ref, absax = O.spmv_accurate(A.row_ptr, A.col, val, xx)
        else:
            ref, absax = O.spmv_rows(A.row_ptr, A.col, val, xx, rows)
    assert y.shape == ref.shape, (y.shape, ref.shape)
    tol = TOL[dtype]
    err = np.abs(y - ref)
    bound = tol * absax
    zero = absax == 0
    assert np.all(y[zero] == 0), "rows with (|A||x|)_i = 0 must give exactly 0"
    bad = np.nonzero(err > bound)[0]
    assert bad.size == 0, (f"{bad.size} rows outside tolerance; first {bad[:5]}, "
                           f"err {err[bad[:5]]}, bound {bound[bad[:5]]}")
    return float(np.max(err / np.where(zero, 1, absax))) if y.size else 0.0
