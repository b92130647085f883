"""Parity at the benchmark's full sizes, in the configuration bench.py times.

Each matrix is planned exactly as the benchmark plans it (learned selector,
autotuned parameters); the output is compared with the oracle on a sample
of rows (first, last, the longest and a few thousand random ones) computed
one by one on the CPU.  The plain CSR kernel and the forced DIA / ELL
kernels are checked the same way where they apply.
"""
import numpy as np
import pytest

from paper_1210_2536_amd import synth as S
from paper_1210_2536_amd import workloads

from gpu_util import assert_parity, note

pytestmark = pytest.mark.gpu


def _sample_rows(A, count=4096, seed=0):
    rng = np.random.default_rng(seed)
    lens = np.diff(A.row_ptr)
    rows = np.concatenate([[0, A.m - 1, int(lens.argmax()), int(lens.argmin())],
                           rng.integers(0, A.m, size=min(count, A.m))])
    return np.unique(rows)


def _check(A, dt, xseed, selectors):
    import torch
    from paper_1210_2536_amd.spmv import Plan, default_selector
    model = default_selector()
    rp = torch.from_numpy(A.row_ptr.astype(np.int32)).cuda()
    col = torch.from_numpy(A.col).cuda()
    val = torch.from_numpy(A.val.astype(dt)).cuda()
    x = S.uniform_vector(A.n, xseed)
    xd = torch.from_numpy(x.astype(dt)).cuda()
    rows = _sample_rows(A)
    for sel in selectors:
        note(f"[fullsize] {A.name} {np.dtype(dt).name} selector={sel} nnz={A.nnz}")
        kw = dict(model=model, autotune=True) if sel == "mlp" else {}
        p = Plan(rp, col, val, n=A.n, selector=sel, **kw)
        y = p.run(xd).cpu().numpy()
        assert_parity(y[rows], A, x, dt, rows=rows)
        p.close()


def test_c5b_laplacian_256():
    A = S.laplace_7pt_large()
    assert A.m == 16_777_216 and A.nnz == 117_047_296
    _check(A, np.float64, (5, 2), ("mlp", "csr_scalar", "dia", "dia_direct", "ell"))


def test_c5a_zipf_8m():
    A = S.zipf_large()
    assert A.m == 8_000_000 and 1.9e8 < A.nnz < 2.2e8
    _check(A, np.float32, (5, 1), ("mlp", "csr_scalar", "coo"))


def test_c4_multilevel_levels_and_batch():
    import torch
    from paper_1210_2536_amd.spmv import Batch, Plan, default_selector
    levels = S.multilevel(160, 6)
    assert [A.m for A in levels] == [4_096_000, 512_000, 64_000, 8_000, 1_000, 125]
    assert levels[0].nnz == 109_215_352
    model = default_selector()
    for dt in (np.float64, np.float32):
        plans, xs, ys, xh = [], [], [], []
        for l, A in enumerate(levels):
            rp = torch.from_numpy(A.row_ptr.astype(np.int32)).cuda()
            col = torch.from_numpy(A.col).cuda()
            val = torch.from_numpy(A.val.astype(dt)).cuda()
            plans.append(Plan(rp, col, val, n=A.n, selector="mlp", model=model, autotune=True))
            x = S.uniform_vector(A.n, (4, l))
            xh.append(x)
            xs.append(torch.from_numpy(x.astype(dt)).cuda())
            ys.append(torch.empty(A.m, dtype=xs[-1].dtype, device="cuda"))
        for mode in (0, 1):
            note(f"[fullsize] multilevel {np.dtype(dt).name} batch mode {mode}")
            B = Batch(plans, mode=mode)
            B.run(xs, ys)
            torch.cuda.synchronize()
            for A, x, y in zip(levels, xh, ys):
                rows = _sample_rows(A, 2048)
                assert_parity(y.cpu().numpy()[rows], A, x, dt, rows=rows)


def test_sweep_all_matrices_sampled():
    """All 200 sweep matrices in both precisions, planned as the benchmark does."""
    import torch
    from paper_1210_2536_amd.spmv import Plan, default_selector
    model = default_selector()
    for A, dt, xseed in workloads.build("sweep"):
        rp = torch.from_numpy(A.row_ptr.astype(np.int32)).cuda()
        col = torch.from_numpy(A.col).cuda()
        val = torch.from_numpy(A.val.astype(dt)).cuda()
        x = S.uniform_vector(A.n, xseed)
        p = Plan(rp, col, val, n=A.n, selector="mlp", model=model, autotune=True)
        y = p.run(torch.from_numpy(x.astype(dt)).cuda()).cpu().numpy()
        rows = _sample_rows(A, 512)
        assert_parity(y[rows], A, x, dt, rows=rows)
        p.close()
