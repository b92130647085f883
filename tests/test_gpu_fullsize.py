"""Parity at the benchmark's full sizes, in the configuration bench.py times.

Each matrix is planned exactly as the benchmark plans it (learned selector,
autotuned parameters) and the WHOLE output vector is compared with the
oracle (float64, compensated sums, OpenMP over rows), element by element,
within 1e-12 (|A||x|)_i in float64 and 2e-6 (|A||x|)_i in float32.  The plain
CSR kernel and the forced DIA / ELL / COO kernels are checked the same way
where they apply, so every row block, x panel and tile boundary that only
occurs at full size is covered.  The 7-point Laplacian on 256^3 is also run
on the integer vector i^2 + j^2 + k^2, where every format must reproduce the
oracle bit for bit (integer partial sums are exact in any order).
"""
import numpy as np
import pytest

from oracle import spmv as O
from paper_1210_2536_amd import synth as S
from paper_1210_2536_amd import workloads

from gpu_util import assert_parity, note

pytestmark = pytest.mark.gpu


def _oracle(A, x, dt):
    val = np.asarray(A.val).astype(dt).astype(np.float64)
    xx = np.asarray(x).astype(dt).astype(np.float64)
    return O.spmv_accurate(A.row_ptr, A.col, val, xx)


def _check(A, dt, xseed, selectors, ref=None):
    import torch
    from paper_1210_2536_amd.spmv import Plan, default_selector
    model = default_selector()
    rp = torch.from_numpy(A.row_ptr.astype(np.int32)).cuda()
    col = torch.from_numpy(A.col).cuda()
    val = torch.from_numpy(A.val.astype(dt)).cuda()
    x = S.uniform_vector(A.n, xseed)
    xd = torch.from_numpy(x.astype(dt)).cuda()
    ref = _oracle(A, x, dt) if ref is None else ref
    for sel in selectors:
        note(f"[fullsize] {A.name} {np.dtype(dt).name} selector={sel} nnz={A.nnz}")
        kw = dict(model=model, autotune=True) if sel == "mlp" else {}
        p = Plan(rp, col, val, n=A.n, selector=sel, **kw)
        y = p.run(xd).cpu().numpy()
        assert_parity(y, A, x, dt, ref=ref)
        p.close()
    return rp, col, val


def test_c5b_laplacian_256():
    import torch
    from paper_1210_2536_amd.spmv import Plan
    A = S.laplace_7pt_large()
    assert A.m == 16_777_216 and A.nnz == 117_047_296
    sels = ("mlp", "csr_scalar", "dia", "dia_direct", "ell")
    rp, col, val = _check(A, np.float64, (5, 2), sels)
    # integer polynomial x = i^2 + j^2 + k^2: exact, so bitwise equal
    g = 256
    r = np.arange(A.n, dtype=np.int64)
    i, j, k = r // (g * g), (r // g) % g, r % g
    xp = (i * i + j * j + k * k).astype(np.float64)
    ref, _ = O.spmv_accurate(A.row_ptr, A.col, A.val, xp)
    interior = ((i > 0) & (i < g - 1) & (j > 0) & (j < g - 1) & (k > 0) & (k < g - 1))
    assert np.all(ref[interior] == -6.0)
    xd = torch.from_numpy(xp).cuda()
    for sel in sels:
        if sel == "mlp":
            continue
        note(f"[fullsize] {A.name} float64 selector={sel} integer x, bitwise")
        p = Plan(rp, col, val, n=A.n, selector=sel)
        y = p.run(xd).cpu().numpy()
        assert np.array_equal(y, ref), sel
        p.close()


def test_c5a_zipf_8m():
    A = S.zipf_large()
    assert A.m == 8_000_000 and 1.9e8 < A.nnz < 2.2e8
    _check(A, np.float32, (5, 1), ("mlp", "csr_scalar", "coo", "csr_adaptive", "csr_panel"))


def test_c4_multilevel_levels_and_batch():
    import torch
    from paper_1210_2536_amd.spmv import Batch, Plan, default_selector
    levels = S.multilevel(160, 6)
    assert [A.m for A in levels] == [4_096_000, 512_000, 64_000, 8_000, 1_000, 125]
    assert levels[0].nnz == 109_215_352
    model = default_selector()
    for dt in (np.float64, np.float32):
        plans, xs, ys, xh, refs = [], [], [], [], []
        for l, A in enumerate(levels):
            rp = torch.from_numpy(A.row_ptr.astype(np.int32)).cuda()
            col = torch.from_numpy(A.col).cuda()
            val = torch.from_numpy(A.val.astype(dt)).cuda()
            plans.append(Plan(rp, col, val, n=A.n, selector="mlp", model=model, autotune=True))
            x = S.uniform_vector(A.n, (4, l))
            xh.append(x)
            refs.append(_oracle(A, x, dt))
            xs.append(torch.from_numpy(x.astype(dt)).cuda())
            ys.append(torch.empty(A.m, dtype=xs[-1].dtype, device="cuda"))
        note(f"[fullsize] multilevel {np.dtype(dt).name} level plans, one run each")
        for A, p, x, xd, ref in zip(levels, plans, xh, xs, refs):
            assert_parity(p.run(xd).cpu().numpy(), A, x, dt, ref=ref)
        for mode in (0, 1):
            note(f"[fullsize] multilevel {np.dtype(dt).name} batch mode {mode}")
            B = Batch(plans, mode=mode)
            if mode == 0:
                B.tune(xs, ys)
            for y in ys:
                y.fill_(float("nan"))
            B.run(xs, ys)
            torch.cuda.synchronize()
            for A, x, y, ref in zip(levels, xh, ys, refs):
                assert_parity(y.cpu().numpy(), A, x, dt, ref=ref)
            B.close()


def test_sweep_all_matrices_full_vectors():
    """All 200 sweep matrices in both precisions, planned as the benchmark
    does, every output element checked."""
    import torch
    from paper_1210_2536_amd.spmv import Plan, default_selector
    model = default_selector()
    kinds = {}
    for A, dt, xseed in workloads.build("sweep"):
        rp = torch.from_numpy(A.row_ptr.astype(np.int32)).cuda()
        col = torch.from_numpy(A.col).cuda()
        val = torch.from_numpy(A.val.astype(dt)).cuda()
        x = S.uniform_vector(A.n, xseed)
        p = Plan(rp, col, val, n=A.n, selector="mlp", model=model, autotune=True)
        info = p.info()
        note(f"[fullsize] {A.name} {np.dtype(dt).name} {info['kernel_name']} nnz={A.nnz}")
        y = p.run(torch.from_numpy(x.astype(dt)).cuda()).cpu().numpy()
        assert_parity(y, A, x, dt)
        tag = info["kernel_name"] + ("+tiles" if info["params"]["long_lds"] == 3
                                     and info["long_rows"] else "")
        kinds[tag] = kinds.get(tag, 0) + 1
        p.close()
    note(f"[fullsize] sweep plans by kernel: {kinds}")
