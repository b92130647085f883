"""GPU parity: every kernel of the HIP library against the CPU oracle.

Float64 results must lie within 1e-12 (|A||x|)_i of the oracle, float32 within
2e-6 (|A||x|)_i; integer stencils on polynomial vectors are exact in any
summation order, so there the GPU must match the oracle bit for bit.
"""
import numpy as np
import pytest

from oracle import features as OF
from oracle import spmv as O
from paper_1210_2536_amd import synth as S

from gpu_util import assert_parity, dev, note, vec

pytestmark = pytest.mark.gpu

KERNELS = ("csr_scalar", "csr_vector", "csr_adaptive", "ell", "dia", "dia_direct", "coo",
           "csr_panel", "bcsr")
DTYPES = (np.float64, np.float32)


def _plan(A, dtype, kernel, **kw):
    from paper_1210_2536_amd.spmv import Plan
    rp, col, val = dev(A, dtype)
    return Plan(rp, col, val, n=A.n, selector=kernel, **kw)


def _feasible(A, kernel):
    f = OF.extract(A.m, A.n, A.row_ptr, A.col)
    if kernel == "csr_panel":
        # rows longer than one 256-thread workgroup can sum (1,024,000 entries)
        # are not held by column panels (SPMV_EUNSUPPORTED, checked below)
        return f["max_RD"] <= 1_024_000
    if kernel == "ell":
        return f["ell_feasible"]
    if kernel in ("dia", "dia_direct"):
        return f["dia_feasible"]
    if kernel == "bcsr":
        # zero-fill rule on 4x4 blocks: stored slots at most 20x the entries
        return f["blocks4"] > 0 and 16 * f["blocks4"] <= 20 * f["NNZ"]
    return True


def _run_all(A, dtype, x, kernels=KERNELS, **kw):
    out = {}
    for k in kernels:
        if not _feasible(A, k):
            continue
        note(f"[parity] {A.name} {np.dtype(dtype).name} {k} m={A.m} nnz={A.nnz}")
        p = _plan(A, dtype, k, **kw)
        assert p.info()["kernel_name"] == k
        y = p.run(vec(x, dtype)).cpu().numpy()
        out[k] = y
    return out


def test_c1_laplacian_all_formats():
    """5-point Laplacian 64x64 (n = 4096, nnz = 20224), float64, x from seed 1."""
    A = S.stencil_5pt(64)
    x = S.uniform_vector(A.n, 1)
    ys = _run_all(A, np.float64, x)
    assert set(ys) == set(KERNELS)
    for k, y in ys.items():
        assert_parity(y, A, x, np.float64)
    # integer polynomial: exact in any order -> bitwise equal to the oracle
    g = 64
    i, j = np.divmod(np.arange(A.n), g)
    xp = (i * i + j * j).astype(np.float64)
    ref, _ = O.spmv_accurate(A.row_ptr, A.col, A.val, xp)
    for dtype in DTYPES:
        for k, y in _run_all(A, dtype, xp).items():
            assert np.array_equal(y.astype(np.float64), ref), (k, dtype)
    # the call form plan(x, out=y) on the current torch stream
    import torch
    from paper_1210_2536_amd.spmv import Plan
    rp, col, val = dev(A, np.float64)
    plan = Plan(rp, col, val, n=A.n)
    out = torch.full((A.m,), float("nan"), dtype=torch.float64, device="cuda")
    assert plan(vec(xp, np.float64), out=out) is out
    assert np.array_equal(out.cpu().numpy(), ref)


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
@pytest.mark.parametrize("gen", range(4), ids=S.GEN_NAMES)
def test_generators_all_kernels(gen, dtype):
    for s, n in enumerate((1000, 5003, 30011)):
        rng = np.random.default_rng([40, gen, s])
        A = (S.band_g0, S.uniform_g1, S.zipf_g2, S.blocks_g3)[gen](rng, n)
        A.name = f"g{gen}_{A.name}"
        x = S.uniform_vector(A.n, [41, gen, s])
        for k, y in _run_all(A, dtype, x).items():
            assert_parity(y, A, x, dtype)


def _edge_matrices():
    rng = np.random.default_rng(77)
    mats = []
    # empty rows at the start, middle and end, explicit zeros, rectangular
    m, n = 300, 170
    dense = (rng.random((m, n)) < 0.05) * rng.uniform(-1, 1, (m, n))
    dense[:7] = 0
    dense[100:160] = 0
    dense[-11:] = 0
    dense[50, :] = rng.uniform(-1, 1, n)         # one dense row
    r, c = np.nonzero(dense != 0)
    vals = dense[r, c]
    vals[::17] = 0.0                             # explicit stored zeros
    rp = np.zeros(m + 1, np.int64)
    np.cumsum(np.bincount(r, minlength=m), out=rp[1:])
    mats.append(S.CSR(m, n, rp, c.astype(np.int32), vals, "edge_rect_empty_rows"))
    # 1 x 1, one row, one column
    mats.append(S.CSR(1, 1, np.array([0, 1]), np.array([0], np.int32), np.array([2.5]), "one"))
    k = 100_000
    mats.append(S.CSR(1, k, np.array([0, k]), np.arange(k, dtype=np.int32),
                      rng.uniform(-1, 1, k), "dense_row_1e5"))
    mats.append(S.CSR(64, 1, np.arange(65), np.zeros(64, np.int32), rng.uniform(-1, 1, 64),
                      "one_column"))
    # wide-offset band: DIA windows far apart (offsets +-g^2)
    mats.append(S.stencil_7pt(20))
    # a few very long rows among short ones (exercises every adaptive bin)
    m = 20_000
    lens = np.ones(m, np.int64)
    lens[[5, 6000, 19999]] = [15_000, 9_000, 20_000]
    lens[100:200] = 70
    lens[300:400] = 3000
    cols = S._sorted_distinct_cols(np.random.default_rng(5), lens, m)
    rp = np.zeros(m + 1, np.int64)
    np.cumsum(lens, out=rp[1:])
    mats.append(S.CSR(m, m, rp, cols, rng.uniform(-1, 1, cols.size), "mixed_long_rows"))
    # a row longer than one workgroup may sum alone: split into segments
    k, n = 1_100_000, 1_200_000
    lens = np.array([k, 10, 0, 3])
    cols = S._sorted_distinct_cols(np.random.default_rng(6), lens, n)
    rp = np.concatenate([[0], np.cumsum(lens)])
    mats.append(S.CSR(4, n, rp, cols, rng.uniform(-1, 1, cols.size), "split_row"))
    return mats


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
def test_edge_cases(dtype):
    from paper_1210_2536_amd import capi as C
    for A in _edge_matrices():
        x = S.uniform_vector(A.n, [42, A.m])
        for k, y in _run_all(A, dtype, x).items():
            assert_parity(y, A, x, dtype)
        if not _feasible(A, "csr_panel"):
            with pytest.raises(C.SpmvError) as ei:
                _plan(A, dtype, "csr_panel")
            assert ei.value.status == C.SPMV_EUNSUPPORTED


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
def test_tiny_tiles_force_every_boundary(dtype):
    """COO chunks of 64 entries, DIA windows of one diagonal, small workgroups."""
    A = _edge_matrices()[-2]
    x = S.uniform_vector(A.n, 43)
    for prm in ({"coo_chunk": 1}, {"coo_chunk": 3}, {"adaptive_wg_min": 64, "adaptive_rows_per_lane": 1},
                {"vector_lanes": 64}, {"vector_lanes": 1, "block": 64}):
        for k, y in _run_all(A, dtype, x, kernels=("coo", "csr_adaptive", "csr_vector"),
                             params=prm).items():
            assert_parity(y, A, x, dtype)
    # column panels in one launch, eight at a time (one per XCD): one group
    # (default), two groups (16 KiB panels), 160 panels of 1 KiB; or panels of
    # 1 KiB / 8 KiB of x one after another with running sums carried across
    for prm in ({}, {"panel_kib": 16}, {"panel_kib": 1}, {"panel_kib": 1, "panel_xcd": 2},
                {"panel_kib": 8, "panel_xcd": 2, "stream_nt": 1}):
        for k, y in _run_all(A, dtype, x, kernels=("csr_panel",), params=prm).items():
            assert_parity(y, A, x, dtype)
    for gen in range(4):
        G = (S.band_g0, S.uniform_g1, S.zipf_g2, S.blocks_g3)[gen](np.random.default_rng([46, gen]), 9000)
        xg = S.uniform_vector(G.n, [46, gen])
        for prm in ({}, {"panel_kib": 4}, {"panel_kib": 8, "panel_xcd": 2}):
            for k, y in _run_all(G, dtype, xg, kernels=("csr_panel",), params=prm).items():
                assert_parity(y, G, xg, dtype)
    # BCSR with every lane width, on shapes that are not multiples of 4
    # (49 x 49 stencil, 37 x 53 rectangular) and on 4x4 dense blocks
    rng = np.random.default_rng(48)
    for M in (S.stencil_5pt(7), S.random_csr(rng, 37, 53, 0.25),
              S.blocks_g3(np.random.default_rng([48, 1]), 3000)):
        xm = S.uniform_vector(M.n, [48, M.m])
        for prm in ({}, {"bcsr_lanes": 1}, {"bcsr_lanes": 4, "block": 64}, {"bcsr_lanes": 64},
                    {"bcsr_lanes": 8}, {"bcsr_lanes": 32, "block": 64},
                    {"bcsr_lanes": 16, "stream_nt": 1}):
            for k, y in _run_all(M, dtype, xm, kernels=("bcsr",), params=prm).items():
                assert_parity(y, M, xm, dtype)
    B = S.stencil_27pt(12)
    xb = S.uniform_vector(B.n, 44)
    for prm in ({"dia_span": 0}, {"dia_span": 1, "dia_rows_per_thread": 1},
                {"dia_rows_per_thread": 8}, {"ell_unroll": 1}, {"ell_unroll": 2}):
        for k, y in _run_all(B, dtype, xb, kernels=("dia", "dia_direct", "ell"), params=prm).items():
            assert_parity(y, B, xb, dtype)
    # wide loads (a lane owns 16 bytes of consecutive rows) and one row per
    # lane, on 1728 rows and on 2197 rows (not a multiple of the row group)
    Cm = S.stencil_7pt(13)
    xc = S.uniform_vector(Cm.n, 47)
    for M, xm in ((B, xb), (Cm, xc)):
        ref = {}
        for prm in ({"wide_loads": 1}, {"wide_loads": 2},
                    {"wide_loads": 1, "block": 64, "dia_rows_per_thread": 1, "ell_unroll": 1},
                    {"wide_loads": 1, "dia_rows_per_thread": 8, "dia_span": 0},
                    {"wide_loads": 1, "dia_span": 1, "ell_unroll": 2, "stream_nt": 1}):
            for k, y in _run_all(M, dtype, xm, kernels=("dia", "dia_direct", "ell"),
                                 params=prm).items():
                assert_parity(y, M, xm, dtype)
                # same per-row operations in the same order: bitwise equal
                if k in ref:
                    assert np.array_equal(ref[k], y), (M.name, k, prm)
                ref.setdefault(k, y)


def test_empty_matrices():
    import torch
    from paper_1210_2536_amd.spmv import Plan
    for k in KERNELS:
        # m = 0
        rp = torch.zeros(1, dtype=torch.int32, device="cuda")
        col = torch.zeros(0, dtype=torch.int32, device="cuda")
        val = torch.zeros(0, dtype=torch.float64, device="cuda")
        if k in ("ell", "dia", "dia_direct", "bcsr"):
            continue
        p = Plan(rp, col, val, n=5, selector=k)
        p.run(torch.ones(5, dtype=torch.float64, device="cuda"))
    # nnz = 0, m > 0: y is all zero for every kernel that accepts it
    for k in KERNELS:
        rp = torch.zeros(33, dtype=torch.int32, device="cuda")
        col = torch.zeros(0, dtype=torch.int32, device="cuda")
        val = torch.zeros(0, dtype=torch.float32, device="cuda")
        try:
            p = Plan(rp, col, val, n=7, selector=k)
        except RuntimeError:
            assert k in ("ell", "dia", "dia_direct", "bcsr")
            continue
        y = p.run(torch.ones(7, dtype=torch.float32, device="cuda"),
                  torch.full((32,), 9.0, dtype=torch.float32, device="cuda"))
        assert torch.all(y == 0)


def test_determinism_bitwise():
    A = S.zipf_g2(np.random.default_rng([45, 0]), 50_000)
    x = S.uniform_vector(A.n, 45)
    for k in KERNELS:
        if not _feasible(A, k):
            continue
        p = _plan(A, np.float64, k, params={"coo_chunk": 2})
        xv = vec(x, np.float64)
        y1 = p.run(xv).cpu().numpy()
        y2 = p.run(xv).cpu().numpy()
        assert np.array_equal(y1.view(np.uint64), y2.view(np.uint64)), k


def test_run_argument_errors():
    import torch
    from paper_1210_2536_amd import capi as C
    A = S.stencil_5pt(8)
    p = _plan(A, np.float64, "csr_vector")
    buf = torch.zeros(2 * A.n, dtype=torch.float64, device="cuda")
    st = C.lib().spmv_run(p.handle, C.ctypes.c_void_p(buf.data_ptr()),
                          C.ctypes.c_void_p(buf.data_ptr() + 8 * 10), None)
    assert st == C.SPMV_EINVAL and b"overlap" in C.lib().spmv_last_error()
    assert C.lib().spmv_run(None, None, None, None) == C.SPMV_EINVAL
    assert C.lib().spmv_plan_destroy(None) == C.SPMV_OK


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
def test_segmented_plans(dtype):
    """Row segments of about nnz/S entries, each planned on its own: parity,
    segment boundaries, the kernels chosen per segment, the round trip and a
    batch holding a segmented plan."""
    import torch
    from paper_1210_2536_amd.spmv import Batch, Plan
    rng = np.random.default_rng(49)
    mats = [S.mixed_stencil_zipf(g=16, kmax=500, seed=(49, 0)),
            S.random_csr(rng, 301, 170, 0.05, explicit_zeros=True), _edge_matrices()[0]]
    for A in mats:
        x = S.uniform_vector(A.n, [49, A.m])
        rp, col, val = dev(A, dtype)
        for seg in (2, 3, 7, 64):
            for sel in ("rules", "exhaustive"):
                note(f"[segments] {A.name} {np.dtype(dtype).name} S={seg} {sel}")
                p = Plan(rp, col, val, n=A.n, selector=sel, segments=seg)
                info = p.info()
                parts = p.segments()
                assert info["n_segments"] == len(parts) >= 1
                r0s = [r0 for r0, _ in parts]
                assert r0s[0] == 0 and all(b > a for a, b in zip(r0s, r0s[1:]))
                assert sum(q.m for _, q in parts) == A.m and sum(q.nnz for _, q in parts) == A.nnz
                y = p.run(vec(x, dtype)).cpu().numpy()
                assert_parity(y, A, x, dtype)
                rp2, col2, v2 = p.roundtrip()
                assert np.array_equal(rp2.cpu().numpy(), A.row_ptr.astype(np.int32))
                assert np.array_equal(col2.cpu().numpy(), A.col)
                assert np.array_equal(v2.cpu().numpy().view(np.uint8),
                                      A.val.astype(dtype).view(np.uint8))
    # planned as three nnz-balanced segments, the first lies inside the
    # stencil half and the last inside the random half: the rules give them
    # different formats
    A = mats[0]
    rp, col, val = dev(A, dtype)
    p = Plan(rp, col, val, n=A.n, selector="rules", segments=3)
    kinds = [q.info()["kernel_name"] for _, q in p.segments()]
    assert kinds[0] in ("dia", "dia_direct") and kinds[-1] not in ("dia", "dia_direct"), kinds
    x = vec(S.uniform_vector(A.n, 50), dtype)
    ref = p.run(x).cpu().numpy()
    for mode in (0, 1):
        B = Batch([p], mode=mode)
        y = torch.full((A.m,), float("nan"), dtype=x.dtype, device="cuda")
        B.run([x], [y])
        torch.cuda.synchronize()
        assert np.array_equal(y.cpu().numpy().view(np.uint8), ref.view(np.uint8)), mode
        B.close()


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
def test_autotuned_plans_every_point_agrees(dtype):
    """The autotuner checks every parameter point it times against its
    starting point on an all-ones probe (twice the accuracy bound); on these
    matrices no point is rejected, and the kept plan matches the oracle."""
    from paper_1210_2536_amd.spmv import Plan
    mats = [S.stencil_7pt(24), S.stencil_27pt(14),
            S.uniform_g1(np.random.default_rng([80, 0]), 30_000),
            S.zipf_g2(np.random.default_rng([80, 1]), 60_000),
            S.blocks_g3(np.random.default_rng([80, 2]), 40_000)]
    for i, A in enumerate(mats):
        for sel in ("rules", "mlp"):
            note(f"[autotune] {A.name} {np.dtype(dtype).name} {sel}")
            rp, col, val = dev(A, dtype)
            p = Plan(rp, col, val, n=A.n, selector=sel, autotune=True)
            info = p.info()
            assert info["tune_rejected"] == 0, (A.name, info["kernel_name"])
            x = np.random.default_rng([81, i]).uniform(-1, 1, A.n)
            assert_parity(p.run(vec(x, dtype)).cpu().numpy(), A, x, dtype)


def test_tune_cache_round_trip(tmp_path):
    """A tuned plan's kernel and parameters go into the JSON cache; a new
    cache read from the file plans the same matrix with them, without
    selection or search, and the result matches the oracle."""
    from paper_1210_2536_amd.spmv import TuneCache
    path = str(tmp_path / "tune.json")
    A = S.zipf_g2(np.random.default_rng([82, 0]), 50_000)
    x = np.random.default_rng([82, 1]).uniform(-1, 1, A.n)
    for dtype in (np.float64, np.float32):
        rp, col, val = dev(A, dtype)
        c1 = TuneCache(path)
        p1 = c1.plan(rp, col, val, n=A.n, selector="mlp")
        assert c1.misses == 1 and c1.hits == 0
        c1.save()
        c2 = TuneCache(path)
        p2 = c2.plan(rp, col, val, n=A.n)
        assert c2.hits == 1 and c2.misses == 0
        i1, i2 = p1.info(), p2.info()
        assert i2["kernel"] == i1["kernel"] and i2["params"] == i1["params"]
        assert i2["t_tune_ms"] == 0.0 and i2["selector_used"] == 3  # forced
        assert_parity(p2.run(vec(x, dtype)).cpu().numpy(), A, x, dtype)
    # both dtypes are kept apart
    assert len(TuneCache(path).entries) == 2


def test_plan_memory_from_the_callers_allocator():
    """Plans take their device memory from the caller's allocator (here
    PyTorch's caching allocator through spmv_allocator) and give it back on
    destruction; with no allocator the library's own is used.  Results are
    the same either way."""
    import torch
    from paper_1210_2536_amd.spmv import Plan, TorchAllocator
    A = S.zipf_g2(np.random.default_rng([83, 0]), 40_000)
    x = np.random.default_rng([83, 1]).uniform(-1, 1, A.n)
    rp, col, val = dev(A, np.float64)
    ta = TorchAllocator(torch.device("cuda", torch.cuda.current_device()))
    for k in ("csr_adaptive", "coo", "ell", "csr_panel", "mlp"):
        if k == "ell" and not OF.extract(A.m, A.n, A.row_ptr, A.col)["ell_feasible"]:
            continue
        note(f"[allocator] {k}")
        kw = {"params": {"panel_kib": 16}} if k == "csr_panel" else {}
        p = Plan(rp, col, val, n=A.n, selector=k, allocator=ta, autotune=(k == "mlp"), **kw)
        held = ta.bytes_held()
        assert held >= p.info()["device_bytes"] > 0, (k, held)
        y = p.run(vec(x, np.float64)).cpu().numpy()
        assert_parity(y, A, x, np.float64)
        rp2, col2, v2 = p.roundtrip()    # temporaries through the allocator too
        assert np.array_equal(col2.cpu().numpy(), A.col)
        assert ta.bytes_held() == held
        p.close()
        assert ta.bytes_held() == 0, k
        q = Plan(rp, col, val, n=A.n, selector=k, allocator=None, **kw)
        assert ta.bytes_held() == 0
        assert_parity(q.run(vec(x, np.float64)).cpu().numpy(), A, x, np.float64)
        q.close()



def test_plan_closed_while_another_stream_runs_it():
    """A plan built on the current stream runs on a side stream; closing it
    while those launches are still queued hands its blocks back to PyTorch's
    caching allocator only once the device is idle, so a tensor allocated
    and overwritten right after the close (it may take the same blocks)
    cannot change what the queued runs read."""
    import torch
    from paper_1210_2536_amd.spmv import Plan
    A = S.zipf_g2(np.random.default_rng([91, 0]), 200_000)
    x = np.random.default_rng([91, 1]).uniform(-1, 1, A.n)
    rp, col, val = dev(A, np.float64)
    xd = vec(x, np.float64)
    side = torch.cuda.Stream()
    for k in ("csr_adaptive", "coo", "csr_panel"):
        note(f"[side stream] {k}")
        p = Plan(rp, col, val, n=A.n, selector=k)
        held = p.info()["device_bytes"]
        ys = [torch.empty(A.m, dtype=torch.float64, device="cuda") for _ in range(16)]
        side.wait_stream(torch.cuda.current_stream())
        for y in ys:
            p.run(xd, y, stream=side)
        p.close()
        junk = torch.full((held // 8 + 4096,), float("nan"), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        for y in ys:
            assert_parity(y.cpu().numpy(), A, x, np.float64)
        del junk

def test_long_rows_through_lds():
    """float64 rows of the longest bin taken by the kernel that streams x
    through LDS in column chunks (several chunks and a partial one, rows
    that skip chunks), inside the binned CSR kernel and the column panels,
    alone and in a persistent batch; float32 ignores the switch."""
    import torch
    from paper_1210_2536_amd.spmv import Batch, Plan
    rng = np.random.default_rng(84)
    mats = [S.zipf_g2(np.random.default_rng([84, 0]), 20_000),       # 3 chunks of 8192
            S.uniform_g1(np.random.default_rng([84, 1]), 9000),
            S.random_csr(rng, 300, 17_000, 0.02),                   # 340 per row, 3 chunks
            S.random_csr(rng, 50, 5000, 0.3)]                       # one partial chunk
    for i, A in enumerate(mats):
        x = np.random.default_rng([85, i]).uniform(-1, 1, A.n)
        for k, extra in (("csr_adaptive", {}), ("csr_panel", {"panel_kib": 16}),
                         ("csr_panel", {"panel_kib": 16, "panel_xcd": 2})):
            for wg in (64, 256):
                note(f"[long lds] {A.name} {k} {extra} wg_min={wg}")
                prm = dict(extra, long_lds=1, adaptive_wg_min=wg)
                rp, col, val = dev(A, np.float64)
                p = Plan(rp, col, val, n=A.n, selector=k, params=prm)
                assert p.info()["params"]["long_lds"] in (1, 2)
                y = p.run(vec(x, np.float64)).cpu().numpy()
                assert_parity(y, A, x, np.float64)
                if k == "csr_adaptive":
                    B = Batch([p], mode=0)
                    yb = torch.full((A.m,), float("nan"), dtype=torch.float64, device="cuda")
                    B.run([vec(x, np.float64)], [yb])
                    torch.cuda.synchronize()
                    assert np.array_equal(yb.cpu().numpy().view(np.uint8), y.view(np.uint8))
        rp, col, val = dev(A, np.float32)
        p = Plan(rp, col, val, n=A.n, selector="csr_adaptive",
                 params={"long_lds": 1, "adaptive_wg_min": 64})
        assert p.info()["params"]["long_lds"] == 2
        assert_parity(p.run(vec(x, np.float32)).cpu().numpy(), A, x, np.float32)
    # the switch is used where it was asked for
    A = mats[0]
    rp, col, val = dev(A, np.float64)
    on = Plan(rp, col, val, n=A.n, selector="csr_adaptive",
              params={"long_lds": 1, "adaptive_wg_min": 64}).info()["params"]["long_lds"]
    off = Plan(rp, col, val, n=A.n, selector="csr_adaptive",
               params={"long_lds": 2, "adaptive_wg_min": 64}).info()["params"]["long_lds"]
    assert on == 1 and off == 2


def test_long_rows_by_tiles():
    """Rows of the longest bin taken by x-panel tiles (long_lds 3), both
    dtypes: several panels and a partial last one, rows that skip panels,
    one row with all its entries in one panel, mixed row lengths (blocks of
    different lanes per row); inside the binned CSR kernel and the column
    panels, repeatable bit for bit, and in both batch modes.  Tiles that
    would cost too much fall back to x chunks (float64) or the binned launch."""
    import torch
    from paper_1210_2536_amd.spmv import Batch, Plan
    rng = np.random.default_rng(86)
    band = S.random_csr(rng, 400, 40_000, 0.01)                      # 400 per row, 5 f64 panels
    band.col[band.row_ptr[7]:band.row_ptr[8]] = np.arange(band.row_ptr[8] - band.row_ptr[7],
                                                          dtype=np.int32)   # row 7 in panel 0
    mats = [S.random_csr(rng, 300, 17_000, 0.02),                   # 340 per row
            S.zipf_g2(np.random.default_rng([86, 0]), 30_000),
            band]
    for i, A in enumerate(mats):
        x = np.random.default_rng([87, i]).uniform(-1, 1, A.n)
        for dt in (np.float64, np.float32):
            rp, col, val = dev(A, dt)
            for k, extra in (("csr_adaptive", {}), ("csr_panel", {"panel_kib": 16}),
                             ("csr_panel", {"panel_kib": 16, "panel_xcd": 2})):
                note(f"[long tiles] {A.name} {np.dtype(dt).name} {k} {extra}")
                p = Plan(rp, col, val, n=A.n, selector=k,
                         params=dict(extra, long_lds=3, adaptive_wg_min=64))
                info = p.info()
                assert info["params"]["long_lds"] == 3, (A.name, info["params"]["long_lds"])
                assert info["long_rows"] > 0 and info["long_lanes"] in (8, 16, 32, 64)
                y = p.run(vec(x, dt)).cpu().numpy()
                assert_parity(y, A, x, dt)
                y2 = p.run(vec(x, dt)).cpu().numpy()
                assert np.array_equal(y.view(np.uint8), y2.view(np.uint8))
                if k == "csr_adaptive":
                    for mode in (0, 1):
                        B = Batch([p], mode=mode)
                        yb = torch.full((A.m,), float("nan"), dtype=vec(x, dt).dtype,
                                        device="cuda")
                        B.run([vec(x, dt)], [yb])
                        torch.cuda.synchronize()
                        assert np.array_equal(yb.cpu().numpy().view(np.uint8), y.view(np.uint8))
                        B.close()
    # too many panels for the long rows' length: chunks (float64) or binned (float32)
    m, n, k = 200, 3_000_000, 120                                   # 367 float64 panels
    cols = np.concatenate([np.sort(rng.choice(n, k, replace=False)) for _ in range(m)])
    A = S.CSR(m, n, np.arange(0, m * k + 1, k, dtype=np.int64), cols.astype(np.int32),
              rng.uniform(-1, 1, m * k), "rand_200x3M")
    x = np.random.default_rng(88).uniform(-1, 1, A.n)
    for dt, want in ((np.float64, 1), (np.float32, 2)):
        rp, col, val = dev(A, dt)
        p = Plan(rp, col, val, n=A.n, selector="csr_adaptive",
                 params={"long_lds": 3, "adaptive_wg_min": 64})
        assert p.info()["params"]["long_lds"] == want
        assert_parity(p.run(vec(x, dt)).cpu().numpy(), A, x, dt)


def test_long_rows_default_mode():
    """Default: tiles take the rows longer than 1024 when there are at least
    1024 of them; with fewer, the binned launch keeps its own threshold
    (rows up to adaptive_wg_min with 64 lanes each), and both give the
    oracle's result."""
    from paper_1210_2536_amd.spmv import Plan
    rng = np.random.default_rng(89)
    n = 50_000

    def mat(n_long, n_short):
        lens = np.concatenate([rng.integers(1100, 3000, n_long), rng.integers(1, 40, n_short)])
        rng.shuffle(lens)
        cols = [np.sort(rng.choice(n, k, replace=False)) for k in lens]
        rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
        return S.CSR(len(lens), n, rp, np.concatenate(cols).astype(np.int32),
                     rng.uniform(-1, 1, int(rp[-1])), f"long{n_long}")
    for A, want in ((mat(2100, 3000), 3), (mat(300, 3000), 2)):
        x = np.random.default_rng(90).uniform(-1, 1, A.n)
        for dt in (np.float64, np.float32):
            for k in ("csr_adaptive", "csr_panel"):
                note(f"[long default] {A.name} {np.dtype(dt).name} {k}")
                rp, col, val = dev(A, dt)
                p = Plan(rp, col, val, n=A.n, selector=k)
                info = p.info()
                assert info["params"]["long_lds"] == want, (A.name, k, info["params"]["long_lds"])
                assert info["long_rows"] == (2100 if want == 3 else 0)
                assert_parity(p.run(vec(x, dt)).cpu().numpy(), A, x, dt)


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
def test_panel_short_bins_direct(dtype):
    """Column panels with the shortest length bins summed by the binned
    kernel without panels (params.panel_direct_max): rows of at most 4, 16
    or 64 entries direct, the others in the panels (one launch or one per
    panel), the longest ones by tiles or x chunks; on the 7-point stencil
    every row is direct from 16 on and the panel launch is empty.  Each
    output matches the oracle and repeats bit for bit."""
    from paper_1210_2536_amd.spmv import Plan
    mats = [S.zipf_g2(np.random.default_rng([88, 0]), 30_000),
            S.uniform_g1(np.random.default_rng([88, 1]), 12_000),
            S.stencil_7pt(16)]
    for i, A in enumerate(mats):
        x = np.random.default_rng([89, i]).uniform(-1, 1, A.n)
        rp, col, val = dev(A, dtype)
        xd = vec(x, dtype)
        for d in (4, 16, 64):
            for extra in ({"panel_kib": 16}, {"panel_kib": 16, "panel_xcd": 2},
                          {"panel_kib": 16, "long_lds": 3, "adaptive_wg_min": 64}):
                prm = dict(extra, panel_direct_max=d)
                note(f"[panel direct] {A.name} {np.dtype(dtype).name} {prm}")
                p = Plan(rp, col, val, n=A.n, selector="csr_panel", params=prm)
                assert p.info()["params"]["panel_direct_max"] == d
                y = p.run(xd).cpu().numpy()
                assert_parity(y, A, x, dtype)
                y2 = p.run(xd).cpu().numpy()
                assert np.array_equal(y.view(np.uint8), y2.view(np.uint8))
                p.close()
