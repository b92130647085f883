"""Exact integer cases on the GPU: every kernel must reproduce the oracle bit
for bit.

Every format re-encodes the same stored entries (Section 2.1), so on inputs
whose partial sums are all integers below 2^24 the product is exact in any
summation order, in float32 as in float64 (the float32 kernels accumulate in
float64 and round once; an integer below 2^24 survives that rounding):

* the 7-point (6 / -1) and 27-point (26 / -1) Laplacians on x = i^2 + j^2 +
  k^2, whose action is -6 and -54 at interior grid points;
* the 2x2x2-aggregation Galerkin coarse levels of the 27-point operator on
  tensor-product integer vectors u (x) v (x) w, whose action has the closed
  form A_l (u (x) v (x) w) = 27 8^l u (x) v (x) w - (B_l u) (x) (B_l v) (x)
  (B_l w), B_l = tridiag(1, 3 2^l - 2, 1) of the level's grid size.

Each kernel runs with its default launch shape and, for DIA / ELL, with the
16-byte wide form; the column-panel kernel also with many small panels in
both modes.  The GPU output is compared with np.array_equal against the
oracle, and the oracle against the closed form.
"""
import numpy as np
import pytest

from oracle import spmv as O
from paper_1210_2536_amd import synth as S

from gpu_util import dev, note, vec
from test_gpu_parity import KERNELS, _feasible

pytestmark = pytest.mark.gpu

DTYPES = (np.float64, np.float32)


def _variants(kernel, n, elt):
    out = [None]
    if kernel in ("dia", "dia_direct", "ell"):
        out.append({"wide_loads": 1})
    if kernel == "csr_panel":
        kib = max(1, (n * elt) // (24 * 1024))   # about 24 panels of x
        out += [{"panel_kib": kib, "panel_xcd": 1}, {"panel_kib": kib, "panel_xcd": 2}]
    return out


def _all_kernels_bitwise(A, x, ref):
    from paper_1210_2536_amd.spmv import Plan
    ran = 0
    for dt in DTYPES:
        rp, col, val = dev(A, dt)
        # the matrix and vector are integers, exact in float32
        assert np.array_equal(A.val.astype(dt).astype(np.float64), A.val)
        assert np.array_equal(x.astype(dt).astype(np.float64), x)
        xd = vec(x, dt)
        for k in KERNELS:
            if not _feasible(A, k):
                continue
            for prm in _variants(k, A.n, np.dtype(dt).itemsize):
                note(f"[exact] {A.name} {np.dtype(dt).name} {k} {prm or ''}")
                p = Plan(rp, col, val, n=A.n, selector=k, params=prm)
                y = p.run(xd).cpu().numpy().astype(np.float64)
                bad = np.nonzero(y != ref)[0]
                assert bad.size == 0, (A.name, np.dtype(dt).name, k, prm, bad[:5], y[bad[:5]],
                                       ref[bad[:5]])
                p.close()
                ran += 1
    return ran


def _grid(g):
    r = np.arange(g ** 3, dtype=np.int64)
    return r // (g * g), (r // g) % g, r % g


@pytest.mark.parametrize("g", [40], ids=["g40"])
def test_7pt_polynomial_bitwise(g):
    A = S.stencil_7pt(g)
    i, j, k = _grid(g)
    x = (i * i + j * j + k * k).astype(np.float64)
    ref, _ = O.spmv_accurate(A.row_ptr, A.col, A.val, x)
    inner = (i > 0) & (i < g - 1) & (j > 0) & (j < g - 1) & (k > 0) & (k < g - 1)
    assert np.all(ref[inner] == -6.0)
    assert _all_kernels_bitwise(A, x, ref) >= 2 * len(KERNELS)


@pytest.mark.parametrize("g", [30], ids=["g30"])
def test_27pt_polynomial_bitwise(g):
    A = S.stencil_27pt(g)
    i, j, k = _grid(g)
    x = (i * i + j * j + k * k).astype(np.float64)
    ref, _ = O.spmv_accurate(A.row_ptr, A.col, A.val, x)
    inner = (i > 0) & (i < g - 1) & (j > 0) & (j < g - 1) & (k > 0) & (k < g - 1)
    assert np.all(ref[inner] == -54.0)
    # linear x: the interior action vanishes
    xl = (3 * i - 2 * j + k).astype(np.float64)
    refl, _ = O.spmv_accurate(A.row_ptr, A.col, A.val, xl)
    assert np.all(refl[inner] == 0.0)
    assert _all_kernels_bitwise(A, x, ref) >= 2 * len(KERNELS)
    _all_kernels_bitwise(A, xl, refl)


def _tridiag_apply(u, d):
    out = d * u
    out[1:] += u[:-1]
    out[:-1] += u[1:]
    return out


def test_galerkin_levels_tensor_vectors_bitwise():
    g0 = 32
    levels = S.multilevel(g0, 5)
    rng = np.random.default_rng([42, 0])
    for l, A in enumerate(levels):
        g = g0 >> l
        assert A.m == g ** 3
        u, v, w = (rng.choice(np.array([-3, -2, -1, 1, 2, 3], np.int64), size=g)
                   for _ in range(3))
        x = np.kron(u, np.kron(v, w)).astype(np.float64)
        d = 3 * 2 ** l - 2
        closed = 27 * 8 ** l * np.kron(u, np.kron(v, w)) - np.kron(
            _tridiag_apply(u, d), np.kron(_tridiag_apply(v, d), _tridiag_apply(w, d)))
        ref, absax = O.spmv_accurate(A.row_ptr, A.col, A.val, x)
        assert np.all(absax < 2 ** 24) and np.all(absax > 0)
        assert np.array_equal(ref, closed.astype(np.float64)), l
        A.name = f"galerkin27_{g0}^3_level{l}"
        _all_kernels_bitwise(A, x, ref)


def test_long_tiles_panel_boundaries_bitwise():
    """Long rows by x-panel tiles on integer data: every row holds the
    columns on both sides of every panel boundary (80 KB panels: 10240
    float64 or 20480 float32 values) plus random ones, so each tile entry's
    16-bit panel offset takes its extreme values 0 and W - 1.  The products
    and sums are integers far below 2^24, so y must equal the exact integer
    product bit for bit, in both dtypes, for the binned CSR kernel and the
    column panels, and for tiles from rows of 256, 1024 and 4096 entries."""
    from paper_1210_2536_amd.spmv import Plan
    rng = np.random.default_rng(1210)
    n = 30 * 20480 + 777         # many panels of either width, a partial last one, and
                                 # x above the 2 MiB the column panels need
    edges = np.unique(np.concatenate([np.arange(w, n, w) + d for w in (10240, 20480)
                                      for d in (-1, 0)]))
    edges = edges[(edges >= 0) & (edges < n)]
    lens = np.concatenate([rng.integers(300, 5000, 1200), rng.integers(1, 30, 4000)])
    rng.shuffle(lens)
    rows = []
    for k in lens:
        if k >= 300:
            extra = rng.choice(n, int(k), replace=False)
            c = np.union1d(np.concatenate([edges, [0, n - 1]]), extra)
        else:
            c = np.sort(rng.choice(n, int(k), replace=False))
        rows.append(c)
    rp = np.concatenate([[0], np.cumsum([len(c) for c in rows])]).astype(np.int64)
    col = np.concatenate(rows).astype(np.int32)
    val = rng.integers(-3, 4, col.size).astype(np.float64)
    A = S.CSR(len(rows), n, rp, col, val, "tile_edges")
    x = rng.integers(-4, 5, n).astype(np.float64)
    ref = np.zeros(A.m)
    for i in range(A.m):   # exact: integers well inside float64's 2^53
        ref[i] = float(np.dot(val[rp[i]:rp[i + 1]].astype(np.int64),
                              x[col[rp[i]:rp[i + 1]]].astype(np.int64)))
    assert np.abs(ref).max() < 2 ** 24
    for dt in DTYPES:
        rp_d, col_d, val_d = dev(A, dt)
        xd = vec(x, dt)
        for k in ("csr_adaptive", "csr_panel"):
            for trm in (256, 1024, 4096):
                note(f"[exact tiles] {np.dtype(dt).name} {k} tile_row_min={trm}")
                p = Plan(rp_d, col_d, val_d, n=A.n, selector=k,
                         params={"long_lds": 3, "tile_row_min": trm})
                assert p.info()["params"]["long_lds"] == 3
                assert p.info()["long_rows"] > 0
                y = p.run(xd).cpu().numpy().astype(np.float64)
                bad = np.nonzero(y != ref)[0]
                assert bad.size == 0, (np.dtype(dt).name, k, trm, bad[:5], y[bad[:5]], ref[bad[:5]])
                p.close()
