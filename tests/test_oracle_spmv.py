"""Pins of the CPU SpMV oracle to things other than itself (CPU only).

* exact rational brute force on tiny matrices of every generator,
* long single rows against an exact rational sum,
* closed-form actions of integer stencils on polynomial vectors (exact in any
  summation order),
* the Galerkin coarse-level closed form A_l = 27 8^l I - B_l (x) B_l (x) B_l,
* special matrices (identity, permutation, diagonal, empty rows, one column,
  rectangular).
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import spmv as O
from paper_1210_2536_amd import synth as S

U64 = 2.0 ** -53


def _check_exact(A, x, slack=1e-15):
    y, absax = O.spmv_accurate(A.row_ptr, A.col, A.val, x)
    ex = O.spmv_dense_exact(A.row_ptr, A.col, A.val, x)
    for i, e in enumerate(ex):
        err = abs(Fraction(float(y[i])) - e)
        bound = Fraction(2 * U64) * abs(e) + Fraction(slack) * Fraction(float(absax[i]))
        assert err <= bound, (A.name, i, float(err), float(bound))
    # the brute-force dense product agrees to rounding as well
    dense = np.zeros((A.m, A.n))
    rows = np.repeat(np.arange(A.m), np.diff(A.row_ptr))
    dense[rows, A.col] = A.val
    np.testing.assert_allclose(y, dense @ x, rtol=0, atol=1e-13 * max(1.0, absax.max(initial=0)))
    return y, absax


def _tiny_matrices():
    rng = np.random.default_rng(123)
    mats = [S.stencil_5pt(5), S.stencil_7pt(3), S.stencil_27pt(3)]
    mats.append(S.band_g0(np.random.default_rng([9, 1]), 40))
    mats.append(S.uniform_g1(np.random.default_rng([9, 2]), 70))
    mats.append(S.zipf_g2(np.random.default_rng([9, 3]), 60))
    mats.append(S.blocks_g3(np.random.default_rng([9, 4]), 48))
    mats.append(S.random_csr(rng, 17, 23, 0.3, explicit_zeros=True))
    mats.append(S.random_csr(rng, 9, 4, 0.5))
    return mats


@pytest.mark.parametrize("A", _tiny_matrices(), ids=lambda A: A.name)
def test_tiny_vs_exact_rational(A):
    x = S.uniform_vector(A.n, [7, A.m])
    _check_exact(A, x)
    # float32-representable data, widened exactly, behaves the same way
    Af = A.astype(np.float32).astype(np.float64)
    _check_exact(Af, x.astype(np.float32).astype(np.float64))


@pytest.mark.parametrize("k", [1000, 10_000, 100_000])
def test_long_row_accuracy(k):
    rng = np.random.default_rng([11, k])
    n = 2 * k
    cols = np.sort(rng.choice(n, size=k, replace=False)).astype(np.int32)
    # wide dynamic range and cancellation make naive summation visibly wrong
    val = rng.uniform(-1, 1, k) * np.exp2(rng.integers(-30, 30, k))
    x = rng.uniform(-1, 1, n)
    rp = np.array([0, k], dtype=np.int64)
    y, absax = O.spmv_accurate(rp, cols, val, x)
    exact = sum((Fraction(float(a)) * Fraction(float(x[c])) for a, c in zip(val, cols)), Fraction(0))
    err = abs(Fraction(float(y[0])) - exact)
    # compensated summation: u |y| plus a second-order term in k u^2 sum|a x|
    bound = Fraction(2 * U64) * abs(exact) + Fraction(4 * k) * Fraction(U64) ** 2 * Fraction(float(absax[0]))
    assert err <= bound
    # and a naive float64 sum of the same products is measurably worse here
    naive = 0.0
    for a, c in zip(val, cols):
        naive += a * x[c]
    assert abs(Fraction(naive) - exact) >= err


def _grid_coords(shape):
    return [c.ravel().astype(np.int64) for c in np.indices(shape)]


def test_5pt_closed_forms():
    g = 64
    A = S.stencil_5pt(g)
    i, j = _grid_coords((g, g))
    interior = (i > 0) & (i < g - 1) & (j > 0) & (j < g - 1)
    # x = i^2 + j^2: the discrete Laplacian of a quadratic is constant (-4)
    y, _ = O.spmv_accurate(A.row_ptr, A.col, A.val, (i * i + j * j).astype(np.float64))
    assert np.all(y[interior] == -4.0)
    assert y[0] == -2.0
    assert np.abs(y).max() == 16126.0
    # linear x is annihilated at interior points
    y, _ = O.spmv_accurate(A.row_ptr, A.col, A.val, (3 * i - 5 * j + 7).astype(np.float64))
    assert np.all(y[interior] == 0.0)
    # x = 1 counts the missing neighbours
    missing = (i == 0).astype(int) + (i == g - 1) + (j == 0) + (j == g - 1)
    y, _ = O.spmv_accurate(A.row_ptr, A.col, A.val, np.ones(g * g))
    assert np.array_equal(y, missing.astype(np.float64))


@pytest.mark.parametrize("kind", ["7pt", "27pt"])
def test_3d_stencil_closed_forms(kind):
    g = 12
    A = S.stencil_7pt(g) if kind == "7pt" else S.stencil_27pt(g)
    i, j, k = _grid_coords((g, g, g))
    interior = (i > 0) & (i < g - 1) & (j > 0) & (j < g - 1) & (k > 0) & (k < g - 1)
    x = (i * i + j * j + k * k).astype(np.float64)
    y, _ = O.spmv_accurate(A.row_ptr, A.col, A.val, x)
    # sum of squared displacements over the stencil: 2 per axis (7pt), 18 per axis (27pt)
    assert np.all(y[interior] == (-6.0 if kind == "7pt" else -54.0))
    y, _ = O.spmv_accurate(A.row_ptr, A.col, A.val, (2 * i - j + 4 * k).astype(np.float64))
    assert np.all(y[interior] == 0.0)
    y, _ = O.spmv_accurate(A.row_ptr, A.col, A.val, np.ones(g ** 3))
    if kind == "7pt":
        missing = sum(((c == 0).astype(int) + (c == g - 1)) for c in (i, j, k))
    else:
        # neighbours in a 3x3x3 box: product of per-axis in-range counts
        per = [3 - (c == 0) - (c == g - 1) for c in (i, j, k)]
        missing = 27 - per[0] * per[1] * per[2]
    assert np.array_equal(y, missing.astype(np.float64))


def _tridiag(g, d):
    import scipy.sparse as sp
    return sp.diags([np.ones(g - 1), np.full(g, float(d)), np.ones(g - 1)], [-1, 0, 1])


def test_galerkin_levels_closed_form_and_tensor_action():
    import scipy.sparse as sp
    g0 = 16
    levels = S.multilevel(g0, 4)
    g = g0
    for l, A in enumerate(levels):
        B = _tridiag(g, 3 * 2 ** l - 2)
        ref = (27 * 8 ** l) * sp.identity(g ** 3) - sp.kron(B, sp.kron(B, B))
        ref = ref.tocsr()
        ref.sum_duplicates(); ref.eliminate_zeros(); ref.sort_indices()
        assert np.array_equal(ref.indptr, A.row_ptr)
        assert np.array_equal(ref.indices, A.col)
        assert np.array_equal(ref.data, A.val)
        assert A.nnz == (3 * g - 2) ** 3
        # exact action on a tensor-product vector of small integers
        rng = np.random.default_rng([13, l])
        u, v, w = (rng.integers(-4, 5, g).astype(np.float64) for _ in range(3))
        x = np.kron(u, np.kron(v, w))
        Bd = B.toarray()
        expect = (27 * 8 ** l) * x - np.kron(Bd @ u, np.kron(Bd @ v, Bd @ w))
        y, _ = O.spmv_accurate(A.row_ptr, A.col, A.val, x)
        assert np.array_equal(y, expect)
        g //= 2


def test_special_matrices():
    rng = np.random.default_rng(5)
    n = 257
    x = rng.uniform(-1, 1, n)
    eye_rp = np.arange(n + 1, dtype=np.int64)
    # identity: y = x bit for bit
    y, _ = O.spmv_accurate(eye_rp, np.arange(n, dtype=np.int32), np.ones(n), x)
    assert np.array_equal(y, x)
    # permutation
    perm = rng.permutation(n).astype(np.int32)
    y, _ = O.spmv_accurate(eye_rp, perm, np.ones(n), x)
    assert np.array_equal(y, x[perm])
    # diagonal: one correctly rounded product per row
    d = rng.uniform(-3, 3, n)
    y, _ = O.spmv_accurate(eye_rp, np.arange(n, dtype=np.int32), d, x)
    assert np.array_equal(y, d * x)
    # all-empty rows give +0
    y, a = O.spmv_accurate(np.zeros(n + 1, dtype=np.int64), np.zeros(0, np.int32), np.zeros(0), x)
    assert np.all(y == 0) and not np.any(np.signbit(y)) and np.all(a == 0)
    # single column, rectangular m != n
    m = 31
    rp = np.arange(m + 1, dtype=np.int64)
    y, _ = O.spmv_accurate(rp, np.zeros(m, np.int32), np.arange(m, dtype=np.float64), np.array([2.5]))
    assert np.array_equal(y, 2.5 * np.arange(m))


def test_plain_mode_matches_and_is_thread_count_independent():
    A = S.zipf_g2(np.random.default_rng([9, 30]), 20_000)
    x = S.uniform_vector(A.n, 3)
    y_acc, absax = O.spmv_accurate(A.row_ptr, A.col, A.val, x)
    y1 = O.spmv_plain(A.row_ptr, A.col, A.val, x, nthreads=1)
    y4 = O.spmv_plain(A.row_ptr, A.col, A.val, x, nthreads=4)
    assert np.array_equal(y1, y4)
    kmax = int(np.diff(A.row_ptr).max())
    assert np.all(np.abs(y1 - y_acc) <= (kmax + 1) * 1.2e-16 * absax + 1e-300)


def test_rows_subset_matches_full():
    A = S.uniform_g1(np.random.default_rng([9, 31]), 5000)
    x = S.uniform_vector(A.n, 4)
    y, a = O.spmv_accurate(A.row_ptr, A.col, A.val, x)
    rows = np.array([0, 17, 4999, 2500])
    ys, as_ = O.spmv_rows(A.row_ptr, A.col, A.val, x, rows)
    assert np.array_equal(ys, y[rows]) and np.array_equal(as_, a[rows])


def test_plain_f32_mode_rounds_the_float64_sum_once():
    """The float32-storage plain mode: float32 values and x, float64 sums,
    each row rounded once.  Pinned by the exact product on the same widened
    data (error <= 2^-24 |y| + the float64 chain's, far below 2e-6 (|A||x|)),
    by exact integer stencils (bitwise) and by thread-count independence."""
    A = S.zipf_g2(np.random.default_rng([9, 32]), 20_000)
    x = S.uniform_vector(A.n, 5).astype(np.float32)
    v32 = A.val.astype(np.float32)
    y_acc, absax = O.spmv_accurate(A.row_ptr, A.col, v32.astype(np.float64), x.astype(np.float64))
    y1 = O.spmv_plain_f32(A.row_ptr, A.col, v32, x, nthreads=1)
    y3 = O.spmv_plain_f32(A.row_ptr, A.col, v32, x, nthreads=3)
    assert y1.dtype == np.float32 and np.array_equal(y1, y3)
    kmax = int(np.diff(A.row_ptr).max())
    err = np.abs(y1.astype(np.float64) - y_acc)
    assert np.all(err <= 2.0 ** -24 * np.abs(y_acc) + (kmax + 1) * 1.2e-16 * absax + 1e-300)
    # 7-point stencil on i^2 + j^2 + k^2: integers, exact in float32 storage
    g = 12
    B = S.stencil_7pt(g)
    r = np.arange(B.n)
    i, j, k = r // (g * g), (r // g) % g, r % g
    xp = (i * i + j * j + k * k).astype(np.float32)
    yb = O.spmv_plain_f32(B.row_ptr, B.col, B.val.astype(np.float32), xp)
    ref, _ = O.spmv_accurate(B.row_ptr, B.col, B.val, xp.astype(np.float64))
    assert np.array_equal(yb.astype(np.float64), ref)
