"""Seeded synthetic sparse matrices and vectors.

This module only *generates inputs*: it builds CSR matrices and dense vectors
from ``numpy.random.default_rng`` (PCG64) seeds.  It contains none of the
SpMV method's arithmetic (no products, no format conversion, no features), so
both the independent CPU oracle and the GPU path can consume what it makes.

The paper measured on the UF (SuiteSparse) collection (Section 2.2, Table 1),
which is not available here.  The generators below stand in for it; they span
the structural classes the paper's parameters key on (Section 4, Table 3):

* G0 banded / stencil matrices (DIA-like: few, full diagonals),
* G1 uniform-k random rows (ELL-like: constant row degree),
* G2 Zipf row degrees (COO-like: power-law degrees, Section 4 on R),
* G3 dense 4x4 blocks (block structure, Section 2.1 on blocked formats),

plus the closed-form PDE stencils and AMG-style Galerkin coarse levels
(Section 1 motivates AMG level matrices).

Every CSR returned is canonical: ``row_ptr`` int64 of length m+1, ``col``
int32 strictly increasing inside each row, ``val`` float64.  The float32
version of a matrix is the rounded cast of the same float64 draw.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "CSR", "stencil_5pt", "stencil_7pt", "stencil_27pt", "galerkin_coarsen",
    "multilevel", "band_g0", "uniform_g1", "zipf_g2", "blocks_g3",
    "sweep_matrix", "selector_matrix", "zipf_large", "laplace_7pt_large",
    "uniform_vector", "SWEEP_SIZE", "GEN_NAMES",
]

GEN_NAMES = ("band", "uniform", "zipf", "blocks")
SWEEP_SIZE = 200


@dataclass
class CSR:
    m: int
    n: int
    row_ptr: np.ndarray  # int64[m+1]
    col: np.ndarray      # int32[nnz]
    val: np.ndarray      # float64[nnz]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def astype(self, dtype) -> "CSR":
        return CSR(self.m, self.n, self.row_ptr, self.col,
                   self.val.astype(dtype), self.name)


def _finish(m, n, row_len, col, val, name):
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(row_len, out=row_ptr[1:])
    return CSR(int(m), int(n), row_ptr, col.astype(np.int32, copy=False),
               val, name)


# ---------------------------------------------------------------------------
# structured grids
# ---------------------------------------------------------------------------

def _grid_stencil(shape, offsets, values, name):
    """CSR of a constant-coefficient stencil on a row-major grid, Dirichlet.

    ``offsets`` are per-axis displacement tuples; a coupling exists only when
    the neighbour lies inside the grid (no wrap-around).  Columns come out in
    ascending order because the offsets are visited in ascending linear order.
    """
    shape = tuple(int(s) for s in shape)
    m = int(np.prod(shape))
    strides = [int(np.prod(shape[a + 1:])) for a in range(len(shape))]
    lin = [sum(o[a] * strides[a] for a in range(len(shape))) for o in offsets]
    order = np.argsort(lin, kind="stable")
    coords = np.indices(shape).reshape(len(shape), -1)
    rows = np.arange(m, dtype=np.int64)
    masks = []
    for o in offsets:
        ok = np.ones(m, dtype=bool)
        for a, d in enumerate(o):
            if d:
                c = coords[a] + d
                ok &= (c >= 0) & (c < shape[a])
        masks.append(ok)
    row_len = np.zeros(m, dtype=np.int64)
    for ok in masks:
        row_len += ok
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(row_len, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    pos = row_ptr[:-1].copy()
    for k in order:
        ok = masks[k]
        p = pos[ok]
        col[p] = (rows[ok] + lin[k]).astype(np.int32)
        val[p] = values[k]
        pos[ok] += 1
    return CSR(m, m, row_ptr, col, val, name)


def stencil_5pt(g: int) -> CSR:
    """2-D 5-point Laplacian on a g x g grid, values 4 / -1, row r = g*i + j."""
    offs = [(0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)]
    vals = [4.0, -1.0, -1.0, -1.0, -1.0]
    return _grid_stencil((g, g), offs, vals, f"lap5_{g}x{g}")


def stencil_7pt(g: int) -> CSR:
    """3-D 7-point Laplacian on g^3, values 6 / -1, row r = (i*g + j)*g + k."""
    offs = [(0, 0, 0)] + [tuple(s * (a == b) for b in range(3))
                          for a in range(3) for s in (-1, 1)]
    vals = [6.0] + [-1.0] * 6
    return _grid_stencil((g, g, g), offs, vals, f"lap7_{g}^3")


def stencil_27pt(g: int) -> CSR:
    """3-D 27-point stencil on g^3, values 26 (centre) / -1 (26 neighbours)."""
    offs = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)]
    vals = [26.0 if o == (0, 0, 0) else -1.0 for o in offs]
    return _grid_stencil((g, g, g), offs, vals, f"lap27_{g}^3")


def galerkin_coarsen(A: CSR, g: int) -> CSR:
    """A_c = P^T A P for 2x2x2 aggregation on a g^3 grid (g even).

    P is the 0/1 piecewise-constant prolongation: fine point (i,j,k) belongs
    to coarse point (i//2, j//2, k//2).  Each fine nonzero (r, c, v) is
    re-indexed to (agg r, agg c, v) and duplicates are summed; with integer
    entries this sum is exact in float64.
    """
    import scipy.sparse as sp

    assert g % 2 == 0
    gc = g // 2
    idx = np.arange(A.m, dtype=np.int64)
    i, rem = np.divmod(idx, g * g)
    j, k = np.divmod(rem, g)
    agg = ((i // 2) * gc + (j // 2)) * gc + (k // 2)
    rows = np.repeat(agg, np.diff(A.row_ptr))
    cols = agg[A.col.astype(np.int64)]
    mc = gc ** 3
    C = sp.coo_matrix((A.val, (rows, cols)), shape=(mc, mc)).tocsr()
    C.sum_duplicates()
    C.sort_indices()
    return CSR(mc, mc, C.indptr.astype(np.int64), C.indices.astype(np.int32),
               C.data.astype(np.float64), f"galerkin_{gc}^3")


def multilevel(g0: int = 160, nlevels: int = 6) -> list:
    """27-point matrix on g0^3 plus nlevels-1 Galerkin coarse levels."""
    levels = [stencil_27pt(g0)]
    g = g0
    for _ in range(nlevels - 1):
        levels.append(galerkin_coarsen(levels[-1], g))
        g //= 2
    return levels


# ---------------------------------------------------------------------------
# random rows
# ---------------------------------------------------------------------------

def _sorted_distinct_cols(rng, row_len: np.ndarray, n: int) -> np.ndarray:
    """For each row i draw row_len[i] distinct columns of [0, n), ascending.

    Sorted uniforms are taken from normalised exponential spacings (no sort
    needed); v_k = floor(U_(k) * (n - L + 1)) is non-decreasing in
    [0, n-L] and c_k = v_k + k is then strictly increasing in [0, n-1].
    """
    row_len = np.asarray(row_len, dtype=np.int64)
    m = row_len.size
    nnz = int(row_len.sum())
    if nnz == 0:
        return np.zeros(0, dtype=np.int32)
    assert int(row_len.max()) <= n
    seg = row_len + 1
    seg_start = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(seg, out=seg_start[1:])
    e = rng.standard_exponential(int(seg_start[-1]))
    np.cumsum(e, out=e)
    base = np.zeros(m, dtype=np.float64)
    base[1:] = e[seg_start[1:-1] - 1]
    total = e[seg_start[1:] - 1] - base
    # drop the last spacing of every row: keep the first L partial sums
    keep = np.ones(e.size, dtype=bool)
    keep[seg_start[1:] - 1] = False
    part = e[keep]
    rowid = np.repeat(np.arange(m, dtype=np.int64), row_len)
    u = (part - base[rowid]) / total[rowid]
    span = (n - row_len + 1)[rowid]
    v = np.minimum(np.floor(u * span).astype(np.int64), span - 1)
    starts = np.repeat(np.cumsum(row_len) - row_len, row_len)
    k = np.arange(nnz, dtype=np.int64) - starts
    return (v + k).astype(np.int32)


def _uniform_vals(rng, count):
    return rng.uniform(-1.0, 1.0, size=count)


def band_g0(rng, n: int) -> CSR:
    """G0: banded stencil with D ~ U{3..15} diagonals, every in-range slot set."""
    D = int(rng.integers(3, 16))
    if D % 2 == 1 and rng.random() < 0.5:
        h = (D - 1) // 2
        offs = list(range(-h, h + 1))
    else:
        g = int(round(n ** (1.0 / 3.0))) if D > 9 else int(round(math.sqrt(n)))
        g = max(g, 3)
        cand = [0, 1, -1, g, -g, g + 1, -(g + 1), g - 1, -(g - 1),
                g * g, -g * g, 2, -2, 2 * g, -2 * g]
        offs = []
        for o in cand:
            if o not in offs and -n < o < n:
                offs.append(o)
            if len(offs) == D:
                break
    offs = sorted(offs)
    rows = np.arange(n, dtype=np.int64)
    masks = [(rows + o >= 0) & (rows + o < n) for o in offs]
    row_len = np.zeros(n, dtype=np.int64)
    for mk in masks:
        row_len += mk
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(row_len, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    col = np.empty(nnz, dtype=np.int32)
    pos = row_ptr[:-1].copy()
    for o, mk in zip(offs, masks):
        col[pos[mk]] = (rows[mk] + o).astype(np.int32)
        pos[mk] += 1
    val = _uniform_vals(rng, nnz)
    return CSR(n, n, row_ptr, col, val, f"band_D{D}_n{n}")


def uniform_g1(rng, n: int) -> CSR:
    """G1: every row holds k ~ U{8..64} distinct uniform columns."""
    k = int(rng.integers(8, 65))
    k = min(k, n)
    row_len = np.full(n, k, dtype=np.int64)
    col = _sorted_distinct_cols(rng, row_len, n)
    val = _uniform_vals(rng, col.size)
    return _finish(n, n, row_len, col, val, f"uniform_k{k}_n{n}")


def zipf_g2(rng, n: int) -> CSR:
    """G2: row degrees min(Zipf(alpha), n//10), alpha ~ U(1.5, 2.5)."""
    alpha = float(rng.uniform(1.5, 2.5))
    cap = max(1, n // 10)
    row_len = np.minimum(rng.zipf(alpha, size=n), cap).astype(np.int64)
    col = _sorted_distinct_cols(rng, row_len, n)
    val = _uniform_vals(rng, col.size)
    return _finish(n, n, row_len, col, val, f"zipf_a{alpha:.2f}_n{n}")


def blocks_g3(rng, n: int) -> CSR:
    """G3: dense 4x4 blocks, b = clamp(round(0.01 n / 4), 1, 16) per block row."""
    n4 = ((n + 3) // 4) * 4
    nb = n4 // 4
    b = int(min(16, max(1, round(0.01 * n4 / 4))))
    b = min(b, nb)
    bcols = _sorted_distinct_cols(rng, np.full(nb, b, dtype=np.int64), nb)
    bcols = bcols.reshape(nb, b).astype(np.int64)
    # row r = 4*br + t holds, for each of its block row's blocks, 4 columns
    cols = (bcols[:, None, :, None] * 4 + np.arange(4)[None, None, None, :])
    cols = np.broadcast_to(cols, (nb, 4, b, 4)).reshape(-1)
    row_len = np.full(n4, 4 * b, dtype=np.int64)
    val = _uniform_vals(rng, cols.size)
    return _finish(n4, n4, row_len, cols.astype(np.int32), val,
                   f"blocks_b{b}_n{n4}")


_GENS = (band_g0, uniform_g1, zipf_g2, blocks_g3)


def sweep_matrix(k: int) -> CSR:
    """Matrix k of the 200-matrix sweep: generator k mod 4, n = 10^U(3,6)."""
    rng = np.random.default_rng([2, k])
    n = int(round(10 ** rng.uniform(3.0, 6.0)))
    A = _GENS[k % 4](rng, n)
    A.name = f"sweep{k}_{A.name}"
    return A


def selector_matrix(i: int, heldout: bool = False, nnz_cap: int = 30_000_000,
                    n_hi: float = 6.0) -> CSR:
    """Matrix i of the selector set (train seeds [3, i], held-out [3, 1e6+i]).

    Same generators and n range as the sweep; a draw whose nnz exceeds
    ``nnz_cap`` is redrawn from the same stream so labelling stays bounded.
    """
    seed = [3, (1_000_000 + i) if heldout else i]
    rng = np.random.default_rng(seed)
    while True:
        n = int(round(10 ** rng.uniform(3.0, n_hi)))
        A = _GENS[i % 4](rng, n)
        if A.nnz <= nnz_cap:
            A.name = f"sel{'H' if heldout else 'T'}{i}_{A.name}"
            return A


def zipf_large(n: int = 8_000_000, kmax: int = 800_000, seed=(5, 0)) -> CSR:
    """Row degrees floor(k), p(k) ~ k^-2 on [2, kmax] by inverse CDF."""
    rng = np.random.default_rng(list(seed))
    u = rng.random(n)
    a, b = 0.5, 1.0 / kmax
    k = 1.0 / (a - u * (a - b))
    row_len = np.minimum(np.floor(k).astype(np.int64), kmax)
    row_len = np.minimum(row_len, n)
    col = _sorted_distinct_cols(rng, row_len, n)
    val = _uniform_vals(rng, col.size)
    return _finish(n, n, row_len, col, val, f"zipf2_n{n}")


def mixed_stencil_zipf(g: int = 128, kmax: int = 20_000, seed=(6, 0)) -> CSR:
    """Two halves of one square matrix, n = 2 g^3: rows [0, g^3) are the
    7-point Laplacian on g^3 (6 / -1, columns in the first half), rows
    [g^3, 2 g^3) have degrees floor(k), p(k) ~ k^-2 on [2, kmax], with
    distinct uniform columns over all n.  No single format suits both
    halves (the random half makes DIA and ELL infeasible)."""
    rng = np.random.default_rng(list(seed))
    S1 = stencil_7pt(g)
    h = S1.m
    n = 2 * h
    u = rng.random(h)
    a, b = 0.5, 1.0 / kmax
    row_len2 = np.minimum(np.floor(1.0 / (a - u * (a - b))).astype(np.int64), kmax)
    col2 = _sorted_distinct_cols(rng, row_len2, n)
    val2 = _uniform_vals(rng, col2.size)
    row_len = np.concatenate([np.diff(S1.row_ptr), row_len2])
    col = np.concatenate([S1.col, col2]).astype(np.int32)
    val = np.concatenate([S1.val.astype(np.float64), val2])
    return _finish(n, n, row_len, col, val, f"mixed_lap7_{g}^3+zipf2")


def laplace_7pt_large(g: int = 256) -> CSR:
    return stencil_7pt(g)


def uniform_vector(n: int, seed) -> np.ndarray:
    """x uniform[-1, 1] in float64 from ``default_rng(seed)``."""
    rng = np.random.default_rng(seed if isinstance(seed, int) else list(seed))
    return rng.uniform(-1.0, 1.0, size=n)


def random_csr(rng, m: int, n: int, density: float, explicit_zeros=False) -> CSR:
    """Small random canonical CSR (used for edge-case tests)."""
    mask = rng.random((m, n)) < density
    row_len = mask.sum(axis=1).astype(np.int64)
    rr, cc = np.nonzero(mask)
    val = rng.uniform(-1.0, 1.0, size=rr.size)
    if explicit_zeros and val.size:
        z = rng.random(val.size) < 0.2
        val[z] = 0.0
    return _finish(m, n, row_len, cc.astype(np.int32), val, f"rand_{m}x{n}")
