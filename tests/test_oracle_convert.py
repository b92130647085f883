"""Pins of the oracle's format layouts (CPU only).

Round trips CSR -> {COO, ELL, DIA, BCSR} -> CSR must be the identity bit for bit
(explicit +0.0 / -0.0 and NaN payloads included), and chosen slots of each
layout are checked against the dense matrix by their definitions.
"""
import numpy as np
import pytest

from oracle import convert as C
from paper_1210_2536_amd import synth as S


def _mats():
    out = [S.stencil_5pt(8), S.stencil_27pt(4)]
    for g, gen in enumerate((S.band_g0, S.uniform_g1, S.zipf_g2, S.blocks_g3)):
        out.append(gen(np.random.default_rng([21, g]), 300))
    rng = np.random.default_rng(3)
    out.append(S.random_csr(rng, 37, 53, 0.2, explicit_zeros=True))
    out.append(S.random_csr(rng, 50, 20, 0.3))
    out.append(_with_empty_rows(rng))
    return out


def _with_empty_rows(rng):
    m, n = 60, 45
    dense = (rng.random((m, n)) < 0.2) * rng.uniform(-1, 1, (m, n))
    dense[10:25] = 0.0
    dense[-3:] = 0.0
    rows, cols = np.nonzero(dense)
    rp = np.zeros(m + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=m), out=rp[1:])
    return S.CSR(m, n, rp, cols.astype(np.int32), dense[rows, cols], "empty_rows")


def _poison(val):
    """Replace some values by -0.0, +0.0 and NaNs with payloads."""
    v = val.copy()
    bits = v.view(np.uint64)
    if v.size >= 8:
        v[0] = -0.0
        v[1] = 0.0
        bits[2] = np.uint64(0x7FF0000000000001)   # signalling-pattern NaN
        bits[3] = np.uint64(0xFFF8DEADBEEF0001)   # negative quiet NaN, payload
    return v


def _same_bits(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return a.dtype == b.dtype and a.shape == b.shape and np.array_equal(
        a.view(np.uint8), b.view(np.uint8))


@pytest.mark.parametrize("A", _mats(), ids=lambda A: A.name)
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_round_trips_bit_exact(A, dtype):
    val = _poison(A.val).astype(dtype) if dtype == np.float64 else A.val.astype(np.float32)
    if dtype == np.float32 and val.size >= 4:
        b = val.view(np.uint32)
        val[0] = -0.0
        b[2] = np.uint32(0x7FC0BEEF)
    m, n = A.m, A.n
    m_pad = ((m + 63) // 64) * 64
    r, c, v = C.csr_to_coo(A.row_ptr, A.col, val)
    rp2, c2, v2 = C.coo_to_csr(m, r, c, v)
    assert np.array_equal(rp2, A.row_ptr) and np.array_equal(c2, A.col) and _same_bits(v2, val)
    K, ec, ev = C.csr_to_ell(A.row_ptr, A.col, val, m_pad)
    rp2, c2, v2 = C.ell_to_csr(m, K, m_pad, ec, ev)
    assert np.array_equal(rp2, A.row_ptr) and np.array_equal(c2, A.col) and _same_bits(v2, val)
    offs, data, words = C.csr_to_dia(m, n, A.row_ptr, A.col, val, m_pad)
    rp2, c2, v2 = C.dia_to_csr(m, n, offs, m_pad, data, words)
    assert np.array_equal(rp2, A.row_ptr) and np.array_equal(c2, A.col) and _same_bits(v2, val)
    brp, bc, bv, bw = C.csr_to_bcsr(m, n, A.row_ptr, A.col, val)
    rp2, c2, v2 = C.bcsr_to_csr(m, n, brp, bc, bv, bw)
    assert np.array_equal(rp2, A.row_ptr) and np.array_equal(c2, A.col) and _same_bits(v2, val)


def test_layout_definitions_on_5pt():
    g = 8
    A = S.stencil_5pt(g)
    m = A.m
    m_pad = 128
    dense = np.zeros((m, m))
    rows = np.repeat(np.arange(m), np.diff(A.row_ptr))
    dense[rows, A.col] = A.val
    # ELL: slot k of row i at k*m_pad + i, pads -1 / +0.0, K = max row degree
    K, ec, ev = C.csr_to_ell(A.row_ptr, A.col, A.val, m_pad)
    assert K == 5
    for i in (0, 9, 63):
        nz = np.nonzero(dense[i])[0]
        for k in range(K):
            if k < nz.size:
                assert ec[k * m_pad + i] == nz[k] and ev[k * m_pad + i] == dense[i, nz[k]]
            else:
                assert ec[k * m_pad + i] == -1 and ev[k * m_pad + i] == 0.0
                assert not np.signbit(ev[k * m_pad + i])
    assert np.all(ec.reshape(K, m_pad)[:, m:] == -1)
    # DIA: offsets ascending {-g, -1, 0, 1, g}; slot (d, i) holds A[i, i+off_d]
    offs, data, words = C.csr_to_dia(m, m, A.row_ptr, A.col, A.val, m_pad)
    assert offs.tolist() == [-g, -1, 0, 1, g]
    bits = np.unpackbits(words.view(np.uint8), bitorder="little")
    assert int(bits.sum()) == A.nnz
    for d, o in enumerate(offs):
        for i in range(m):
            j = i + o
            expect = dense[i, j] if 0 <= j < m else 0.0
            assert data[d * m_pad + i] == expect
            s = d * m_pad + i
            present = (words[s >> 5] >> (s & 31)) & 1
            assert present == (1 if (0 <= j < m and dense[i, j] != 0) else 0)
    # COO row indices expand row_ptr
    r, _, _ = C.csr_to_coo(A.row_ptr, A.col, A.val)
    assert np.array_equal(r, rows)


def test_rectangular_dia_offsets_span():
    rng = np.random.default_rng(8)
    A = S.random_csr(rng, 7, 19, 0.5)
    offs = C.dia_offsets(A.m, A.n, A.row_ptr, A.col)
    assert offs.min() >= -(A.m - 1) and offs.max() <= A.n - 1


def test_bcsr_hand_worked_example():
    """5 x 6 matrix, 4 x 4 blocks, worked out by hand from the definition:
    block row 0 (rows 0-3) holds column blocks 0 and 1, block row 1 (row 4)
    column block 0; an explicit -0.0 keeps its presence bit."""
    rp = np.array([0, 2, 3, 3, 4, 6])
    col = np.array([0, 5, 1, 4, 0, 2], np.int32)
    val = np.array([1.0, 2.0, 3.0, 4.0, 5.0, -0.0])
    brp, bc, bv, bw = C.csr_to_bcsr(5, 6, rp, col, val)
    assert brp.tolist() == [0, 2, 3] and bc.tolist() == [0, 1, 0]
    expect = np.zeros(48)
    expect[0], expect[5] = 1.0, 3.0            # block 0: (0,0), (1,1)
    expect[16 + 1], expect[16 + 12] = 2.0, 4.0  # block 1: (0,5) -> rr 0 cc 1; (3,4) -> rr 3 cc 0
    expect[32 + 0] = 5.0                        # block 2: (4,0); (4,2) is -0.0 at 34
    assert np.array_equal(bv, expect) and np.signbit(bv[34])
    assert bw.tolist() == [1 | (1 << 5) | (1 << 17) | (1 << 28), 1 | (1 << 2)]


@pytest.mark.parametrize("A", _mats(), ids=lambda A: A.name)
def test_bcsr_blocks_against_dense(A):
    """Every block equals the dense matrix's 4 x 4 tile at (4 R, 4 bcol), the
    tiles not listed are all zero, and the block count is the feature pass's
    count of nonempty aligned 4 x 4 blocks."""
    from oracle import features as OF
    m, n = A.m, A.n
    mp, np_ = -(-m // 4) * 4, -(-n // 4) * 4
    dense = np.zeros((mp, np_))
    rows = np.repeat(np.arange(m), np.diff(A.row_ptr))
    dense[rows, A.col] = A.val
    brp, bc, bv, bw = C.csr_to_bcsr(m, n, A.row_ptr, A.col, A.val)
    listed = np.zeros((mp // 4, np_ // 4), bool)
    for R in range(mp // 4):
        for k in range(brp[R], brp[R + 1]):
            tile = dense[4 * R:4 * R + 4, 4 * bc[k]:4 * bc[k] + 4]
            assert np.array_equal(bv[16 * k:16 * k + 16].reshape(4, 4), tile)
            listed[R, bc[k]] = True
        assert np.all(np.diff(bc[brp[R]:brp[R + 1]]) > 0)
    tiles = dense.reshape(mp // 4, 4, np_ // 4, 4).swapaxes(1, 2)
    occupied = np.zeros_like(listed)
    occupied[rows // 4, A.col // 4] = True
    assert np.array_equal(listed, occupied)
    assert np.all(tiles[~listed] == 0)
    assert bc.size == OF.extract(m, n, A.row_ptr, A.col)["blocks4"]
