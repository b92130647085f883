"""CSR <-> COO / ELL / DIA layouts (test infrastructure; see package header).

The paper keeps four basic storage formats (Section 2.1); its Figure 1 with
their data structures did not survive, so the standard definitions are used:

COO  every stored entry as (row, col, val), in CSR order (rows ascending,
     columns ascending inside a row).
ELL  K = max_RD slots per row (Section 4, max_RD).  Slot k of row i lives at
     flat index k*m_pad + i (slot-major, i.e. column-major), m_pad >= m.  A
     slot past the row's end holds col -1 and value +0.0.
DIA  one lane per occupied diagonal d = j - i (Section 4, Ndiags), offsets
     ascending.  Entry (i, i+off_d) lives at d*m_pad + i; a slot with no stored
     entry holds +0.0.  A presence bitmap marks stored slots (bit s of the
     little-endian uint32 word s >> 5, s = d*m_pad + i) so explicit zeros
     survive the way back.

BCSR b x b blocks (the blocked formats the paper names as its extension,
     Section 2.1 and the conclusion; b = 4 here).  Block row R covers rows
     [b*R, b*R + b); its blocks are the distinct column blocks col // b of
     those rows, ascending (block row pointer brow_ptr, block column bcol).
     Block k keeps its b*b values row-major at k*b*b + rr*b + cc for entry
     (b*R + rr, b*bcol[k] + cc); a position with no stored entry holds +0.0,
     and presence bit k*b*b + rr*b + cc (same packing as DIA) marks stored
     ones.

Values are moved bit for bit; nothing here does arithmetic on them.
"""
from __future__ import annotations

import numpy as np


def _rows_of_entries(row_ptr):
    rp = np.asarray(row_ptr, dtype=np.int64)
    return np.repeat(np.arange(rp.size - 1, dtype=np.int64), np.diff(rp))


def csr_to_coo(row_ptr, col, val):
    return _rows_of_entries(row_ptr).astype(np.int32), np.asarray(col).copy(), np.asarray(val).copy()


def coo_to_csr(m, row_idx, col, val):
    counts = np.bincount(np.asarray(row_idx, dtype=np.int64), minlength=m)
    rp = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    return rp, np.asarray(col).copy(), np.asarray(val).copy()


def csr_to_ell(row_ptr, col, val, m_pad):
    rp = np.asarray(row_ptr, dtype=np.int64)
    m = rp.size - 1
    assert m_pad >= m
    lens = np.diff(rp)
    K = int(lens.max()) if m else 0
    val = np.asarray(val)
    ecol = np.full(K * m_pad, -1, dtype=np.int32)
    evals = np.zeros(K * m_pad, dtype=val.dtype)
    rows = _rows_of_entries(rp)
    slot = np.arange(rp[-1], dtype=np.int64) - rp[:-1][rows]
    dst = slot * m_pad + rows
    ecol[dst] = col
    evals[dst] = val
    return K, ecol, evals


def ell_to_csr(m, K, m_pad, ecol, evals):
    ecol = np.asarray(ecol).reshape(K, m_pad)[:, :m]
    evals = np.asarray(evals).reshape(K, m_pad)[:, :m]
    present = ecol >= 0
    lens = present.sum(axis=0).astype(np.int64)
    rp = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(lens, out=rp[1:])
    # row-major traversal of the (row, slot) grid keeps slot order per row
    pt = present.T
    return rp, ecol.T[pt].astype(np.int32), evals.T[pt]


def dia_offsets(m, n, row_ptr, col):
    rows = _rows_of_entries(row_ptr)
    d = np.asarray(col, dtype=np.int64) - rows
    return np.unique(d).astype(np.int32)


def csr_to_dia(m, n, row_ptr, col, val, m_pad):
    rp = np.asarray(row_ptr, dtype=np.int64)
    assert m_pad >= m
    val = np.asarray(val)
    rows = _rows_of_entries(rp)
    d = np.asarray(col, dtype=np.int64) - rows
    offsets = np.unique(d)
    D = offsets.size
    slot = np.searchsorted(offsets, d)
    flat = slot * m_pad + rows
    data = np.zeros(D * m_pad, dtype=val.dtype)
    data[flat] = val
    nbits = D * m_pad
    present = np.zeros(nbits, dtype=bool)
    present[flat] = True
    words = np.packbits(np.concatenate([present, np.zeros((-nbits) % 32, bool)]),
                        bitorder="little").view(np.uint32) if nbits else np.zeros(0, np.uint32)
    return offsets.astype(np.int32), data, words


def dia_to_csr(m, n, offsets, m_pad, data, words):
    offsets = np.asarray(offsets, dtype=np.int64)
    D = offsets.size
    nbits = D * m_pad
    bits = np.unpackbits(np.asarray(words, dtype=np.uint32).view(np.uint8),
                         bitorder="little")[:nbits].astype(bool)
    present = bits.reshape(D, m_pad)[:, :m]
    vals = np.asarray(data).reshape(D, m_pad)[:, :m]
    lens = present.sum(axis=0).astype(np.int64)
    rp = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(lens, out=rp[1:])
    pt = present.T
    cols = (np.arange(m, dtype=np.int64)[:, None] + offsets[None, :])[pt]
    return rp, cols.astype(np.int32), vals.T[pt]


def csr_to_bcsr(m, n, row_ptr, col, val, b=4):
    """CSR -> (brow_ptr, bcol, bval, words) with b x b blocks."""
    rp = np.asarray(row_ptr, dtype=np.int64)
    val = np.asarray(val)
    rows = _rows_of_entries(rp)
    cols = np.asarray(col, dtype=np.int64)
    mb, nb = -(-m // b), -(-n // b)
    key = (rows // b) * nb + cols // b
    blocks = np.unique(key)                       # ascending: block row, then block column
    brow_ptr = np.zeros(mb + 1, dtype=np.int64)
    np.cumsum(np.bincount(blocks // nb, minlength=mb), out=brow_ptr[1:])
    k = np.searchsorted(blocks, key)
    flat = k * (b * b) + (rows % b) * b + cols % b
    bval = np.zeros(blocks.size * b * b, dtype=val.dtype)
    bval[flat] = val
    nbits = blocks.size * b * b
    present = np.zeros(nbits, dtype=bool)
    present[flat] = True
    words = np.packbits(np.concatenate([present, np.zeros((-nbits) % 32, bool)]),
                        bitorder="little").view(np.uint32) if nbits else np.zeros(0, np.uint32)
    return brow_ptr, (blocks % nb).astype(np.int32), bval, words


def bcsr_to_csr(m, n, brow_ptr, bcol, bval, words, b=4):
    """Inverse of csr_to_bcsr: the stored entries in CSR order."""
    brow_ptr = np.asarray(brow_ptr, dtype=np.int64)
    bcol = np.asarray(bcol, dtype=np.int64)
    nblk = bcol.size
    nbits = nblk * b * b
    bits = np.unpackbits(np.asarray(words, dtype=np.uint32).view(np.uint8),
                         bitorder="little")[:nbits].astype(bool).reshape(nblk, b, b)
    brow = np.repeat(np.arange(brow_ptr.size - 1, dtype=np.int64), np.diff(brow_ptr))
    kk, rr, cc = np.nonzero(bits)
    rows = brow[kk] * b + rr
    cols = bcol[kk] * b + cc
    vals = np.asarray(bval).reshape(nblk, b, b)[kk, rr, cc]
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    rp = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=m), out=rp[1:])
    return rp, cols.astype(np.int32), vals
