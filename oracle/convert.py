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
