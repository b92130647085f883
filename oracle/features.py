"""Matrix feature parameters (test infrastructure; see package header).

Follows Section 4 of the paper (Table 3 and the formulas beside it), with
these readings of points the text leaves open:

* ER_DIA = NNZ / (Ndiags * M) and ER_ELL = NNZ / (max_RD * M), denominators
  as printed (M, not the true diagonal lengths).
* var_RD = sum_i (k_i - aver_RD)^2 / M, the population variance, evaluated
  exactly as (M * sum k^2 - (sum k)^2) / M^2 from integer sums.
* A diagonal d = j - i is "true" when its stored count exceeds 60% of its
  length len_d = min(M, N - d) - max(0, -d), tested in integers as
  5 * count_d > 3 * len_d (60% is the paper's own ER_DIA breakpoint).
* R is the ordinary least-squares fit of ln(count_k / M) against ln k over
  the row degrees k >= 1 that occur (P(k) ~ k^-R), R = -slope; with fewer than
  two distinct degrees R = 0.
* Zero-fill feasibility (Section 2.3, Section 4, after Bell and Garland): DIA
  needs Ndiags <= 20 * aver_RD, ELL needs max_RD <= 20 * aver_RD, tested in
  integers as Ndiags * M <= 20 * NNZ and max_RD * M <= 20 * NNZ.
* Staged extraction (Section 6): the diagonal census is only taken when DIA
  can still be feasible, i.e. when max_RD * M <= 20 * NNZ (Ndiags >= max_RD
  always).  Otherwise Ndiags is reported as -1 ("more than 20 * aver_RD").

Added for the selector network: bandwidth max |j - i| and the number of
nonempty aligned 4x4 blocks (block fill = NNZ / (16 * blocks)).
"""
from __future__ import annotations

import math

import numpy as np

MLP_FEATURE_NAMES = (
    "n_rows", "nnz", "rd_mean", "rd_max", "rd_std", "ndiags", "dia_fill",
    "ell_pad", "zipf_R", "bandwidth", "block_fill", "is_f64",
)


def power_law_R(row_len) -> float:
    """OLS slope fit of ln P(k) on ln k (Section 4, COO parameter R)."""
    k = np.asarray(row_len, dtype=np.int64)
    m = k.size
    if m == 0:
        return 0.0
    counts = np.bincount(k)
    ks = np.nonzero(counts)[0]
    ks = ks[ks >= 1]
    if ks.size < 2:
        return 0.0
    xs = [math.log(float(v)) for v in ks]
    ys = [math.log(float(counts[v]) / float(m)) for v in ks]
    xbar = math.fsum(xs) / len(xs)
    ybar = math.fsum(ys) / len(ys)
    sxy = math.fsum((a - xbar) * (b - ybar) for a, b in zip(xs, ys))
    sxx = math.fsum((a - xbar) ** 2 for a in xs)
    return -sxy / sxx


def extract(m, n, row_ptr, col) -> dict:
    """All parameters as a dict (integers exact, ratios float64)."""
    rp = np.asarray(row_ptr, dtype=np.int64)
    c = np.asarray(col, dtype=np.int64)
    M, N = int(m), int(n)
    k = np.diff(rp)
    NNZ = int(rp[-1]) if rp.size else 0
    f = {"M": M, "N": N, "NNZ": NNZ}
    s1 = int(k.sum())
    s2 = int((k * k).sum())
    f["sum_rd"] = s1
    f["sum_rd2"] = s2
    f["max_RD"] = int(k.max()) if M else 0
    f["min_RD"] = int(k.min()) if M else 0
    f["aver_RD"] = NNZ / M if M else 0.0
    f["var_RD"] = (M * s2 - s1 * s1) / (M * M) if M else 0.0
    f["std_RD"] = math.sqrt(f["var_RD"])
    f["ER_ELL"] = NNZ / (f["max_RD"] * M) if f["max_RD"] else 0.0
    f["ell_feasible"] = bool(M and f["max_RD"] * M <= 20 * NNZ)
    rows = np.repeat(np.arange(M, dtype=np.int64), k)
    d = c - rows
    f["bandwidth"] = int(np.abs(d).max()) if NNZ else 0
    f["R"] = power_law_R(k)
    blocks = np.unique((rows >> 2) * ((N + 3) // 4 + 1) + (c >> 2)).size if NNZ else 0
    f["blocks4"] = int(blocks)
    f["block_fill"] = NNZ / (16.0 * blocks) if blocks else 0.0
    if M and f["ell_feasible"]:
        offs, cnt = np.unique(d, return_counts=True)
        ln = np.minimum(M, N - offs) - np.maximum(0, -offs)
        nd = int(offs.size)
        nt = int(np.count_nonzero(5 * cnt > 3 * ln))
        f["Ndiags"] = nd
        f["NTdiags"] = nt
        f["NTdiags_ratio"] = nt / nd if nd else 0.0
        f["ER_DIA"] = NNZ / (nd * M) if nd else 0.0
        f["dia_feasible"] = bool(nd * M <= 20 * NNZ)
    else:
        f["Ndiags"] = -1
        f["NTdiags"] = 0
        f["NTdiags_ratio"] = 0.0
        f["ER_DIA"] = 0.0
        f["dia_feasible"] = False
    return f


def mlp_raw_features(f: dict, is_f64: bool) -> np.ndarray:
    """The selector's 12 raw inputs (before log / z-score), float64.

    When the diagonal census was skipped (Ndiags = -1) the diagonal count is
    stood in by NNZ, an upper bound of it.
    """
    nd = f["Ndiags"] if f["Ndiags"] >= 0 else f["NNZ"]
    dia_fill = f["NNZ"] / (nd * f["M"]) if nd and f["M"] else 0.0
    return np.array([
        f["M"], f["NNZ"], f["aver_RD"], f["max_RD"], f["std_RD"], nd,
        dia_fill, 1.0 - f["ER_ELL"], f["R"], f["bandwidth"], f["block_fill"],
        1.0 if is_f64 else 0.0,
    ], dtype=np.float64)
