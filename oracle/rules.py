"""Rule-based format choice (test infrastructure; see package header).

The paper's C5.0 rule sets were never printed (Section 5), so this is the
method without the learned part: the observations of Section 4 turned into
IF-THEN tests, tried in the Section 6 order DIA, ELL, CSR, COO with CSR the
default format (Section 4 opening).  COO is tried before the CSR default
because its only trigger is R.  Every threshold is compared in integers so
both sides of a parity test take the same decision:

  DIA  feasible and Ndiags <= 500 and
       (Ndiags < 25 or ER_DIA > 0.6 or NTdiags_ratio > 0.4)
  ELL  feasible and ER_ELL > 0.9 and (var_RD < 0.5 or max_RD < 5)
  COO  1 <= R < 4  (small-world degree law)
  CSR  otherwise
"""
from __future__ import annotations


def choose_format(f: dict) -> str:
    M, NNZ = f["M"], f["NNZ"]
    nd = f["Ndiags"]
    if f["dia_feasible"] and 0 <= nd <= 500:
        if nd < 25 or 5 * NNZ > 3 * nd * M or 5 * f["NTdiags"] > 2 * nd:
            return "DIA"
    if f["ell_feasible"]:
        mx = f["max_RD"]
        er_ok = 10 * NNZ > 9 * mx * M
        var_ok = 2 * (M * f["sum_rd2"] - f["sum_rd"] ** 2) < M * M
        if er_ok and (var_ok or mx < 5):
            return "ELL"
    if 1.0 <= f["R"] < 4.0:
        return "COO"
    return "CSR"
