"""Named synthetic workloads and the algorithmic traffic model.

Workloads (all seeded, see ``synth``):
  c1          5-point Laplacian 64x64, float64
  sweep       200 matrices, n = 10^U(3,6), four generators, float32 and float64
  large       Zipf rows (n = 8M, p(k) ~ k^-2 on [2, 800000], float32) and the
              7-point Laplacian on 256^3 (float64)
  mixed       half 7-point Laplacian on 128^3, half Zipf rows (float64, float32)
  multilevel  27-point stencil on 160^3 plus five 2x2x2-aggregation Galerkin
              levels, float64 (and float32)

Algorithmic bytes of one SpMV are what the stored format itself must move:
matrix arrays once, x read once, y written once (s = value bytes):
  CSR  nnz (s + 4) + 4 (m + 1) + s (n + m)
  COO  nnz (s + 8) + s (n + m)
  ELL  m K (s + 4) + s (n + m)
  DIA  m D s + 4 D + s (n + m)
  BCSR B (16 s + 4) + 4 (ceil(m/4) + 1) + s (n + m), B stored 4x4 blocks
Flops: 2 nnz (padding not counted).
"""
from __future__ import annotations

import concurrent.futures as cf

import numpy as np

from . import synth as S

def algorithmic_bytes(fmt, m, n, nnz, s, K=0, D=0, blocks=0):
    if fmt == "bcsr":   # 4x4 blocks: 16 values + a block column each, block row pointers
        return blocks * (16 * s + 4) + 4 * ((m + 3) // 4 + 1) + s * (n + m)
    if fmt == "csr":
        return nnz * (s + 4) + 4 * (m + 1) + s * (n + m)
    if fmt == "coo":
        return nnz * (s + 8) + s * (n + m)
    if fmt == "ell":
        return m * K * (s + 4) + s * (n + m)
    if fmt == "dia":
        return m * D * s + 4 * D + s * (n + m)
    raise ValueError(fmt)


def break_even_calls(t_plan_ms, t_plain_ms, t_tuned_ms):
    """Equation 2: calls after which a plan that took t_plan_ms to build has
    paid for itself against plain CSR, t_plan / (t_plain - t_tuned) (inf
    when the tuned SpMV is not faster)."""
    gain = t_plain_ms - t_tuned_ms
    return t_plan_ms / gain if gain > 0 else float("inf")


def plan_bytes(info):
    """Algorithmic bytes of one run of a plan, from its report."""
    s = 8 if info["dtype"] == 1 else 4
    fmt = info["format_name"]
    return algorithmic_bytes(fmt, info["m"], info["n"], info["nnz"], s,
                             K=info.get("ell_width", 0), D=info.get("dia_ndiags", 0),
                             blocks=info.get("bcsr_blocks", 0))


def sweep(threads=8, count=S.SWEEP_SIZE):
    with cf.ThreadPoolExecutor(threads) as ex:
        return list(ex.map(S.sweep_matrix, range(count)))


def build(name, threads=8):
    """List of (matrix, dtype, x_seed) for a workload."""
    if name == "c1":
        return [(S.stencil_5pt(64), np.float64, 1)]
    if name == "sweep":
        mats = sweep(threads)
        out = []
        for k, A in enumerate(mats):
            for dt in (np.float32, np.float64):
                out.append((A, dt, (2, k, 1)))
        return out
    if name == "large":
        with cf.ThreadPoolExecutor(2) as ex:
            fz = ex.submit(S.zipf_large)
            fl = ex.submit(S.laplace_7pt_large)
            return [(fz.result(), np.float32, (5, 1)), (fl.result(), np.float64, (5, 2))]
    if name == "mixed":
        A = S.mixed_stencil_zipf()
        return [(A, np.float64, (6, 1)), (A, np.float32, (6, 1))]
    if name in ("multilevel", "multilevel32"):
        levels = S.multilevel(160, 6)
        dt = np.float64 if name == "multilevel" else np.float32
        return [(A, dt, (4, l)) for l, A in enumerate(levels)]
    raise ValueError(f"unknown workload {name}")
