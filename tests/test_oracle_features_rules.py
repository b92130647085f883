"""Pins of the oracle's features, rules, network and Equation 2 (CPU only).

Features: closed forms of grid stencils derived from their geometry, brute
force over dense patterns of tiny matrices, an exact power law, invariants.
Rules: the printed thresholds of Section 4 (tests/golden) at their
boundaries, and the formats the rules must give for textbook structures.
Network: central finite differences, the first Adam step in closed form.
Equation 2: the paper's own numbers.
"""
import math
import os

import numpy as np
import pytest

from oracle import amortize, features as F, mlp as NN, rules as R
from paper_1210_2536_amd import synth as S

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------- features

def test_5pt_feature_closed_forms():
    g = 64
    A = S.stencil_5pt(g)
    f = F.extract(A.m, A.n, A.row_ptr, A.col)
    M = g * g
    nnz = 5 * M - 4 * g          # each of the 4 sides loses g couplings
    assert (f["M"], f["N"], f["NNZ"]) == (M, M, nnz) == (4096, 4096, 20224)
    assert f["Ndiags"] == 5
    # off-diagonals have g-1 (|off|=1, broken at every row end) or g (|off|=g)
    # fewer entries than the main diagonal; all exceed 60% of their length
    assert f["NTdiags"] == 5 and f["NTdiags_ratio"] == 1.0
    assert (f["max_RD"], f["min_RD"]) == (5, 3)
    assert f["aver_RD"] == nnz / M == 4.9375
    # degrees: 4 corners of 3, 4(g-2) edge points of 4, (g-2)^2 of 5
    cnt = {3: 4, 4: 4 * (g - 2), 5: (g - 2) ** 2}
    mean = sum(k * c for k, c in cnt.items()) / M
    var = sum(c * (k - mean) ** 2 for k, c in cnt.items()) / M
    assert f["var_RD"] == pytest.approx(var, rel=1e-15) and f["var_RD"] == 248 / 4096
    assert f["ER_DIA"] == f["ER_ELL"] == nnz / (5 * M) == 0.9875
    assert f["bandwidth"] == g
    assert f["blocks4"] == 4960
    assert f["block_fill"] == pytest.approx(20224 / (16 * 4960), rel=1e-15)
    # least-squares slope through the three (ln k, ln P(k)) points
    xs = [math.log(k) for k in cnt]
    ys = [math.log(c / M) for c in cnt.values()]
    xb, yb = sum(xs) / 3, sum(ys) / 3
    slope = sum((a - xb) * (b - yb) for a, b in zip(xs, ys)) / sum((a - xb) ** 2 for a in xs)
    assert f["R"] == pytest.approx(-slope, rel=1e-12)
    assert f["R"] == pytest.approx(-13.487, abs=1e-3)
    assert f["dia_feasible"] and f["ell_feasible"]


@pytest.mark.parametrize("kind,g", [("7pt", 10), ("27pt", 9)])
def test_3d_stencil_feature_closed_forms(kind, g):
    A = S.stencil_7pt(g) if kind == "7pt" else S.stencil_27pt(g)
    f = F.extract(A.m, A.n, A.row_ptr, A.col)
    M = g ** 3
    if kind == "7pt":
        nnz, nd, mx, mn, bw = 7 * M - 6 * g * g, 7, 7, 4, g * g
    else:
        nnz, nd, mx, mn, bw = (3 * g - 2) ** 3, 27, 27, 8, g * g + g + 1
    assert (f["NNZ"], f["Ndiags"], f["max_RD"], f["min_RD"]) == (nnz, nd, mx, mn)
    assert f["ER_DIA"] == pytest.approx(nnz / (nd * M), rel=1e-15)
    assert f["bandwidth"] == bw
    assert f["NTdiags"] == nd


def _brute_features(A):
    dense = np.zeros((A.m, A.n), dtype=bool)
    for i in range(A.m):
        for p in range(A.row_ptr[i], A.row_ptr[i + 1]):
            dense[i, A.col[p]] = True
    diags, blocks = {}, set()
    for i in range(A.m):
        for j in range(A.n):
            if dense[i, j]:
                diags[j - i] = diags.get(j - i, 0) + 1
                blocks.add((i // 4, j // 4))
    nt = 0
    for d, c in diags.items():
        length = sum(1 for i in range(A.m) if 0 <= i + d < A.n)
        nt += c / length > 0.6
    deg = dense.sum(axis=1)
    return dict(Ndiags=len(diags), NTdiags=nt, blocks4=len(blocks),
                bandwidth=max((abs(d) for d in diags), default=0),
                max_RD=int(deg.max()), min_RD=int(deg.min()))


@pytest.mark.parametrize("seed", range(6))
def test_features_vs_brute_force(seed):
    rng = np.random.default_rng([31, seed])
    m, n = int(rng.integers(3, 40)), int(rng.integers(3, 40))
    A = S.random_csr(rng, m, n, float(rng.uniform(0.05, 0.6)))
    f = F.extract(A.m, A.n, A.row_ptr, A.col)
    b = _brute_features(A)
    for key in ("blocks4", "bandwidth", "max_RD", "min_RD"):
        assert f[key] == b[key], key
    if f["Ndiags"] >= 0:
        assert f["Ndiags"] == b["Ndiags"] and f["NTdiags"] == b["NTdiags"]
    else:
        assert f["max_RD"] * f["M"] > 20 * f["NNZ"]


def test_exact_power_law_gives_R():
    # counts 4096/k^2 at k = 1, 2, 4, 8: a pure k^-2 law
    lens = np.concatenate([np.full(4096 // (k * k), k) for k in (1, 2, 4, 8)])
    assert F.power_law_R(lens) == pytest.approx(2.0, rel=1e-13)
    lens = np.concatenate([np.full(3 ** (6 - e), 2 ** e) for e in range(6)])
    # count ~ 3^-e at k = 2^e: R = ln 3 / ln 2
    assert F.power_law_R(lens) == pytest.approx(math.log(3) / math.log(2), rel=1e-13)
    assert F.power_law_R(np.full(10, 7)) == 0.0


@pytest.mark.parametrize("gen", range(4))
def test_feature_invariants(gen):
    for s in range(3):
        rng = np.random.default_rng([32, gen, s])
        A = (S.band_g0, S.uniform_g1, S.zipf_g2, S.blocks_g3)[gen](rng, 2000 + 997 * s)
        f = F.extract(A.m, A.n, A.row_ptr, A.col)
        lens = np.diff(A.row_ptr)
        assert f["sum_rd"] == lens.sum() == f["NNZ"]
        assert f["var_RD"] >= 0 and 0 < f["ER_ELL"] <= 1
        assert f["ell_feasible"] == (f["ER_ELL"] >= 0.05)
        if f["Ndiags"] >= 0:
            assert f["Ndiags"] >= f["max_RD"]
            assert f["Ndiags"] >= -(-f["NNZ"] // min(f["M"], f["N"]))
            assert 0 < f["ER_DIA"] <= 1
            assert f["dia_feasible"] == (f["ER_DIA"] >= 0.05)


def test_mlp_raw_features_layout():
    A = S.stencil_5pt(16)
    f = F.extract(A.m, A.n, A.row_ptr, A.col)
    r = F.mlp_raw_features(f, True)
    assert r.shape == (12,) and r[0] == 256 and r[1] == A.nnz and r[5] == 5 and r[11] == 1.0
    assert r[7] == pytest.approx(1 - f["ER_ELL"]) and r[9] == 16


# --------------------------------------------------------------------- rules

def _thresholds():
    out = {}
    with open(os.path.join(GOLD, "section4_thresholds.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                name, value = line.split()[:2]
                out[name] = float(value)
    return out


def _fdict(M, NNZ, nd, nt, mx, s1, s2, Rv, dia_feas=None, ell_feas=None):
    return dict(M=M, NNZ=NNZ, Ndiags=nd, NTdiags=nt, max_RD=mx, sum_rd=s1,
                sum_rd2=s2, R=Rv,
                dia_feasible=(nd * M <= 20 * NNZ) if dia_feas is None else dia_feas,
                ell_feasible=(mx * M <= 20 * NNZ) if ell_feas is None else ell_feas)


def test_rule_threshold_boundaries():
    T = _thresholds()
    M = 1000
    # Ndiags just below / at the "< 25" boundary, with low fill so only it decides
    nd = int(T["dia_ndiags_good"])
    base = dict(nt=0, mx=10 ** 6, s1=0, s2=0, Rv=0.0)
    nnz = 2 * nd * M // 10  # ER_DIA = 0.2
    assert R.choose_format(_fdict(M, nnz, nd - 1, **base)) == "DIA"
    assert R.choose_format(_fdict(M, nnz, nd, **base)) != "DIA"
    # ER_DIA exactly 0.6 is not "> 0.6"; one more nonzero is
    nd = 100
    nnz = int(T["dia_er_good"] * nd * M)
    assert R.choose_format(_fdict(M, nnz, nd, **base)) != "DIA"
    assert R.choose_format(_fdict(M, nnz + 1, nd, **base)) == "DIA"
    # NTdiags_ratio exactly 0.4 vs just above
    nnz = 2 * nd * M // 10
    assert R.choose_format(_fdict(M, nnz, nd, 40, 10 ** 6, 0, 0, 0.0)) != "DIA"
    assert R.choose_format(_fdict(M, nnz, nd, 41, 10 ** 6, 0, 0, 0.0)) == "DIA"
    # more than 500 diagonals never DIA
    nd = int(T["dia_ndiags_bad"]) + 1
    assert R.choose_format(_fdict(M, nd * M, nd, nd, 10 ** 6, 0, 0, 0.0)) != "DIA"
    # ELL: ER_ELL exactly 0.9 is not enough; var_RD < 0.5 or max_RD < 5 needed
    mx = 10
    nnz = 9 * M
    s1, s2 = nnz, 81 * M  # every row 9: var 0
    off = dict(nd=10 ** 6, nt=0, dia_feas=False)
    assert R.choose_format(_fdict(M, nnz, mx=mx, s1=s1, s2=s2, Rv=0.0, **off)) == "CSR"
    assert R.choose_format(_fdict(M, nnz + 1, mx=mx, s1=nnz + 1, s2=s2 + 19, Rv=0.0, **off)) == "ELL"
    # var_RD exactly 0.5 is not "< 0.5": rows 18/19/20 in proportion 1:2:1
    # (mean 19, var 0.5, ER_ELL 0.95, max_RD 20); one unit less of sum k^2 is
    M2 = 1000
    s1 = 19 * M2
    s2 = 250 * 18 ** 2 + 500 * 19 ** 2 + 250 * 20 ** 2
    assert 2 * (M2 * s2 - s1 * s1) == M2 * M2
    assert R.choose_format(_fdict(M2, s1, mx=20, s1=s1, s2=s2, Rv=0.0, **off)) == "CSR"
    assert R.choose_format(_fdict(M2, s1, mx=20, s1=s1, s2=s2 - 1, Rv=0.0, **off)) == "ELL"
    # max_RD < 5 admits ELL whatever the variance (rows 1 and 4 ... ER needs > 0.9)
    s1, s2 = 3900, 100 * 1 + 900 * 16 + 0
    assert R.choose_format(_fdict(1000, 3901, mx=4, s1=3901, s2=100 + 16 * 900 + 9, Rv=0.0, **off)) == "ELL"
    # COO on R in [1, 4)
    offe = dict(nd=10 ** 6, nt=0, mx=10 ** 6, s1=0, s2=0)
    assert R.choose_format(_fdict(M, 5 * M, Rv=T["coo_R_low"], **offe)) == "COO"
    assert R.choose_format(_fdict(M, 5 * M, Rv=np.nextafter(1.0, 0), **offe)) == "CSR"
    assert R.choose_format(_fdict(M, 5 * M, Rv=np.nextafter(4.0, 0), **offe)) == "COO"
    assert R.choose_format(_fdict(M, 5 * M, Rv=T["coo_R_high"], **offe)) == "CSR"


def test_rules_on_structures():
    A = S.stencil_5pt(64)
    assert R.choose_format(F.extract(A.m, A.n, A.row_ptr, A.col)) == "DIA"
    A = S.uniform_g1(np.random.default_rng([33, 0]), 5000)
    assert R.choose_format(F.extract(A.m, A.n, A.row_ptr, A.col)) == "ELL"
    A = S.blocks_g3(np.random.default_rng([33, 1]), 5000)
    assert R.choose_format(F.extract(A.m, A.n, A.row_ptr, A.col)) == "ELL"
    A = S.zipf_large(n=200_000, kmax=20_000, seed=(33, 2))
    f = F.extract(A.m, A.n, A.row_ptr, A.col)
    assert 1.0 <= f["R"] < 4.0 and R.choose_format(f) == "COO"
    # rows of uniformly spread degree 1..200: flat law (R near 0) -> CSR default
    rng = np.random.default_rng([33, 3])
    lens = rng.integers(1, 201, 4000)
    cols = np.concatenate([np.sort(rng.choice(4000, k, replace=False)) for k in lens])
    rp = np.concatenate([[0], np.cumsum(lens)])
    f = F.extract(4000, 4000, rp, cols)
    assert R.choose_format(f) == "CSR"


# --------------------------------------------------------------------- network

def test_mlp_backward_matches_finite_differences():
    rng = np.random.default_rng(41)
    C, B = 7, 9
    params = [rng.normal(0, 0.5, s) for s in NN.param_shapes(C)]
    z = rng.normal(size=(B, 12))
    t = rng.normal(size=(B, C))
    mask = (rng.random((B, C)) < 0.7).astype(np.float64)
    s, cache = NN.forward(params, z)
    grads = NN.backward(params, cache, s, t, mask)
    h = 1e-6
    for P, G in zip(params, grads):
        flat = P.reshape(-1)
        gflat = G.reshape(-1)
        for idx in rng.choice(flat.size, size=min(flat.size, 12), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = NN.loss(NN.forward(params, z)[0], t, mask)
            flat[idx] = old - h
            lm = NN.loss(NN.forward(params, z)[0], t, mask)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert gflat[idx] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_mlp_loss_and_adam_closed_forms():
    C = 4
    params = [np.zeros(s) for s in NN.param_shapes(C)]
    params[5][:] = [1.0, 2.0, 3.0, 4.0]
    z = np.ones((2, 12))
    s, _ = NN.forward(params, z)
    assert np.array_equal(s, np.tile([1.0, 2.0, 3.0, 4.0], (2, 1)))
    t = np.zeros((2, C))
    mask = np.array([[1, 0, 1, 0], [0, 0, 0, 1.0]])
    assert NN.loss(s, t, mask) == (1 + 9 + 16) / 3
    # first Adam step moves each weight by lr * g / (|g| + eps)
    g = np.array([0.5, -2.0, 0.0, 1e-3])
    p, m, v = NN.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    np.testing.assert_allclose(p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    # preprocessing: log1p on the count features, identity elsewhere
    raw = np.arange(12, dtype=np.float64)
    zz = NN.preprocess(raw, np.zeros(12), np.ones(12))
    for j in range(12):
        assert zz[j] == pytest.approx(math.log1p(j) if j in NN.LOG_FEATURES else j, rel=1e-15)
    assert NN.n_params(10) == 64 * 12 + 64 + 64 * 64 + 64 + 10 * 64 + 10


# --------------------------------------------------------------------- Equation 2

def test_equation2_paper_numbers():
    with open(os.path.join(GOLD, "equation2_break_even.txt")) as fh:
        rows = [l.split() for l in fh if l.strip() and not l.startswith("#")]
    for cost, speedup, printed in rows:
        n = amortize.break_even_calls(float(cost), float(speedup))
        assert n == pytest.approx(28.5)
        assert amortize.min_calls(float(cost), float(speedup)) == int(printed)
    assert amortize.break_even_calls(10, 1.0) == math.inf
