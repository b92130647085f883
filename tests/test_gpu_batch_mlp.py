"""Multilevel batch (persistent kernel, HIP graph) and selector-network kernels."""
import numpy as np
import pytest

from oracle import mlp as OM
from paper_1210_2536_amd import capi
from paper_1210_2536_amd import synth as S

from gpu_util import assert_parity, dev, note, vec

pytestmark = pytest.mark.gpu


def _levels():
    return S.multilevel(32, 5)  # 32^3 .. 2^3


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("kernel", ["dia", "dia_direct", "ell", "csr_vector", "csr_scalar",
                                    "csr_adaptive", "bcsr", "mixed", "mixed2", "dia/wide",
                                    "dia_direct/wide", "ell/wide", "mixed/wide", "bcsr/l2",
                                    "bcsr/l32"])
def test_batch_equals_per_level_runs(kernel, dtype):
    """Persistent launch and graph replay give each level's own result bit
    for bit, for every level kind the persistent kernel takes in (adaptive
    CSR included), with one-row and 16-byte-wide DIA / ELL tiles."""
    import torch
    from paper_1210_2536_amd.spmv import Batch, Plan
    levels = _levels()
    kernel, _, opt = kernel.partition("/")
    prm = {"wide_loads": 1 if opt == "wide" else 2}
    if opt.startswith("l"):   # BCSR lanes per block row (float64: at least 8)
        prm["bcsr_lanes"] = int(opt[1:])
    kinds = {"mixed": ["dia", "ell", "csr_vector", "coo", "csr_adaptive"],
             "mixed2": ["bcsr", "ell", "csr_scalar", "dia_direct", "bcsr"]}.get(
                 kernel, [kernel] * len(levels))
    plans, xs, ys_ref = [], [], []
    for l, (A, k) in enumerate(zip(levels, kinds)):
        rp, col, val = dev(A, dtype)
        p = Plan(rp, col, val, n=A.n, selector=k, params=prm)
        plans.append(p)
        x = S.uniform_vector(A.n, [4, l])
        xs.append(vec(x, dtype))
        y = p.run(xs[-1])
        assert_parity(y.cpu().numpy(), A, x, dtype)
        ys_ref.append(y.cpu().numpy())
    for mode in (0, 1):
        note(f"[batch] kernel={kernel} mode={mode} {np.dtype(dtype).name}")
        B = Batch(plans, mode=mode)
        ys = [torch.full((A.m,), float("nan"), dtype=xs[0].dtype, device="cuda") for A in levels]
        for rep in range(3):   # replays must keep giving the same answer
            for y in ys:
                y.fill_(float("nan"))
            B.run(xs, ys)
            torch.cuda.synchronize()
            for y, r in zip(ys, ys_ref):
                assert np.array_equal(y.cpu().numpy().view(np.uint8), r.view(np.uint8)), (mode, rep)
        if mode == 0:
            # the tuned shape (grid, leading levels on their own) changes
            # nothing in the result
            B.tune(xs, ys, reps=2)
            grid, split = B.shape()
            assert grid >= 1 and 0 <= split <= 2
            for y in ys:
                y.fill_(float("nan"))
            B.run(xs, ys)
            torch.cuda.synchronize()
            for y, r in zip(ys, ys_ref):
                assert np.array_equal(y.cpu().numpy().view(np.uint8), r.view(np.uint8)), "tuned"


def test_mlp_forward_backward_adam_match_oracle():
    import torch
    from paper_1210_2536_amd import spmv as G
    C = capi.K_COUNT
    rng = np.random.default_rng(60)
    n_par = OM.n_params(C)
    assert G.mlp_param_count(C) == n_par
    flat = rng.normal(0, 0.3, n_par).astype(np.float32)
    B = 37
    z = rng.normal(size=(B, 12)).astype(np.float32)
    t = rng.normal(size=(B, C)).astype(np.float32)
    mask = (rng.random((B, C)) < 0.8).astype(np.float32)
    params64 = OM.unflatten(flat.astype(np.float64), C)
    s_ref, cache = OM.forward(params64, z.astype(np.float64))
    g_ref = OM.flatten(OM.backward(params64, cache, s_ref, t.astype(np.float64), mask.astype(np.float64)))
    loss_ref = OM.loss(s_ref, t.astype(np.float64), mask.astype(np.float64))
    P = torch.from_numpy(flat).cuda()
    Z = torch.from_numpy(z).cuda()
    s = G.mlp_forward(P, Z, C).cpu().numpy()
    np.testing.assert_allclose(s, s_ref, rtol=1e-4, atol=1e-6)
    g, loss = G.mlp_backward(P, Z, torch.from_numpy(t).cuda(), torch.from_numpy(mask).cuda(), C)
    np.testing.assert_allclose(g.cpu().numpy(), g_ref, rtol=1e-4, atol=1e-6)
    assert float(loss.item()) == pytest.approx(loss_ref, rel=1e-5)
    # one Adam step from zero moments
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    G.mlp_adam(P, g, m, v, step=1, lr=1e-3)
    p_ref, _, _ = OM.adam_step(flat.astype(np.float64), g.cpu().numpy().astype(np.float64),
                               np.zeros(n_par), np.zeros(n_par), 1, lr=1e-3)
    np.testing.assert_allclose(P.cpu().numpy(), p_ref, rtol=1e-5, atol=1e-7)


def test_selector_inference_matches_training_forward_and_oracle():
    import torch
    from paper_1210_2536_amd import spmv as G
    from oracle import features as OF
    C = capi.K_COUNT
    rng = np.random.default_rng(61)
    flat = rng.normal(0, 0.3, OM.n_params(C)).astype(np.float32)
    mats = [S.stencil_5pt(32), S.zipf_g2(np.random.default_rng([62, 0]), 4000),
            S.uniform_g1(np.random.default_rng([62, 1]), 3000)]
    raw = np.stack([OF.mlp_raw_features(OF.extract(A.m, A.n, A.row_ptr, A.col), i % 2 == 0)
                    for i, A in enumerate(mats)])
    mean = raw.mean(axis=0).astype(np.float32)
    std = (raw.std(axis=0) + 1.0).astype(np.float32)
    sel = G.Selector(flat, mean, std)
    sc = sel.score(torch.from_numpy(raw.astype(np.float32)).cuda()).cpu().numpy()
    z = OM.preprocess(raw.astype(np.float32).astype(np.float64), mean.astype(np.float64),
                      std.astype(np.float64))
    s_ref, _ = OM.forward(OM.unflatten(flat.astype(np.float64), C), z)
    np.testing.assert_allclose(sc, s_ref, rtol=1e-4, atol=1e-5)


def test_gather_probe_sums():
    """The random-gather probe computes what it states: per thread, the
    ordered float64 sum of val[i] * table[idx[i]] over its grid-stride
    indices (checked against numpy on a small input with a ragged tail)."""
    import torch
    from paper_1210_2536_amd import capi as C
    from paper_1210_2536_amd.spmv import gather_probe
    G = int(C.lib().spmv_gather_probe_threads())
    rng = np.random.default_rng(71)
    count = 3 * G + 12345
    for dt in (np.float64, np.float32):
        table = rng.uniform(-1, 1, 1000).astype(dt)
        idx = rng.integers(0, 1000, count).astype(np.int32)
        val = rng.uniform(-1, 1, count).astype(dt)
        out = gather_probe(torch.from_numpy(table).cuda(), torch.from_numpy(idx).cuda(),
                           torch.from_numpy(val).cuda()).cpu().numpy()
        prod = val.astype(np.float64) * table[idx].astype(np.float64)
        pad = np.zeros(4 * G)
        pad[:count] = prod
        ref = pad.reshape(4, G).sum(axis=0)
        absref = np.abs(pad).reshape(4, G).sum(axis=0)
        tol = 1e-15 if dt == np.float64 else 2 ** -24
        assert np.all(np.abs(out.astype(np.float64) - ref) <= tol * absref + 1e-300)


def test_graph_batch_of_many_mixed_plans():
    """Graph mode takes many plans of both dtypes and every kernel class
    (column panels, COO, BCSR, segmented plans included): each replay gives
    every plan's own result bit for bit, also after the vectors change.
    Persistent mode takes the 20 plans of each dtype in one launch (the
    kinds it does not hold -- column panels, COO, long rows by tiles --
    after it, on the same stream), with the same bits and after a change of
    vectors; it refuses plans of two dtypes."""
    import torch
    from paper_1210_2536_amd.spmv import Batch, Plan
    mats = [S.stencil_7pt(12), S.blocks_g3(np.random.default_rng([72, 0]), 4000),
            S.zipf_g2(np.random.default_rng([72, 1]), 30_000),
            S.uniform_g1(np.random.default_rng([72, 2]), 5000)]
    choices = [("dia_direct", {}), ("bcsr", {}), ("coo", {}), ("csr_panel", {"panel_kib": 16}),
               ("ell", {}), ("csr_adaptive", {}), ("csr_vector", {}), ("mlp", {}), ("rules", {})]
    plans, xs, refs, mats_of = [], [], [], []
    for i in range(40):
        A = mats[i % len(mats)]
        dt = np.float64 if (i // 2) % 2 == 0 else np.float32
        k, prm = choices[i % len(choices)]
        rp, col, val = dev(A, dt)
        try:
            if k in ("mlp", "rules"):
                p = Plan(rp, col, val, n=A.n, selector=k, segments=3 if i % 3 == 0 else 0)
            else:
                p = Plan(rp, col, val, n=A.n, selector=k, params=prm or None)
        except capi.SpmvError:  # kernel infeasible for this matrix (zero fill)
            p = Plan(rp, col, val, n=A.n, selector="csr_adaptive")
        x = S.uniform_vector(A.n, [73, i])
        xv = vec(x, dt)
        y = p.run(xv)
        assert_parity(y.cpu().numpy(), A, x, dt)
        plans.append(p)
        xs.append(xv)
        refs.append(y.cpu().numpy())
    note("[batch] graph mode, 40 mixed plans")
    B = Batch(plans, mode=1)
    for rep in range(3):
        ys = [torch.full((p.m,), float("nan"), dtype=x.dtype, device="cuda")
              for p, x in zip(plans, xs)]   # new vectors: recapture on the first replay
        for _ in range(2):
            B.run(xs, ys)
            torch.cuda.synchronize()
            for y, r in zip(ys, refs):
                assert np.array_equal(y.cpu().numpy().view(np.uint8), r.view(np.uint8)), rep
            for y in ys:
                y.fill_(float("nan"))
    B.close()
    for dt in (torch.float64, torch.float32):
        idx = [i for i, x in enumerate(xs) if x.dtype == dt]
        note(f"[batch] persistent mode, {len(idx)} plans of {dt}")
        B = Batch([plans[i] for i in idx], mode=0)
        for rep in range(2):
            ys = [torch.full((plans[i].m,), float("nan"), dtype=dt, device="cuda") for i in idx]
            for _ in range(2):
                B.run([xs[i] for i in idx], ys)
                torch.cuda.synchronize()
                for y, i in zip(ys, idx):
                    assert np.array_equal(y.cpu().numpy().view(np.uint8),
                                          refs[i].view(np.uint8)), (rep, i)
                for y in ys:
                    y.fill_(float("nan"))
        B.close()
    with pytest.raises(capi.SpmvError):
        Batch([plans[0], plans[2]], mode=0)   # float64 and float32


@pytest.mark.parametrize("mode", [0, 1], ids=["persistent", "graph"])
def test_batch_at_its_plan_limit(mode):
    """A batch holds up to 4096 plans in either mode (here one plan 4096
    times, each entry with its own x and y): every output equals the plan's
    own run bit for bit; a 4097th plan is refused."""
    import torch
    from paper_1210_2536_amd.spmv import Batch, Plan
    A = S.stencil_5pt(6)
    n = 4096
    rp, col, val = dev(A, np.float64)
    p = Plan(rp, col, val, n=A.n, selector="csr_vector")
    X = torch.from_numpy(np.random.default_rng(74).uniform(-1, 1, (n, A.n))).cuda()
    Y = torch.full((n, A.m), float("nan"), dtype=torch.float64, device="cuda")
    xs, ys = [X[i] for i in range(n)], [Y[i] for i in range(n)]
    note(f"[batch] mode {mode}, {n} plans")
    B = Batch([p] * n, mode=mode)
    B.run(xs, ys)
    torch.cuda.synchronize()
    R = torch.full_like(Y, float("nan"))
    for i in range(n):
        p.run(xs[i], R[i])
    torch.cuda.synchronize()
    assert torch.equal(Y.view(torch.int64), R.view(torch.int64))
    assert_parity(Y[n - 1].cpu().numpy(), A, X[n - 1].cpu().numpy(), np.float64)
    B.close()
    with pytest.raises(capi.SpmvError):
        Batch([p] * (n + 1), mode=mode)
