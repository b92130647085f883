"""What the learned selector gains over the rule-based method.

CPU part: the committed held-out timing tables (every feasible kernel timed
on MI355X for 500 seeded matrices x {float32, float64}, never used in
training) are scored by the committed network through the float64 oracle
forward pass, independently of the GPU inference kernel.  A choice is a hit
when its measured time is within 5% of the exhaustive best.

GPU part: a fresh sample is planned live with the network and with the rules
and both choices are judged against exhaustive timing in the same session.
"""
import json
import os

import numpy as np
import pytest

from oracle import mlp as OM

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "paper_1210_2536_amd", "weights", "selector_gfx950.json")
HELD = os.path.join(ROOT, "paper_1210_2536_amd", "data", "heldout_0000_0500.npz")


def _hit(choice, times):
    best = times.min(axis=1)
    return times[np.arange(len(times)), choice] <= 1.05 * best


def test_network_beats_rules_on_heldout_tables():
    with open(WEIGHTS) as fh:
        w = json.load(fh)
    d = np.load(HELD)
    times, raw, rules = d["times"], d["raw"], d["rules"]
    assert len(times) == 1000
    C = w["n_out"]
    params = OM.unflatten(np.array(w["params"], dtype=np.float64), C)
    z = OM.preprocess(raw.astype(np.float64), np.array(w["mean"]), np.array(w["std"]))
    s, _ = OM.forward(params, z)
    s = np.where(np.isfinite(times), s, np.inf)
    mlp_choice = s.argmin(axis=1)
    mlp_hits = _hit(mlp_choice, times)
    rule_hits = _hit(rules, times)
    # the selector target: within 5% of exhaustive best on >= 90% of matrices
    assert mlp_hits.mean() >= 0.90, mlp_hits.mean()
    assert mlp_hits.mean() >= rule_hits.mean() + 0.3, (mlp_hits.mean(), rule_hits.mean())
    slow_mlp = np.exp(np.mean(np.log(times[np.arange(len(times)), mlp_choice] / times.min(1))))
    slow_rules = np.exp(np.mean(np.log(times[np.arange(len(times)), rules] / times.min(1))))
    assert slow_mlp < slow_rules
    print(f"held-out hit rate: network {mlp_hits.mean():.3f}, rules {rule_hits.mean():.3f}; "
          f"geomean slowdown {slow_mlp:.4f} vs {slow_rules:.4f}")


def _time_pair(plans, x, y, reps=3):
    """Median time of one run of each plan, the two timed in alternation
    (the same session, the same conditions)."""
    import torch
    ts = [[] for _ in plans]
    for _ in range(reps):
        for k, p in enumerate(plans):
            p.run(x, y)
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(5)]
            for a, b in ev:
                a.record()
                for _ in range(8):
                    p.run(x, y)
                b.record()
            torch.cuda.synchronize()
            ts[k].append(np.median([a.elapsed_time(b) for a, b in ev]) / 8)
    return [float(np.median(t)) for t in ts]


@pytest.mark.gpu
def test_live_selection_network_vs_rules():
    """Prediction only (no measurement), judged against exhaustive timing in
    the same session; a choice outside 5% of the table's best but within
    1.5x is timed again beside the best kernel (table noise)."""
    import torch
    from paper_1210_2536_amd import synth
    from paper_1210_2536_amd.spmv import Plan, Selector
    sel = Selector.load(WEIGHTS)
    hits_mlp = hits_rules = total = 0
    for i in range(24):
        # held-out seeds beyond the committed tables, moderate sizes
        A = synth.selector_matrix(10_000 + i, heldout=True, nnz_cap=4_000_000, n_hi=5.5)
        for dt in (np.float32, np.float64):
            rp = torch.from_numpy(A.row_ptr.astype(np.int32)).cuda()
            col = torch.from_numpy(A.col).cuda()
            val = torch.from_numpy(A.val.astype(dt)).cuda()
            x = torch.ones(A.n, dtype=val.dtype, device="cuda")
            y = torch.empty(A.m, dtype=val.dtype, device="cuda")
            ex = Plan(rp, col, val, n=A.n, selector="exhaustive", reps=9).info()
            nm = ex["n_measured"]
            table = dict(zip(ex["measured_kernel"][:nm], ex["measured_ms"][:nm]))
            best = min(table.values())
            best_k = min(table, key=table.get)
            pm = Plan(rp, col, val, n=A.n, selector="mlp", model=sel, tau=0.0,
                      staged=False).info()

            def hit(k):
                if table[k] <= 1.05 * best:
                    return True
                if table[k] > 1.5 * best:
                    return False
                tk, tb = _time_pair([Plan(rp, col, val, n=A.n, selector=int(k)),
                                     Plan(rp, col, val, n=A.n, selector=int(best_k))], x, y)
                return tk <= 1.05 * tb
            hits_mlp += hit(pm["kernel"])
            hits_rules += hit(ex["rules_kernel"])
            total += 1
    print(f"live hit rate: network {hits_mlp / total:.3f}, rules {hits_rules / total:.3f}")
    assert hits_mlp >= hits_rules
    assert hits_mlp / total >= 0.9


@pytest.mark.gpu
def test_out_of_domain_inputs_are_measured_not_trusted():
    """Inputs outside the training range send plan creation to measurement of
    every feasible kernel; the kept kernel is the fastest of those measured,
    up to the switching margin."""
    import torch
    from paper_1210_2536_amd import synth
    from paper_1210_2536_amd.spmv import Plan, Selector
    sel = Selector.load(WEIGHTS)
    assert sel.lo is not None  # the shipped model carries its training range
    A = synth.selector_matrix(20_000, heldout=True, nnz_cap=2_000_000, n_hi=5.0)
    rp = torch.from_numpy(A.row_ptr.astype(np.int32)).cuda()
    col = torch.from_numpy(A.col).cuda()
    val = torch.from_numpy(A.val.astype(np.float64)).cuda()
    inside = Plan(rp, col, val, n=A.n, selector="mlp", model=sel, tau=0.0, staged=False).info()
    assert inside["out_of_domain"] == 0 and inside["n_measured"] == 0
    raw = np.array(inside["mlp_input"], dtype=np.float32)
    # a domain that excludes this matrix's nnz only
    lo, hi = sel.lo.copy(), sel.hi.copy()
    hi[1] = raw[1] - 1
    sel.set_domain(lo, hi)
    out = Plan(rp, col, val, n=A.n, selector="mlp", model=sel, tau=0.0, staged=False).info()
    nfeas = bin(out["feasible_mask"]).count("1")
    assert out["out_of_domain"] == 1 and out["n_measured"] == nfeas
    nm = out["n_measured"]
    times = dict(zip(out["measured_kernel"][:nm], out["measured_ms"][:nm]))
    # the predicted-best kernel is kept unless another measured one is more
    # than 3% faster, so the kept time is within 1/0.97 of the fastest
    assert times[out["kernel"]] <= min(times.values()) / 0.97 * (1 + 1e-12)
    sel.set_domain(None, None)
    again = Plan(rp, col, val, n=A.n, selector="mlp", model=sel, tau=0.0, staged=False).info()
    assert again["out_of_domain"] == 0 and again["n_measured"] == 0


def test_refitted_tree_baseline_on_heldout_tables():
    """The re-fitted rule baseline (a classification tree grown on the same
    training tables) against the paper's fixed rules and the network, on
    the held-out tables; the committed fit is reproduced exactly."""
    from paper_1210_2536_amd import selector as SL
    data = os.path.join(ROOT, "paper_1210_2536_amd", "data")
    ds = SL.load([os.path.join(data, "train_0000_2500.npz"),
                  os.path.join(data, "train_2500_5000.npz")])
    ho = SL.load([HELD])
    meta = SL.tree_baseline(ds, ho, depth=8)
    rules = SL.evaluate_rules(ho)["hit_rate"]
    print(f"held-out hit rate: tree {meta['heldout_tree']['hit_rate']:.3f} "
          f"(with confidence {meta['heldout_tree_tau']['hit_rate']:.3f}), rules {rules:.3f}")
    assert meta["heldout_tree"]["hit_rate"] > rules + 0.5
    with open(os.path.join(ROOT, "paper_1210_2536_amd", "weights", "tree_gfx950.json")) as fh:
        saved = json.load(fh)
    assert saved["heldout_tree"] == meta["heldout_tree"] and saved["leaves"] == meta["leaves"]
    assert all(0.0 < r["confidence"] <= 1.0 and r["support"] >= 5 for r in meta["rules"])


def test_stage_rule_on_heldout_tables():
    """The stage rule of the staged format search: the committed rule is
    reproduced exactly from the training tables; on the held-out tables it
    stops early on a large share of matrices, and the staged pipeline (the
    rule's kernel where it stops, the network with its measurement
    elsewhere) stays within 1% of the network's own hit rate."""
    from paper_1210_2536_amd import capi as C
    from paper_1210_2536_amd import selector as SL
    data = os.path.join(ROOT, "paper_1210_2536_amd", "data")
    ds = SL.load([os.path.join(data, "train_0000_2500.npz"),
                  os.path.join(data, "train_2500_5000.npz")])
    ho = SL.load([HELD])
    with open(WEIGHTS) as fh:
        w = json.load(fh)
    rule, leaves = SL.fit_stage(ds, depth=w["meta"]["stage"]["depth"])
    assert rule == w["stage"] and leaves == w["meta"]["stage"]["leaves"]
    # every test is on an input known after the census; every leaf names a
    # DIA, ELL or CSR kernel; children follow their parents
    for i, f in enumerate(rule["feat"]):
        if f >= 0:
            assert f in SL.STAGE_INPUTS and rule["left"][i] > i and rule["right"][i] > i
        else:
            assert rule["kernel"][i] in SL.STAGE_KERNELS and 0.0 <= rule["conf"][i] <= 1.0
    dom = (w["lo"], w["hi"])
    r = SL.evaluate_stage(rule, ho, dom=dom)
    assert r["exit_share"] >= 0.4 and r["exit_hit_rate"] >= 0.97, r
    # the staged pipeline, with the network scored by the float64 oracle
    times = ho["times"]
    params = OM.unflatten(np.array(w["params"], dtype=np.float64), w["n_out"])
    z = OM.preprocess(ho["raw"].astype(np.float64), np.array(w["mean"]), np.array(w["std"]))
    s, _ = OM.forward(params, z)
    tau = w["meta"]["tau"]
    unstaged = SL.evaluate(s, ho, tau=tau)
    ex, kern = SL.stage_exits(rule, ho["raw"], times, conf=SL.STAGE_CONF, dom=dom)
    choice = unstaged["choice"].copy()
    choice[ex] = kern[ex]
    staged_hits = _hit(choice, np.where(np.isfinite(times), times, np.inf)).mean()
    print(f"held-out: stage rule stops on {ex.mean():.3f} of matrices "
          f"(hit {r['exit_hit_rate']:.3f}); pipeline hit rate staged {staged_hits:.3f}, "
          f"unstaged {unstaged['hit_rate']:.3f}")
    assert staged_hits >= unstaged["hit_rate"] - 0.01
    assert set(np.unique(kern[ex])) <= set(SL.STAGE_KERNELS)
    assert C.KERNELS.index("coo") not in kern[ex]
