"""Offline stage of the auto-tuner: timing dataset, selector training, evaluation.

The paper builds its format model once per platform (Section 5): an
attribute-value dataset of matrix parameters labelled by the measured best
format, mined into rules by C5.0.  Here the dataset is measured on this GPU
over seeded synthetic matrices (the UF collection is not available), every
feasible kernel is timed (brute force, the paper's Table 6 comparison), and
the model is a 12-64-64-C perceptron trained by the library's own HIP
forward / backward / Adam kernels.

  python -m paper_1210_2536_amd.selector collect --start 0 --stop 5000 --out train.npz [--resume --budget S]
  python -m paper_1210_2536_amd.selector collect --heldout --start 0 --stop 500 --out held.npz
  python -m paper_1210_2536_amd.selector train --data train*.npz --out weights.json
  python -m paper_1210_2536_amd.selector eval --weights weights.json --data held.npz

Targets are ln(t_c / t_best) per candidate kernel c (infeasible candidates
masked out), clipped at ln 20 so a hopeless kernel does not dominate the loss.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

import numpy as np

from . import capi as C
from . import synth as S

LOG_FEATURES = (0, 1, 2, 3, 4, 5, 9)
N_IN, HIDDEN = 12, 64
TARGET_CLIP = float(np.log(20.0))


def log(msg):
    print(f"[selector] {msg}", file=sys.stderr, flush=True)


# ----------------------------------------------------------------- collection

def _measure(A, dtype, reps, dev):
    import torch
    from .spmv import Plan
    rp = torch.from_numpy(A.row_ptr.astype(np.int32)).to(dev)
    col = torch.from_numpy(A.col).to(dev)
    val = torch.from_numpy(A.val.astype(dtype)).to(dev)
    p = Plan(rp, col, val, n=A.n, selector="exhaustive", reps=reps)
    info = p.info()
    p.close()
    times = np.full(C.K_COUNT, np.inf)
    for k, t in zip(info["measured_kernel"][:info["n_measured"]],
                    info["measured_ms"][:info["n_measured"]]):
        times[k] = t
    return np.array(info["mlp_input"], dtype=np.float32), times, info["rules_kernel"]


def _save_table(out, cols, heldout, digest):
    tmp = out + ".tmp.npz"
    np.savez(tmp, **{k: np.array(v) for k, v in cols.items()}, heldout=np.array(bool(heldout)),
             sources=np.array(digest))
    os.replace(tmp, out)


def collect(start, stop, heldout, out, reps=7, threads=8, nnz_cap=30_000_000, resume=False,
            budget_s=None):
    """Time every feasible kernel on selector matrices [start, stop) x {f32, f64}.

    The table is written to `out` every 50 matrices and at the end, keyed by
    matrix index; with `resume`, rows already in `out` are kept and the
    collection continues after its last matrix.  `budget_s`: stop (and
    write) once this many seconds have passed.  The table records the digest
    of the kernel sources it was measured on (build.timing_sources_digest)."""
    import torch
    from .build import timing_sources_digest
    dev = torch.device("cuda:0")
    digest = timing_sources_digest()
    keys = ("raw", "times", "rules", "idx", "dtype", "nnz")
    cols = {k: [] for k in keys}
    if resume and os.path.exists(out):
        old = np.load(out)
        if bool(old["heldout"]) != bool(heldout) or str(old["sources"]) != digest:
            raise RuntimeError(f"{out}: other matrices or other kernel sources, not resumed")
        for k in keys:
            cols[k] = list(old[k])
        if len(cols["idx"]):
            start = max(start, int(max(cols["idx"])) + 1)
        log(f"resuming {out} at matrix {start} ({len(cols['idx'])} rows kept)")
    t0 = time.time()
    done = 0
    gen = lambda i: S.selector_matrix(i, heldout=heldout, nnz_cap=nnz_cap)  # noqa: E731
    with cf.ThreadPoolExecutor(threads) as ex:
        futs = {i: ex.submit(gen, i) for i in range(start, min(stop, start + 2 * threads))}
        nxt = start + len(futs)
        for i in range(start, stop):
            if budget_s is not None and time.time() - t0 > budget_s:
                log(f"time budget reached before matrix {i}")
                break
            A = futs.pop(i).result()
            if nxt < stop:
                futs[nxt] = ex.submit(gen, nxt)
                nxt += 1
            for code, dt in ((0, np.float32), (1, np.float64)):
                r, t, rk = _measure(A, dt, reps, dev)
                for k, v in zip(keys, (r, t, rk, i, code, A.nnz)):
                    cols[k].append(v)
            done += 1
            if done % 20 == 0:
                log(f"matrix {i + 1} of [{start}, {stop}), {time.time() - t0:.0f}s")
            if done % 50 == 0:
                _save_table(out, cols, heldout, digest)
        for f in futs.values():
            f.cancel()
    _save_table(out, cols, heldout, digest)
    log(f"wrote {out}: {len(cols['idx'])} rows, {done} matrices in {time.time() - t0:.0f}s")


def load(paths):
    parts = [np.load(p) for p in paths]
    keys = ("raw", "times", "rules", "idx", "dtype", "nnz")
    return {k: np.concatenate([p[k] for p in parts]) for k in keys}


def sources_of(paths):
    """The kernel-source digest the timing tables were measured on (one for
    all of them), or None if they disagree or predate the digest."""
    ds = {str(np.load(p)["sources"]) if "sources" in np.load(p).files else None for p in paths}
    return ds.pop() if len(ds) == 1 else None


# ----------------------------------------------------------------- training

def targets(times):
    best = np.min(times, axis=1, keepdims=True)
    mask = np.isfinite(times)
    t = np.where(mask, np.log(np.where(mask, times, 1.0) / best), 0.0)
    return np.minimum(t, TARGET_CLIP).astype(np.float32), mask.astype(np.float32)


def transform(raw):
    g = np.array(raw, dtype=np.float64)
    for j in LOG_FEATURES:
        g[:, j] = np.log1p(np.maximum(g[:, j], 0.0))
    return g


def standardization(raw):
    g = transform(raw)
    mean = g.mean(axis=0)
    std = np.maximum(g.std(axis=0), 1e-3)
    return mean.astype(np.float32), std.astype(np.float32)


def init_params(n_out=C.K_COUNT, seed=0):
    """He-uniform weights, zero biases, flat in the library's order."""
    rng = np.random.default_rng(seed)
    shapes = [(HIDDEN, N_IN), (HIDDEN,), (HIDDEN, HIDDEN), (HIDDEN,), (n_out, HIDDEN), (n_out,)]
    out = []
    for s in shapes:
        if len(s) == 2:
            lim = np.sqrt(6.0 / s[1])
            out.append(rng.uniform(-lim, lim, size=s).ravel())
        else:
            out.append(np.zeros(s))
    return np.concatenate(out).astype(np.float32)


def train(ds, epochs=300, batch=256, lr=1e-3, seed=0, verbose=True):
    """Train on the GPU with the library's forward / backward / Adam kernels."""
    import torch
    from . import spmv as G
    dev = torch.device("cuda:0")
    mean, std = standardization(ds["raw"])
    z = ((transform(ds["raw"]) - mean) / std).astype(np.float32)
    t, mk = targets(ds["times"])
    Z = torch.from_numpy(z).to(dev)
    T = torch.from_numpy(t).to(dev)
    M = torch.from_numpy(mk).to(dev)
    P = torch.from_numpy(init_params(C.K_COUNT, seed)).to(dev)
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    grad = torch.empty_like(P)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    ws = torch.empty(int(C.lib().spmv_mlp_workspace_floats(batch)), dtype=torch.float32,
                     device=dev)
    rng = np.random.default_rng(seed + 1)
    N = Z.shape[0]
    step = 0
    curve = []
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(N)).to(dev)
        Zp, Tp, Mp = Z[perm].contiguous(), T[perm].contiguous(), M[perm].contiguous()
        tot = 0.0
        nb = 0
        for b0 in range(0, N - batch + 1, batch):
            step += 1
            G.mlp_backward(P, Zp[b0:b0 + batch], Tp[b0:b0 + batch], Mp[b0:b0 + batch],
                           C.K_COUNT, grad=grad, ws=ws, loss=loss)
            G.mlp_adam(P, grad, m, v, step, lr=lr)
            if ep % 25 == 0 or ep == epochs - 1:
                tot += float(loss.item())
                nb += 1
        if nb:
            curve.append((ep, tot / nb))
            if verbose:
                log(f"epoch {ep}: loss {tot / nb:.4f}")
    return P.cpu().numpy(), mean, std, curve


# ----------------------------------------------------------------- evaluation

def scores(params, mean, std, raw):
    import torch
    from .spmv import Selector
    sel = Selector(params, mean, std)
    return sel.score(torch.from_numpy(np.asarray(raw, dtype=np.float32)).cuda()).cpu().numpy()


def evaluate(sc, ds, tau=None, topk=3):
    """Hit rate (t_sel <= 1.05 t_best), geometric-mean slowdown, format accuracy."""
    times = ds["times"]
    feas = np.isfinite(times)
    best = times.min(axis=1)
    s = np.where(feas, sc, np.inf)
    order = np.argsort(s, axis=1)
    choice = order[:, 0]
    measured = np.zeros(len(times), dtype=int)
    if tau is not None:
        srt = np.sort(s, axis=1)
        unsure = (srt[:, 1] - srt[:, 0]) < tau
        for i in np.nonzero(unsure)[0]:
            cand = [c for c in order[i, :topk] if feas[i, c]]
            choice[i] = cand[int(np.argmin(times[i, cand]))]
            measured[i] = len(cand)
    t_sel = times[np.arange(len(times)), choice]
    fmt = lambda k: C.FORMAT_OF[int(k)]  # noqa: E731
    best_k = times.argmin(axis=1)
    return {
        "hit_rate": float(np.mean(t_sel <= 1.05 * best)),
        "geomean_slowdown": float(np.exp(np.mean(np.log(t_sel / best)))),
        "format_accuracy": float(np.mean([fmt(a) == fmt(b) for a, b in zip(choice, best_k)])),
        "mean_measured": float(measured.mean()),
        "choice": choice,
    }


def evaluate_rules(ds):
    sc = np.zeros_like(ds["times"])
    sc[np.arange(len(sc)), ds["rules"]] = -1.0
    return evaluate(sc, ds)


def pick_tau(params, mean, std, ds, topk=3):
    """Smallest margin threshold whose hit rate is within 1% of measuring always."""
    sc = scores(params, mean, std, ds["raw"])
    always = evaluate(sc, ds, tau=1e9, topk=topk)["hit_rate"]
    for tau in (0.0, 0.02, 0.05, 0.1, 0.15, 0.2, 0.3, 0.5, 1.0, 1e9):
        r = evaluate(sc, ds, tau=tau, topk=topk)
        if r["hit_rate"] >= always - 0.01:
            return tau, r
    return 1e9, evaluate(sc, ds, tau=1e9, topk=topk)


FEATURE_NAMES = ("log_m", "log_nnz", "log_aver_rd", "log_max_rd", "log_std_rd", "log_ndiags",
                 "dia_fill", "ell_pad", "zipf_R", "log_bandwidth", "block_fill", "is_f64")


def tree_baseline(ds, ho, depth=8, min_leaf=5, seed=7):
    """Fit the classification-tree baseline on `ds`, choose its confidence
    threshold (leaf-frequency margin between the two best feasible kernels)
    on a 10% validation split as for the network, and score `ho`."""
    from .tree import Tree
    X = transform(ds["raw"])
    y = np.argmin(np.where(np.isfinite(ds["times"]), ds["times"], np.inf), axis=1)
    rng = np.random.default_rng(seed)
    mats = np.unique(ds["idx"])
    vm = set(rng.choice(mats, size=max(1, len(mats) // 10), replace=False).tolist())
    val = np.array([i in vm for i in ds["idx"]])
    t = Tree(C.K_COUNT, max_depth=depth, min_leaf=min_leaf).fit(X[~val], y[~val])
    va = {k: v[val] for k, v in ds.items()}
    sv = t.scores(X[val])
    always = evaluate(sv, va, tau=1e9)["hit_rate"]
    tau = 1e9
    for cand in (0.0, 0.05, 0.1, 0.2, 0.3, 0.5, 1.0):
        if evaluate(sv, va, tau=cand)["hit_rate"] >= always - 0.01:
            tau = cand
            break
    sh = t.scores(transform(ho["raw"]))
    strip = lambda r: {k: v for k, v in r.items() if k != "choice"}  # noqa: E731
    return {"depth": depth, "leaves": t.n_leaves(), "tau": tau,
            "heldout_tree": strip(evaluate(sh, ho)),
            "heldout_tree_tau": strip(evaluate(sh, ho, tau=tau)),
            "rules": t.rules(FEATURE_NAMES, C.KERNELS)}


# Inputs known after the diagonal census (all but R and the block fill) and
# the kernels a staged search may settle on there (DIA, ELL, CSR).
STAGE_INPUTS = (0, 1, 2, 3, 4, 5, 6, 7, 9, 11)
STAGE_KERNELS = tuple(C.KERNELS.index(k) for k in
                      ("csr_scalar", "csr_vector", "csr_adaptive", "csr_panel", "ell", "dia",
                       "dia_direct"))
STAGE_CONF = 0.98


def stage_exits(rule, raw, times, conf=STAGE_CONF, dom=None):
    """Where a staged plan stops early under `rule`: (mask, kernel per row),
    by the library's test (feasible kernel, confidence >= conf, stage inputs
    inside the training domain)."""
    raw = np.asarray(raw, dtype=np.float32)
    feat, thr = rule["feat"], np.asarray(rule["thr"], dtype=np.float32)
    kern = np.empty(len(raw), dtype=np.int64)
    cf_ = np.empty(len(raw))
    for i, x in enumerate(raw):
        node = 0
        while feat[node] >= 0:
            node = rule["left"][node] if x[feat[node]] <= thr[node] else rule["right"][node]
        kern[i], cf_[i] = rule["kernel"][node], rule["conf"][node]
    ok = np.isfinite(times[np.arange(len(raw)), kern]) & (cf_ >= conf)
    if dom is not None:
        lo, hi = (np.asarray(v, dtype=np.float32) for v in dom)
        j = list(STAGE_INPUTS)
        ok &= np.all((raw[:, j] >= lo[j]) & (raw[:, j] <= hi[j]), axis=1)
    return ok, kern


def fit_stage(ds, depth=8, min_leaf=20):
    """Stage rule: a classification tree over the stage inputs, fitted on the
    best-kernel labels, whose leaves name their most reliable DIA / ELL / CSR
    kernel (see tree.stage_rule)."""
    from .tree import Tree, stage_rule
    times = ds["times"]
    feas = np.isfinite(times)
    best = np.where(feas, times, np.inf).min(axis=1)
    hit = feas & (times <= 1.05 * best[:, None])
    X = np.full(ds["raw"].shape, 0.0)
    X[:, list(STAGE_INPUTS)] = ds["raw"][:, list(STAGE_INPUTS)]  # others stay constant
    y = np.argmin(np.where(feas, times, np.inf), axis=1)
    t = Tree(C.K_COUNT, max_depth=depth, min_leaf=min_leaf, quantile_method="lower").fit(X, y)
    return stage_rule(t, X, hit, STAGE_KERNELS), t.n_leaves()


def evaluate_stage(rule, ds, conf=STAGE_CONF, dom=None):
    times = ds["times"]
    best = np.where(np.isfinite(times), times, np.inf).min(axis=1)
    ex, kern = stage_exits(rule, ds["raw"], times, conf=conf, dom=dom)
    t = times[np.arange(len(times)), kern]
    return {"rows": int(len(times)), "exits": int(ex.sum()),
            "exit_share": float(ex.mean()),
            "exit_hit_rate": float(np.mean(t[ex] <= 1.05 * best[ex])) if ex.any() else None,
            "exit_kernels": {C.KERNELS[k]: int(c) for k, c in
                             zip(*np.unique(kern[ex], return_counts=True))}}


def domain(raw):
    """Per-input range [lo, hi] of the raw features the model was fitted on."""
    r = np.asarray(raw, dtype=np.float32)
    return r.min(axis=0), r.max(axis=0)


def save(path, params, mean, std, meta, dom=None):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    d = {"params": [float(v) for v in params], "mean": [float(v) for v in mean],
         "std": [float(v) for v in std], "n_out": C.K_COUNT, "kernels": list(C.KERNELS),
         "meta": meta}
    if dom is not None:
        d["lo"] = [float(v) for v in dom[0]]
        d["hi"] = [float(v) for v in dom[1]]
    with open(path, "w") as fh:
        json.dump(d, fh)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("collect")
    c.add_argument("--start", type=int, default=0)
    c.add_argument("--stop", type=int, default=5000)
    c.add_argument("--heldout", action="store_true")
    c.add_argument("--out", required=True)
    c.add_argument("--reps", type=int, default=7)
    c.add_argument("--threads", type=int, default=8)
    c.add_argument("--resume", action="store_true")
    c.add_argument("--budget", type=float, default=None, help="stop after this many seconds")
    t = sub.add_parser("train")
    t.add_argument("--data", nargs="+", required=True)
    t.add_argument("--heldout", nargs="*", default=[])
    t.add_argument("--out", required=True)
    t.add_argument("--epochs", type=int, default=300)
    tr = sub.add_parser("tree", help="fit the re-fitted rule baseline (classification tree)")
    tr.add_argument("--data", nargs="+", required=True)
    tr.add_argument("--heldout", nargs="+", required=True)
    tr.add_argument("--depth", type=int, default=8)
    tr.add_argument("--out", default="")
    sg = sub.add_parser("stage", help="fit the stage rule of the staged format search "
                                     "and store it in a weights file")
    sg.add_argument("--data", nargs="+", required=True)
    sg.add_argument("--heldout", nargs="*", default=[])
    sg.add_argument("--weights", required=True)
    sg.add_argument("--depth", type=int, default=8)
    e = sub.add_parser("eval")
    e.add_argument("--weights", required=True)
    e.add_argument("--data", nargs="+", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "collect":
        collect(a.start, a.stop, a.heldout, a.out, reps=a.reps, threads=a.threads,
                resume=a.resume, budget_s=a.budget)
    elif a.cmd == "train":
        ds = load(a.data)
        n = len(ds["raw"])
        rng = np.random.default_rng(7)
        val = np.zeros(n, bool)
        # validation split by matrix (both dtypes of a matrix stay together)
        mats = np.unique(ds["idx"])
        vm = set(rng.choice(mats, size=max(1, len(mats) // 10), replace=False).tolist())
        val = np.array([i in vm for i in ds["idx"]])
        tr = {k: v[~val] for k, v in ds.items()}
        va = {k: v[val] for k, v in ds.items()}
        params, mean, std, curve = train(tr, epochs=a.epochs)
        tau, vr = pick_tau(params, mean, std, va)
        meta = {"kernel_sources_sha256": sources_of(a.data + list(a.heldout)),
                "train_rows": int((~val).sum()), "val_rows": int(val.sum()), "tau": tau,
                "val_hit_rate_tau": vr["hit_rate"], "loss_curve": curve,
                "val_rules": {k: v for k, v in evaluate_rules(va).items() if k != "choice"}}
        if a.heldout:
            ho = load(a.heldout)
            sc = scores(params, mean, std, ho["raw"])
            meta["heldout_mlp"] = {k: v for k, v in evaluate(sc, ho).items() if k != "choice"}
            meta["heldout_mlp_tau"] = {k: v for k, v in evaluate(sc, ho, tau=tau).items()
                                       if k != "choice"}
            meta["heldout_rules"] = {k: v for k, v in evaluate_rules(ho).items() if k != "choice"}
        save(a.out, params, mean, std, meta, dom=domain(tr["raw"]))
        log(json.dumps({k: v for k, v in meta.items() if k != "loss_curve"}))
    elif a.cmd == "tree":
        meta = tree_baseline(load(a.data), load(a.heldout), depth=a.depth)
        log(json.dumps({k: v for k, v in meta.items() if k != "rules"}))
        if a.out:
            with open(a.out, "w") as fh:
                json.dump(meta, fh, indent=1)
    elif a.cmd == "stage":
        with open(a.weights) as fh:
            w = json.load(fh)
        dom = (w["lo"], w["hi"]) if "lo" in w else None
        tr = load(a.data)
        rule, leaves = fit_stage(tr, depth=a.depth)
        meta = {"depth": a.depth, "leaves": leaves, "conf": STAGE_CONF,
                "train": evaluate_stage(rule, tr, dom=dom)}
        if a.heldout:
            meta["heldout"] = evaluate_stage(rule, load(a.heldout), dom=dom)
        w["stage"] = rule
        w["meta"]["stage"] = meta
        with open(a.weights, "w") as fh:
            json.dump(w, fh)
        log(json.dumps(meta))
    else:
        with open(a.weights) as fh:
            w = json.load(fh)
        ds = load(a.data)
        sc = scores(np.array(w["params"], np.float32), np.array(w["mean"], np.float32),
                    np.array(w["std"], np.float32), ds["raw"])
        tau = w["meta"].get("tau")
        out = {"mlp": evaluate(sc, ds), "mlp_tau": evaluate(sc, ds, tau=tau),
               "rules": evaluate_rules(ds)}
        print(json.dumps({k: {kk: vv for kk, vv in v.items() if kk != "choice"}
                          for k, v in out.items()}))


if __name__ == "__main__":
    main()
