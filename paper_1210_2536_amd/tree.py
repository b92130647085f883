"""A classification tree over the selector's inputs: the re-fitted rule
baseline (the paper's offline rule mining, Section 5, done here on this
GPU's own timing tables instead of the C5.0 tool).

The tree is grown top-down on the best-kernel label of each training row
(argmin of its measured times) by Gini impurity; every leaf keeps its class
counts, so a prediction is the most frequent class in the leaf among the
kernels feasible for the matrix, and the leaf's purity is the confidence of
its rule.  Features are the 12 raw selector inputs (log-scaled where the
network scales them; a tree is unchanged by monotone rescaling anyway).
"""
from __future__ import annotations

import json

import numpy as np


def _gini(counts):
    n = counts.sum(axis=-1, keepdims=True)
    p = counts / np.maximum(n, 1)
    return 1.0 - (p * p).sum(axis=-1)


class Tree:
    def __init__(self, n_classes, max_depth=8, min_leaf=10, n_thresholds=64,
                 quantile_method="linear"):
        self.C = n_classes
        self.max_depth = max_depth
        self.min_leaf = min_leaf
        self.n_thr = n_thresholds
        # "lower" keeps every threshold a data value, so float32 inputs compare
        # the same way against it in float32 and in float64
        self.qmethod = quantile_method
        # nodes: feature, threshold, left, right (-1 for leaves), class counts
        self.feat, self.thr, self.left, self.right, self.counts = [], [], [], [], []

    def _new(self, counts):
        self.feat.append(-1)
        self.thr.append(0.0)
        self.left.append(-1)
        self.right.append(-1)
        self.counts.append(counts)
        return len(self.feat) - 1

    def fit(self, X, y):
        X = np.asarray(X, dtype=np.float64)
        y = np.asarray(y, dtype=np.int64)
        onehot = np.eye(self.C)[y]
        root = self._new(onehot.sum(axis=0))
        stack = [(root, np.arange(len(y)), 0)]
        while stack:
            node, idx, depth = stack.pop()
            if depth >= self.max_depth or len(idx) < 2 * self.min_leaf:
                continue
            parent = _gini(self.counts[node][None])[0] * len(idx)
            best = (0.0, -1, 0.0, None)
            for f in range(X.shape[1]):
                xs = X[idx, f]
                cand = np.unique(np.quantile(xs, np.linspace(0, 1, self.n_thr + 2)[1:-1],
                                             method=self.qmethod))
                if cand.size == 0:
                    continue
                # class counts left of every candidate threshold
                below = xs[:, None] <= cand[None, :]
                left = below.T.astype(np.float64) @ onehot[idx]            # [T, C]
                nl = left.sum(axis=1)
                right = self.counts[node][None, :] - left
                nr = right.sum(axis=1)
                ok = (nl >= self.min_leaf) & (nr >= self.min_leaf)
                if not ok.any():
                    continue
                cost = _gini(left) * nl + _gini(right) * nr
                cost = np.where(ok, cost, np.inf)
                t = int(np.argmin(cost))
                gain = parent - cost[t]
                if gain > best[0] + 1e-12:
                    best = (gain, f, float(cand[t]), xs <= cand[t])
            if best[1] < 0:
                continue
            _, f, thr, mask = best
            li, ri = idx[mask], idx[~mask]
            self.feat[node], self.thr[node] = f, thr
            self.left[node] = self._new(onehot[li].sum(axis=0))
            self.right[node] = self._new(onehot[ri].sum(axis=0))
            stack.append((self.left[node], li, depth + 1))
            stack.append((self.right[node], ri, depth + 1))
        return self

    def leaf(self, x):
        node = 0
        while self.feat[node] >= 0:
            node = self.left[node] if x[self.feat[node]] <= self.thr[node] else self.right[node]
        return node

    def scores(self, X):
        """Negative leaf class frequencies (lower is better, like the network's
        predicted slowdowns), one row per input."""
        X = np.asarray(X, dtype=np.float64)
        out = np.empty((len(X), self.C))
        for i, x in enumerate(X):
            c = self.counts[self.leaf(x)]
            out[i] = -c / max(1.0, c.sum())
        return out

    def n_leaves(self):
        return sum(1 for f in self.feat if f < 0)

    def rules(self, names, kernels):
        """The tree as if-then rules with their purity (confidence) and support."""
        out = []

        def walk(node, conds):
            if self.feat[node] < 0:
                c = self.counts[node]
                k = int(np.argmax(c))
                out.append({"if": " and ".join(conds) or "true", "then": kernels[k],
                            "confidence": float(c[k] / max(1.0, c.sum())),
                            "support": int(c.sum())})
                return
            f, t = names[self.feat[node]], self.thr[node]
            walk(self.left[node], conds + [f"{f} <= {t:.4g}"])
            walk(self.right[node], conds + [f"{f} > {t:.4g}"])

        walk(0, [])
        return out

    def to_json(self):
        return json.dumps({"C": self.C, "feat": self.feat, "thr": self.thr, "left": self.left,
                           "right": self.right, "counts": [c.tolist() for c in self.counts]})


def stage_rule(tree, X, hit, allowed):
    """Leaf rules of a tree for the staged format search: every leaf names
    the allowed kernel that ran within 5% of the fastest (`hit`, boolean
    [rows, C]) on the largest share of the leaf's training rows, with that
    share as its confidence.  Returns the node lists of the library's stage
    rule (feat, thr, left, right, kernel, conf); inner nodes carry kernel -1
    and confidence 0, leaves feature -1."""
    X = np.asarray(X, dtype=np.float64)
    leaves = np.array([tree.leaf(x) for x in X], dtype=np.int64)
    mask = np.zeros(tree.C, bool)
    mask[list(allowed)] = True
    n = len(tree.feat)
    kernel = [-1] * n
    conf = [0.0] * n
    for node in range(n):
        if tree.feat[node] >= 0:
            continue
        rows = leaves == node
        if not rows.any():          # no training row reached it: never trusted
            kernel[node] = int(np.flatnonzero(mask)[0])
            continue
        share = np.where(mask, hit[rows].mean(axis=0), -1.0)
        kernel[node] = int(np.argmax(share))
        conf[node] = float(share[kernel[node]])
    return {"feat": [int(f) for f in tree.feat], "thr": [float(t) for t in tree.thr],
            "left": [int(v) for v in tree.left], "right": [int(v) for v in tree.right],
            "kernel": kernel, "conf": conf}
