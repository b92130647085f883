"""Selector network in float64 (test infrastructure; see package header).

The paper learns its format choice offline (Section 5, Equation 1: features
and thresholds map to one of the formats) with C5.0 rule sets.  The learned
part here is a small multilayer perceptron instead; this module is its plain
float64 definition, used to check the GPU forward, backward and Adam kernels.

Inputs: 12 raw features (see ``features.MLP_FEATURE_NAMES``).  Preprocessing:
log1p on the count-like inputs (rows, nnz, row-degree mean / max / std,
diagonal count, bandwidth: indices 0-5 and 9), then z = (g - mean) / std with
stored per-feature mean and std.

Network: h1 = relu(W1 z + b1), h2 = relu(W2 h1 + b2), s = W3 h2 + b3 with
W1 64x12, W2 64x64, W3 Cx64 (row-major).  s_c predicts the log slowdown
ln(t_c / t_best) of candidate kernel c; the choice is argmin over feasible c.

Loss: masked mean squared error, sum_{b,c} mask (s - t)^2 / max(1, sum mask).
Optimiser: Adam (Kingma and Ba 2015) with bias correction.

Flat parameter order (shared interface with the GPU buffer):
W1, b1, W2, b2, W3, b3.
"""
from __future__ import annotations

import numpy as np

LOG_FEATURES = (0, 1, 2, 3, 4, 5, 9)
N_IN = 12
HIDDEN = 64


def param_shapes(n_out):
    return [(HIDDEN, N_IN), (HIDDEN,), (HIDDEN, HIDDEN), (HIDDEN,),
            (n_out, HIDDEN), (n_out,)]


def n_params(n_out):
    return sum(int(np.prod(s)) for s in param_shapes(n_out))


def unflatten(flat, n_out):
    out, o = [], 0
    for s in param_shapes(n_out):
        size = int(np.prod(s))
        out.append(np.asarray(flat[o:o + size], dtype=np.float64).reshape(s))
        o += size
    return out


def flatten(params):
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in params])


def preprocess(raw, mean, std):
    g = np.array(raw, dtype=np.float64, copy=True)
    for j in LOG_FEATURES:
        g[..., j] = np.log1p(np.maximum(g[..., j], 0.0))
    return (g - mean) / std


def forward(params, z):
    W1, b1, W2, b2, W3, b3 = params
    a1 = z @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    s = h2 @ W3.T + b3
    return s, (z, a1, h1, a2, h2)


def loss(s, target, mask):
    cnt = max(1.0, float(mask.sum()))
    r = np.where(mask > 0, s - target, 0.0)
    return float((r * r).sum() / cnt)


def backward(params, cache, s, target, mask):
    W1, b1, W2, b2, W3, b3 = params
    z, a1, h1, a2, h2 = cache
    cnt = max(1.0, float(mask.sum()))
    ds = np.where(mask > 0, 2.0 * (s - target) / cnt, 0.0)
    gW3 = ds.T @ h2
    gb3 = ds.sum(axis=0)
    dh2 = ds @ W3
    da2 = dh2 * (a2 > 0)
    gW2 = da2.T @ h1
    gb2 = da2.sum(axis=0)
    dh1 = da2 @ W2
    da1 = dh1 * (a1 > 0)
    gW1 = da1.T @ z
    gb1 = da1.sum(axis=0)
    return [gW1, gb1, gW2, gb2, gW3, gb3]


def adam_step(p, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update of flat arrays; returns (p, m, v) as new arrays."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v

