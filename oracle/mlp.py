"""CPU ORACLE -- test infrastructure only.

fp64 reference of the launch cost model (not from the paper: the learned dispatcher
is an addition).  Same parameter layout as the library: mu[6], sigma[6], W1[64][6],
b1[64], W2[64][64], b2[64], W3[64][64], b3[64], W4[K][64], b4[K]; ReLU hidden
layers; loss = masked mean squared error sum(M (Y - T)^2) / max(1, sum M).
Written from the definitions of a multilayer perceptron and of backpropagation;
pinned by central finite differences in tests/test_mlp_reference.py.
"""
from __future__ import annotations

import numpy as np

IN, H = 6, 64


def layout(k: int):
    sizes = [("mu", IN), ("sig", IN), ("W1", H * IN), ("b1", H), ("W2", H * H), ("b2", H),
             ("W3", H * H), ("b3", H), ("W4", k * H), ("b4", k)]
    out, o = {}, 0
    for name, size in sizes:
        out[name] = (o, o + size)
        o += size
    return out, o


def unpack(w, k):
    lay, _ = layout(k)
    g = {n: np.asarray(w[a:b], dtype=np.float64) for n, (a, b) in lay.items()}
    g["W1"] = g["W1"].reshape(H, IN)
    g["W2"] = g["W2"].reshape(H, H)
    g["W3"] = g["W3"].reshape(H, H)
    g["W4"] = g["W4"].reshape(k, H)
    return g


def forward(w, X, k):
    p = unpack(w, k)
    X = np.asarray(X, dtype=np.float64)
    xn = (X - p["mu"]) / p["sig"]
    z1 = xn @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    z3 = h2 @ p["W3"].T + p["b3"]
    h3 = np.maximum(z3, 0.0)
    y = h3 @ p["W4"].T + p["b4"]
    return y, (xn, z1, h1, z2, h2, z3, h3)


def loss(w, X, T, M, k):
    y, _ = forward(w, X, k)
    M = np.asarray(M, dtype=np.float64)
    d = np.where(M != 0, y - T, 0.0)
    return float((d * d).sum() / max(1.0, float((M != 0).sum())))


def gradient(w, X, T, M, k):
    """Gradient of loss with respect to every parameter (zero for mu and sigma)."""
    p = unpack(w, k)
    y, (xn, z1, h1, z2, h2, z3, h3) = forward(w, X, k)
    M = np.asarray(M, dtype=np.float64)
    cnt = max(1.0, float((M != 0).sum()))
    dy = np.where(M != 0, 2.0 * (y - T) / cnt, 0.0)
    g = {}
    g["W4"] = dy.T @ h3
    g["b4"] = dy.sum(axis=0)
    dh3 = dy @ p["W4"]
    dz3 = dh3 * (z3 > 0)
    g["W3"] = dz3.T @ h2
    g["b3"] = dz3.sum(axis=0)
    dh2 = dz3 @ p["W3"]
    dz2 = dh2 * (z2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ p["W2"]
    dz1 = dh1 * (z1 > 0)
    g["W1"] = dz1.T @ xn
    g["b1"] = dz1.sum(axis=0)
    lay, total = layout(k)
    out = np.zeros(total)
    for name, (a, b) in lay.items():
        if name in g:
            out[a:b] = g[name].ravel()
    return out


MARGIN = float(np.log2(1.10))  # the decision departs from the heuristic only for a 10 % predicted gain


def choose(w, X, ncurr, k, fused=(0, 1), fused_limit=2048, heuristic_limit=2048, margin=MARGIN):
    """The decision rule: the valid choice with the least predicted time, when it is
    predicted faster than the heuristic's launch (fused up to heuristic_limit frontier
    edges, else wide) by more than `margin` (log2 units); otherwise, and whenever an
    output is not finite, the heuristic's launch.  Returns (choice, y) with y the
    outputs, invalid choices set to +inf."""
    y, _ = forward(w, X, k)
    y = y.copy()
    ncurr = np.asarray(ncurr)
    h = np.where(ncurr <= heuristic_limit, 0, 2)
    finite = np.all(np.isfinite(y), axis=1)
    big = ncurr > fused_limit
    for c in fused:
        y[big, c] = np.inf
    best = np.argmin(y, axis=1)
    rows = np.arange(len(y))
    use = finite & (y[rows, best] + margin < y[rows, h])
    return np.where(use, best, h), y
