"""Oracle: the learned-quadrature network in FP64 (forward, loss, gradient).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Network 3 -> 64 (tanh) -> 64 (tanh) -> 24 with parameters packed as
W1[64][3] b1[64] W2[64][64] b2[64] W3[24][64] b3[24]; loss = masked mean
squared error sum M (out - Y)^2 / sum M.  The gradient is the chain rule
written out layer by layer; a finite-difference test pins it.
"""
from __future__ import annotations

import numpy as np

H, IN, OUT = 64, 3, 24
SHAPES = [("W1", (H, IN)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (OUT, H)),
          ("b3", (OUT,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(p):
    p = np.asarray(p, np.float64)
    out, k = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = p[k:k + n].reshape(shp)
        k += n
    return out


def forward(p, X):
    q = unpack(p)
    X = np.asarray(X, np.float64)
    h1 = np.tanh(X @ q["W1"].T + q["b1"])
    h2 = np.tanh(h1 @ q["W2"].T + q["b2"])
    return h2 @ q["W3"].T + q["b3"], (h1, h2)


def loss(p, X, Y, M):
    out, _ = forward(p, X)
    M = np.asarray(M, np.float64)
    return float((M * (out - Y) ** 2).sum() / M.sum())


def grad(p, X, Y, M):
    q = unpack(p)
    X = np.asarray(X, np.float64)
    M = np.asarray(M, np.float64)
    out, (h1, h2) = forward(p, X)
    d_out = 2.0 * M * (out - Y) / M.sum()
    g = {"W3": d_out.T @ h2, "b3": d_out.sum(0)}
    d2 = (d_out @ q["W3"]) * (1.0 - h2 ** 2)
    g["W2"] = d2.T @ h1
    g["b2"] = d2.sum(0)
    d1 = (d2 @ q["W2"]) * (1.0 - h1 ** 2)
    g["W1"] = d1.T @ X
    g["b1"] = d1.sum(0)
    return np.concatenate([g[name].ravel() for name, _ in SHAPES])


def features(x_min, x_max, n_tau):
    """(log x_min, log R / log 1e4, n_tau / 12)."""
    return np.array([np.log(x_min), np.log(x_max / x_min) / np.log(1e4), n_tau / 12.0])
