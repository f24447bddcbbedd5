"""Pins of the oracle's network gradient and of the quadrature tables."""
import numpy as np

from oracle import mlp


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(3)
    p = rng.standard_normal(mlp.NPARAM) * 0.3
    X = rng.standard_normal((7, 3))
    Y = rng.standard_normal((7, 24))
    M = (rng.uniform(size=(7, 24)) < 0.6).astype(float)
    g = mlp.grad(p, X, Y, M)
    h = 1e-6
    for k in rng.choice(mlp.NPARAM, 60, replace=False):
        e = np.zeros(mlp.NPARAM)
        e[k] = h
        fd = (mlp.loss(p + e, X, Y, M) - mlp.loss(p - e, X, Y, M)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 + 1e-6 * abs(g[k])


def test_masked_outputs_do_not_contribute():
    rng = np.random.default_rng(4)
    p = rng.standard_normal(mlp.NPARAM) * 0.3
    X = rng.standard_normal((5, 3))
    Y = rng.standard_normal((5, 24))
    M = np.zeros((5, 24))
    M[:, :4] = 1
    Y2 = Y.copy()
    Y2[:, 4:] += 100.0
    assert np.allclose(mlp.grad(p, X, Y, M), mlp.grad(p, X, Y2, M))
