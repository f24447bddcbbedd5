"""Pins of the oracle's minimax Laplace quadrature."""
import math

import numpy as np
import pytest

from oracle.quadrature import (minimax_unit, minimax_laplace, max_rel_error,
                               alternation_points, rel_error_curve)


@pytest.mark.parametrize("R", [10.0, 133.0, 1242.0, 1.45e4])
def test_one_term_closed_form(R):
    # N = 1: e(1) = e(R) = -E and the interior maximum of y exp(-alpha y) at
    # 1/alpha gives alpha = ln R / (R - 1), beta = 2 / (e^-alpha + 1/(alpha e))
    a, b, d = minimax_unit(1, R)
    al = math.log(R) / (R - 1.0)
    be = 2.0 / (math.exp(-al) + 1.0 / (al * math.e))
    assert abs(a[0] - al) <= 1e-10 * al
    assert abs(b[0] - be) <= 1e-10 * be
    assert abs(d - (1.0 - be * math.exp(-al))) < 1e-9


def test_golden_one_term_table():
    # stored values of the N = 1 closed form (tests/golden/quad_n1.txt)
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "quad_n1.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    for R, al, be, E in rows:
        a, b, d = minimax_unit(1, float(R))
        assert abs(a[0] - float(al)) <= 1e-10 * float(al)
        assert abs(b[0] - float(be)) <= 1e-10 * float(be)


@pytest.mark.parametrize("N,R", [(6, 133.0), (8, 133.0), (8, 1242.0), (10, 1.45e4)])
def test_equioscillation(N, R):
    # alternation theorem: 2N + 1 alternating extrema of equal size
    a, b, d = minimax_unit(N, R)
    ys, es, emax = alternation_points(N, R, np.log(a), np.log(b))
    assert len(ys) == 2 * N + 1
    assert np.all(np.sign(es[1:]) == -np.sign(es[:-1]))
    assert (np.abs(es).max() - np.abs(es).min()) <= 1e-6 * np.abs(es).min()
    assert abs(d - np.abs(es).max()) <= 1e-6 * d


def test_error_decreases_with_points():
    ds = [minimax_unit(N, 1242.0)[2] for N in (4, 6, 8, 10)]
    assert all(x > y for x, y in zip(ds, ds[1:]))


def test_scale_covariance():
    t1, w1, d1 = minimax_laplace(0.1, 13.3, 8)
    t2, w2, d2 = minimax_laplace(0.5, 66.5, 8)
    assert np.allclose(t1 * 0.1, t2 * 0.5, rtol=1e-9)
    assert np.allclose(w1 * 0.1, w2 * 0.5, rtol=1e-9)


def test_laplace_integral_check():
    # int_0^inf exp(-x tau) dtau = 1/x (Eq. SCHLT): the quadrature reproduces
    # 1/x within delta on random x of the interval, and the dense-grid error measure
    # agrees with the certified delta
    tau, w, d = minimax_laplace(0.122, 16.2, 8)
    x = np.random.default_rng(0).uniform(0.122, 16.2, 1000)
    assert np.abs(rel_error_curve(x, tau, w)).max() <= d * (1 + 1e-6)
    assert abs(max_rel_error(0.122, 16.2, tau, w) - d) <= 1e-6 * d
    assert np.all(tau > 0) and np.all(w > 0) and np.all(np.diff(tau) > 0)
