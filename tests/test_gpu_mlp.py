"""GPU tests of the learned Laplace quadrature (network kernels, training,
polish + certification + fallback) against the oracle."""
import os
import sys
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "paper_1611_06797_amd", "data", "laplace_mlp.bin")


def _say(*a):
    print("[gpu-case]", *a, flush=True)


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1611_06797_amd import ltmp2
    return ltmp2


def test_forward_and_gradient_vs_oracle(L):
    from oracle import mlp
    _say("mlp forward/backward vs oracle")
    X, Y, M, _ = L.mlp_dataset(96, 9, n_taus=(6, 10))
    p = L.mlp_init(5)
    out = L.mlp_forward(p, X)
    ref, _ = mlp.forward(p.astype(np.float64), X)
    assert np.abs(out - ref).max() <= 1e-5 * max(1.0, np.abs(ref).max())
    g, loss = L.mlp_grad(p, X, Y, M)
    gr = mlp.grad(p.astype(np.float64), X, Y, M)
    assert abs(loss - mlp.loss(p.astype(np.float64), X, Y, M)) <= 1e-5 * loss
    assert np.linalg.norm(g - gr) <= 1e-5 * np.linalg.norm(gr)
    assert np.abs(g - gr).max() <= 1e-5 * np.abs(gr).max()


def test_training_reduces_loss_and_is_deterministic(L):
    _say("mlp short training")
    X, Y, M, _ = L.mlp_dataset(4096, 21, n_taus=(6, 8))
    p1 = L.mlp_init(1)
    h1 = L.mlp_train(p1, X, Y, M, 8, 256, 3e-3, 7)
    p2 = L.mlp_init(1)
    h2 = L.mlp_train(p2, X, Y, M, 8, 256, 3e-3, 7)
    assert h1[-1] < 0.2 * h1[0]
    assert np.array_equal(p1, p2) and np.array_equal(h1, h2)


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="trained weights not present")
def test_trained_network_certifies_and_gains(L):
    # what the trained network gains: a certified minimax quadrature from the
    # proposal + 3 Remez passes, against the plain continuation fit
    from oracle.quadrature import minimax_laplace
    p = L.read_mlp_weights(WEIGHTS)
    X, Y, M, xr = L.mlp_dataset(60, 12345)
    cert = 0
    t_l = t_p = 0.0
    for k in range(len(X)):
        n = int(round(X[k, 2] * 12))
        a, b = xr[k]
        t0 = time.perf_counter()
        tau, w, d, fl = L.learned_quadrature(p, a, b, n)
        t1 = time.perf_counter()
        tp, wp, dp = L.quadrature(a, b, n)
        t2 = time.perf_counter()
        t_l += t1 - t0
        t_p += t2 - t1
        cert += fl & 1
        to, wo, do = minimax_laplace(a, b, n)
        assert abs(d - do) <= 2e-6 * do            # certified or fallback: minimax quality
        if fl & 1:
            assert np.allclose(tau, to, rtol=1e-4) and np.allclose(w, wo, rtol=1e-4)
    print(f"[mlp] certified {cert}/{len(X)}  learned {1e3 * t_l / len(X):.2f} ms  "
          f"plain {1e3 * t_p / len(X):.2f} ms per fit", flush=True)
    assert cert >= 0.9 * len(X)
    assert t_l < t_p


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="trained weights not present")
def test_learned_mode_in_setup_and_fallback(L, tmp_path):
    # LTMP2_QUAD_LEARNED inside ltmp2_setup: certified proposal or plain fit;
    # a corrupt weight file falls back to the plain fit and says so
    from synthetic import make_cell, C1
    from oracle.quadrature import minimax_laplace
    m, e, c = make_cell(C1)
    _say("learned mode setup C1")
    with L.Context(C1.L, C1.n, C1.ecut, C1.eaux, m, e, c, C1.n_occ, C1.n_tau,
                   quad_mode=L.QUAD_LEARNED, mlp_weights=WEIGHTS) as ctx:
        tau, w, d = ctx.get_quadrature()
        flags = ctx.info.quad_flags
    to, wo, do = minimax_laplace(ctx.info.x_min, ctx.info.x_max, C1.n_tau)
    assert abs(d - do) <= 2e-6 * do
    assert flags & 3
    bad = tmp_path / "bad.bin"
    bad.write_bytes(b"LTMP2MLP" + b"\x01\x00\x00\x00" + b"\x00" * 40)
    with L.Context(C1.L, C1.n, C1.ecut, C1.eaux, m, e, c, C1.n_occ, C1.n_tau,
                   quad_mode=L.QUAD_LEARNED, mlp_weights=str(bad)) as ctx:
        assert ctx.info.quad_flags == 6
        t2, w2, d2 = ctx.get_quadrature()
    assert np.allclose(t2, to, rtol=1e-9)


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="trained weights not present")
@pytest.mark.parametrize("x_min,x_max,n", [(0.0045, 65.3, 10), (0.0023, 65.3, 10)])
def test_learned_quadrature_at_the_40_cube_range(L, x_min, x_max, n):
    # the 40^3 cell's denominator range lies outside the training ranges
    # (x_min below 0.05 Ha, R = 1.45e4 and 2.8e4 above 1e4): the proposal is
    # either certified after 3 Remez passes or replaced by the plain fit, and
    # in both cases the error is the oracle's minimax error
    from oracle.quadrature import minimax_laplace
    p = L.read_mlp_weights(WEIGHTS)
    _say("learned quadrature out of range", x_min, x_max, n)
    tau, w, d, fl = L.learned_quadrature(p, x_min, x_max, n)
    to, wo, do = minimax_laplace(x_min, x_max, n)
    print(f"[mlp ood] R={x_max / x_min:.3g} flags={fl} delta={d:.6e} oracle={do:.6e}", flush=True)
    assert fl & 3
    assert abs(d - do) <= 2e-6 * do
    if fl & 1:
        assert np.allclose(tau, to, rtol=1e-4) and np.allclose(w, wo, rtol=1e-4)
