"""Host-side checks of the C ABI: exports, validation, host quadrature.

Nothing here launches a kernel: every error path of ltmp2_setup returns
before the first device call, and the quadrature is host code.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

from synthetic import make_cell, C1, tiny_spec

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_1611_06797_amd import ltmp2
    return ltmp2


def test_exports_every_declared_symbol(lib):
    header = open(os.path.join(ROOT, "include", "ltmp2.h")).read()
    names = set(re.findall(r"\b(ltmp2_[a-z_]+)\s*\(", header))
    assert {"ltmp2_setup", "ltmp2_green", "ltmp2_chi", "ltmp2_energy"} <= names
    so = C.CDLL(lib.LIB_PATH)
    for n in sorted(names):
        assert hasattr(so, n), n
    assert set(lib.EXPORTED) == names


def test_supported_grids(lib):
    g = lib.supported_grids()
    assert {12, 32, 40} <= set(g)


@pytest.mark.parametrize("xmin,xmax,n", [(0.122, 16.2, 8), (0.037, 46.4, 8), (0.5, 30.0, 6),
                                         (1.0, 10.0, 1)])
def test_host_quadrature_matches_oracle(lib, xmin, xmax, n):
    from oracle.quadrature import minimax_laplace
    t, w, d = lib.quadrature(xmin, xmax, n)
    to, wo, do = minimax_laplace(xmin, xmax, n)
    assert np.allclose(t, to, rtol=1e-9, atol=0)
    assert np.allclose(w, wo, rtol=1e-9, atol=0)
    assert abs(d - do) <= 1e-8 * do


def test_host_quadrature_rejects_bad_input(lib):
    for args in [(1.0, 0.5, 8), (0.0, 1.0, 8), (1.0, 2.0, 0), (1.0, 2.0, 17)]:
        with pytest.raises(lib.LTMP2Error) as e:
            lib.quadrature(*args)
        assert e.value.status == 1


@pytest.fixture(scope="module")
def cell():
    s = tiny_spec(seed=1, L=6.0, n=12, ecut=3.0, eaux=2.0, n_occ=3)
    return s, make_cell(s)


def _setup(lib, s, m, e, c, **kw):
    args = dict(L=s.L, n_fft=s.n, ecut=s.ecut, eaux=s.eaux, miller=m, eps=e, coeff=c,
                n_occ=s.n_occ, n_tau=8, stream=0)
    args.update(kw)
    return lib.Context(**args)


def _expect(lib, status, fn):
    with pytest.raises(lib.LTMP2Error) as e:
        fn()
    assert e.value.status == status, str(e.value)
    return str(e.value)


def test_validation_paths(lib, cell):
    s, (m, e, c) = cell
    E, G = 1, 2
    _expect(lib, E, lambda: _setup(lib, s, m, e, c, L=-1.0))
    _expect(lib, E, lambda: _setup(lib, s, m, e, c, n_fft=14))       # not 2,3,5-smooth
    _expect(lib, E, lambda: _setup(lib, s, m, e, c, n_fft=6))        # basis outside grid
    _expect(lib, E, lambda: _setup(lib, s, m, e, c, n_occ=0))
    _expect(lib, E, lambda: _setup(lib, s, m, e, c, n_occ=len(e)))
    _expect(lib, E, lambda: _setup(lib, s, m, e, c, n_tau=0))
    _expect(lib, E, lambda: _setup(lib, s, m, e, c, n_tau=17))
    _expect(lib, E, lambda: _setup(lib, s, m, e, c, ecut=1.0))       # basis beyond ecut
    _expect(lib, E, lambda: _setup(lib, s, m, e[::-1].copy(), c))    # eps not ascending
    e2 = e.copy()
    e2[s.n_occ] = e2[s.n_occ - 1]
    _expect(lib, G, lambda: _setup(lib, s, m, e2, c))                # zero gap
    c2 = c * np.exp(0.3j)
    msg = _expect(lib, E, lambda: _setup(lib, s, m, e, c2))          # not real on the grid
    assert "real" in msg
    c3 = c * 1.01
    _expect(lib, E, lambda: _setup(lib, s, m, e, c3))                # not normalised
    c4 = c.copy()
    c4[0, 0] = np.nan
    _expect(lib, E, lambda: _setup(lib, s, m, e, c4))
    e4 = e.copy()
    e4[5] = np.inf
    _expect(lib, E, lambda: _setup(lib, s, m, e4, c))
    m2 = m.copy()
    m2[1] = m2[0]
    _expect(lib, E, lambda: _setup(lib, s, m2, e, c))                # duplicate Miller index
    keep = np.ones(len(m), bool)
    keep[np.argmax(m[:, 0])] = False                                  # basis not symmetric
    _expect(lib, E, lambda: _setup(lib, s, m[keep], e[keep], c[np.ix_(keep, keep)]))
    _expect(lib, E, lambda: _setup(lib, s, m, e, c, tau=np.ones(8), w=None, quad_mode=2))
    _expect(lib, E, lambda: _setup(lib, s, m, e, c, tau=-np.ones(8), w=np.ones(8)))
    _expect(lib, E, lambda: _setup(lib, s, m, e, c, prec=7))
    _expect(lib, E, lambda: _setup(lib, s, m, e, c, quad_mode=9))


def test_workspace_cap_enomem(lib, cell):
    s, (m, e, c) = cell
    _expect(lib, 3, lambda: _setup(lib, s, m, e, c, workspace_cap=1024))


def test_last_error_for_null_context(lib):
    lib.load().ltmp2_destroy(None)          # NULL is ignored
    assert isinstance(lib.load().ltmp2_last_error(None), bytes)


def test_quadrature_table_matches_oracle(lib):
    from oracle.quadrature import minimax_unit
    R = np.array([12.0, 40.0, 133.0, 900.0, 5000.0])
    a, b, d = lib.quadrature_table(8, R)
    for k, r in enumerate(R):
        ao, bo, do = minimax_unit(8, r)
        assert np.allclose(a[k], ao, rtol=1e-7) and np.allclose(b[k], bo, rtol=1e-7)
        assert abs(d[k] - do) <= 1e-6 * do


def test_mlp_dataset_targets_are_minimax_fits(lib):
    from oracle.quadrature import minimax_unit
    X, Y, M, xr = lib.mlp_dataset(300, 5, n_taus=(6, 8))
    assert np.all(M.sum(1) == 2 * np.round(X[:, 2] * 12))
    assert np.all((xr[:, 0] >= 0.05) & (xr[:, 0] <= 1.0))
    R = xr[:, 1] / xr[:, 0]
    assert np.all((R >= 10 - 1e-9) & (R <= 1e4 + 1e-6))
    for k in (0, 17, 299):
        n = int(round(X[k, 2] * 12))
        a, b, d = minimax_unit(n, R[k])
        assert np.allclose(Y[k, :n], np.log(a), atol=1e-6)
        assert np.allclose(Y[k, 12:12 + n], np.log(b), atol=1e-6)
    X2, Y2, M2, _ = lib.mlp_dataset(300, 5, n_taus=(6, 8))
    assert np.array_equal(X, X2) and np.array_equal(Y, Y2)


def test_mlp_init_and_weight_file(lib, tmp_path):
    p = lib.mlp_init(11)
    assert p.shape == (lib.MLP_NPARAM,) and np.all(np.isfinite(p))
    assert np.array_equal(p, lib.mlp_init(11)) and not np.array_equal(p, lib.mlp_init(12))
    f = tmp_path / "w.bin"
    lib.write_mlp_weights(str(f), p)
    assert np.array_equal(lib.read_mlp_weights(str(f)), p)
