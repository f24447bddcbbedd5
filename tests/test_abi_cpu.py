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
    c2 = c.copy()                                                     # one state a single
    k = int(np.argmax(m[:, 0]))                                       # plane wave G != 0:
    c2[s.n_occ + 2] = 0.0                                             # no real form
    c2[s.n_occ + 2, k] = 1.0
    msg = _expect(lib, E, lambda: _setup(lib, s, m, e, c2))
    assert "real" in msg
    holed = np.ones(len(m), bool)                                     # symmetric hole inside
    mid = [k for k, v in enumerate(m.tolist()) if v[1] == 0 and v[2] == 0 and abs(v[0]) == 1]
    holed[mid] = False                                                # the (0, 0) column
    msg = _expect(lib, E, lambda: _setup(lib, s, m[holed], e[holed], c[np.ix_(holed, holed)]))
    assert "consecutive" in msg
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
    _expect(lib, E, lambda: _setup(lib, s, m, e, c, n_extrap=1))   # one cutoff: no fit
    _expect(lib, E, lambda: _setup(lib, s, m, e, c, n_extrap=9))
    _expect(lib, E, lambda: _setup(lib, s, m, e, c, n_extrap=8, extrap_alpha=0.9))
    _expect(lib, E, lambda: _setup(lib, s, m, e, c, quad_mode=9))


def test_unrestricted_validation_paths(lib, cell):
    # the second spin channel is validated on the host like the first
    s, (m, e, c) = cell
    E, G = 1, 2
    for nb in (0, len(e)):
        msg = _expect(lib, E, lambda: _setup(lib, s, m, e, c, second_spin=(e, c, nb)))
        assert "spin channel 2" in msg
    _expect(lib, E, lambda: _setup(lib, s, m, e, c, second_spin=(e[::-1].copy(), c, 3)))
    e2 = e.copy()
    e2[2] = e2[1]
    msg = _expect(lib, G, lambda: _setup(lib, s, m, e, c, second_spin=(e2, c, 2)))
    assert "spin channel 2" in msg
    _expect(lib, E, lambda: _setup(lib, s, m, e, c, second_spin=(e, c * 1.01, 3)))
    _expect(lib, E, lambda: _setup(lib, s, m, e, c, n_occ=0, second_spin=(e, c, 3)))
    with pytest.raises(ValueError):
        _setup(lib, s, m, e, c, second_spin=(e[:-1], c[:-1], 3))


def test_kpoint_validation_paths(lib):
    # every error of the k-point entry is found on the host
    import dataclasses
    from synthetic import make_cell_kmesh
    s = dataclasses.replace(tiny_spec(seed=3, L=5.0, n=8, ecut=2.5, eaux=2.0), amp=1.0)
    kap, mills, eps, coeffs = make_cell_kmesh(s, 2)

    def mk(n_occ=1, n_k=2, e=eps, c=coeffs, m=mills, **kw):
        return lib.Context(s.L, s.n, s.ecut, s.eaux, m, e, c, n_occ, 6, kmesh=n_k, stream=0,
                           **kw)
    _expect(lib, 2, lambda: mk(n_occ=3))                         # bands overlap across k
    _expect(lib, 1, lambda: mk(n_k=0))
    _expect(lib, 1, lambda: mk(n_occ=0))
    e2 = eps.copy()
    e2[3, [4, 5]] = e2[3, [5, 4]]
    e2[3, 4] += 1e-3
    _expect(lib, 1, lambda: mk(e=e2))                             # not ascending at one k
    m2 = [m.copy() for m in mills]
    m2[1][0] = m2[1][1]
    _expect(lib, 1, lambda: mk(m=m2))                             # duplicate plane wave
    with pytest.raises(ValueError):
        mk(c=coeffs[:-1])


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


def _is_real_on_grid(m, c, tol=1e-12):
    pos = {tuple(v): k for k, v in enumerate(m.tolist())}
    neg = np.array([pos[(-a, -b, -d)] for a, b, d in m.tolist()])
    return np.abs(c[:, neg] - np.conj(c)).max() <= tol


def test_real_orbitals_removes_phases(lib, cell):
    # states real up to a phase each: the helper returns them real, equal to
    # the real states up to a sign
    s, (m, e, c) = cell
    th = np.random.default_rng(3).uniform(0, 2 * np.pi, len(e))
    out = lib.real_orbitals(m, e, c * np.exp(1j * th)[:, None], s.n_occ)
    assert _is_real_on_grid(m, out)
    ov = np.einsum("pg,pg->p", np.conj(c), out)
    assert np.allclose(np.abs(ov), 1.0, atol=1e-12) and np.allclose(ov.imag, 0.0, atol=1e-12)
    assert np.array_equal(lib.real_orbitals(m, e, c, s.n_occ), c)   # real input untouched


def test_real_orbitals_complex_eigensolver(lib):
    # a complex Hermitian eigensolver's output (arbitrary phases) on the
    # 12^3 workload: real on the grid afterwards, same states up to a sign
    from synthetic import make_cell_complex
    m, e, c = make_cell_complex(C1, phase_seed=5)
    mr, er, cr = make_cell(C1)
    assert np.array_equal(m, mr) and np.allclose(e, er, atol=1e-10)
    out = lib.real_orbitals(m, e, c, C1.n_occ)
    assert _is_real_on_grid(m, out)
    ov = np.abs(np.einsum("pg,pg->p", np.conj(cr), out))
    assert np.allclose(ov, 1.0, atol=1e-8)


def test_real_orbitals_degenerate_block(lib, cell):
    # two degenerate virtual states mixed by a complex rotation: neither is
    # real up to a phase, the pair is time-reversal invariant; the helper
    # returns a real orthonormal basis of the same span
    s, (m, e, c) = cell
    a, b = s.n_occ + 4, s.n_occ + 5
    e2 = e.copy()
    e2[b] = e2[a]
    c2 = c.copy()
    c2[a] = (c[a] + 1j * c[b]) / np.sqrt(2.0)
    c2[b] = (c[a] - 1j * c[b]) / np.sqrt(2.0)
    out = lib.real_orbitals(m, e2, c2, s.n_occ)
    assert _is_real_on_grid(m, out, 1e-10)
    blk = out[[a, b]]
    assert np.allclose(blk @ np.conj(blk).T, np.eye(2), atol=1e-12)
    P0 = c[[a, b]].T @ np.conj(c[[a, b]])
    P1 = blk.T @ np.conj(blk)
    assert np.abs(P0 - P1).max() <= 1e-12
    others = np.setdiff1d(np.arange(len(e)), [a, b])
    assert np.array_equal(out[others], c[others])
    # without the degeneracy the same input has no real form
    with pytest.raises(lib.LTMP2Error) as ex:
        lib.real_orbitals(m, e, c2, s.n_occ)
    assert ex.value.status == 1


def test_real_orbitals_block_across_the_gap(lib, cell):
    s, (m, e, c) = cell
    a, b = s.n_occ - 1, s.n_occ
    e2 = e.copy()
    e2[b] = e2[a]
    c2 = c.copy()
    c2[a] = (c[a] + 1j * c[b]) / np.sqrt(2.0)
    c2[b] = (c[a] - 1j * c[b]) / np.sqrt(2.0)
    with pytest.raises(lib.LTMP2Error) as ex:
        lib.real_orbitals(m, e2, c2, s.n_occ)
    assert ex.value.status == 2


@pytest.mark.parametrize("xmin,xmax,n", [(0.122, 16.2, 8), (0.037, 46.4, 8), (0.5, 30.0, 6),
                                         (0.0045, 65.3, 10), (0.05, 500.0, 12)])
def test_host_quadrature_equioscillates(lib, xmin, xmax, n):
    # the library's fit is certified on its own: the relative error on the
    # unit interval [1, max(R, R_floor)] has 2 n + 1 alternating extrema of
    # equal size (alternation theorem), located by the oracle's extremum
    # search, and that size is the delta the library reports
    from oracle.quadrature import alternation_points, r_floor
    t, w, d = lib.quadrature(xmin, xmax, n)
    R = max(xmax / xmin, r_floor(n))
    ys, es, emax = alternation_points(n, R, np.log(t * xmin), np.log(w * xmin))
    assert len(ys) == 2 * n + 1
    assert np.all(np.sign(es[1:]) == -np.sign(es[:-1]))
    assert (np.abs(es).max() - np.abs(es).min()) <= 1e-6 * np.abs(es).min()
    assert abs(d - np.abs(es).max()) <= 1e-6 * d
