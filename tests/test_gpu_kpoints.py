"""GPU parity of k-point meshes (ltmp2_setup_kpoints) against the k-point
oracle (oracle.kpoints), through the C ABI.

Inputs: seeded Bloch states of synthetic cells on Gamma-centred meshes
(synthetic.make_cell_kmesh, exact time reversal).  Energies per unit cell are
compared at the same (tau, w): FP64 to 1e-9 relative, BF16x3 to 1 uHa per
occupied band of the supercell.  The small workload's cell on the 2^3 mesh is
compared with stored oracle energies (tests/golden/make_kpoints.py).
"""
import dataclasses
import json
import os
import sys

import numpy as np
import pytest

from synthetic import make_cell_kmesh, make_cell, tiny_spec, C1

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _kctx(spec, n_k, mills, eps, coeffs, n_occ, tau, w, **kw):
    from paper_1611_06797_amd import Context
    return Context(spec.L, spec.n, spec.ecut, spec.eaux, mills, eps, coeffs, n_occ, len(tau),
                   tau=tau, w=w, kmesh=n_k, **kw)


def _tiny(amp=1.0, seed=3):
    return dataclasses.replace(tiny_spec(seed=seed, L=5.0, n=8, ecut=2.5, eaux=2.0, n_occ=1),
                               amp=amp)


@pytest.mark.parametrize("n_k,n_occ", [(2, 1), (2, 2), (3, 1)])
def test_tiny_mesh_vs_oracle(torch_cuda, n_k, n_occ):
    from oracle.kpoints import KProblem
    from oracle.quadrature import minimax_laplace
    s = _tiny()
    kap, mills, eps, coeffs = make_cell_kmesh(s, n_k)
    K = KProblem(s.L, s.n, s.eaux, n_k, kap, mills, eps, coeffs, n_occ)
    tau, w, _ = minimax_laplace(*K.x_range(), 6)
    ref = K.energies(tau, w)
    _say("tiny cell, k mesh", n_k, "n_occ", n_occ)
    with _kctx(s, n_k, mills, eps, coeffs, n_occ, tau, w) as ctx:
        ed, ex, pt, qe = ctx.energy()
        info = ctx.info
    print(f"[kmesh {n_k} occ {n_occ}] n_grid={info.n_grid} n_g={info.n_g} "
          f"dE_d={ed - ref['e_d_lt']:.3e} dE_x={ex - ref['e_x_lt']:.3e}")
    assert info.n_k == n_k and info.n_occ == n_k ** 3 * n_occ
    assert abs(ed - ref["e_d_lt"]) <= 1e-9 * abs(ref["e_d_lt"])
    assert abs(ex - ref["e_x_lt"]) <= 1e-9 * abs(ref["e_x_lt"])
    assert np.allclose(pt[:, 0], ref["per_tau_d"], rtol=1e-9, atol=0)
    assert np.allclose(pt[:, 1], ref["per_tau_x"], rtol=1e-9, atol=0)


def test_tiny_mesh_per_tau_entry_points(torch_cuda):
    # ltmp2_chi, ltmp2_exchange and ltmp2_direct_hartree return per-cell
    # values that match ltmp2_energy's per-tau terms
    from oracle.kpoints import KProblem
    from oracle.quadrature import minimax_laplace
    s = _tiny()
    n_k, n_occ = 2, 1
    kap, mills, eps, coeffs = make_cell_kmesh(s, n_k)
    K = KProblem(s.L, s.n, s.eaux, n_k, kap, mills, eps, coeffs, n_occ)
    tau, w, _ = minimax_laplace(*K.x_range(), 6)
    _say("tiny cell, k mesh 2, per-tau entry points")
    with _kctx(s, n_k, mills, eps, coeffs, n_occ, tau, w) as ctx:
        ed, ex, pt, qe = ctx.energy()
        for t in (0, 3, 5):
            d_chi = ctx.chi(t)
            d_h = ctx.direct_hartree(t)
            x = ctx.exchange(t)
            assert abs(d_chi - pt[t, 0]) <= 1e-12 * abs(pt[t, 0])
            assert abs(d_h - pt[t, 0]) <= 1e-10 * abs(pt[t, 0])
            assert abs(x - pt[t, 1]) <= 1e-12 * abs(pt[t, 1])


def test_single_point_mesh_equals_gamma_context(torch_cuda):
    from paper_1611_06797_amd import Context
    from oracle.quadrature import minimax_laplace
    s = dataclasses.replace(_tiny(amp=0.3), n_occ=2, n=12)   # a compiled grid
    kap, mills, eps, coeffs = make_cell_kmesh(s, 1)
    e0, c0 = eps[0], coeffs[0]
    tau, w, _ = minimax_laplace(2 * (e0[2] - e0[1]), 2 * (e0[-1] - e0[0]), 6)
    _say("k mesh 1 vs Gamma-only context")
    with _kctx(s, 1, mills, eps, coeffs, 2, tau, w) as ctx:
        a = ctx.energy()
    with Context(s.L, s.n, s.ecut, s.eaux, mills[0], e0, c0, 2, 6, tau=tau, w=w) as ctx:
        b = ctx.energy()
    assert abs(a[0] - b[0]) <= 1e-13 * abs(b[0]) and abs(a[1] - b[1]) <= 1e-13 * abs(b[1])


def test_tiny_mesh_cutoff_extrapolation(torch_cuda):
    # energies of the nested auxiliary cutoffs, per unit cell
    from oracle.kpoints import KProblem
    from oracle.quadrature import minimax_laplace
    from oracle.extrapolation import cutoffs
    s = _tiny()
    n_k, n_occ = 2, 1
    kap, mills, eps, coeffs = make_cell_kmesh(s, n_k)
    K = KProblem(s.L, s.n, s.eaux, n_k, kap, mills, eps, coeffs, n_occ)
    tau, w, _ = minimax_laplace(*K.x_range(), 6)
    _say("tiny cell, k mesh 2, cutoff extrapolation")
    with _kctx(s, n_k, mills, eps, coeffs, n_occ, tau, w, n_extrap=4) as ctx:
        ctx.energy()
        ea, edn, exn, einf = ctx.extrapolation(4)
    assert np.allclose(ea, cutoffs(s.eaux, 4), rtol=1e-15)
    for n, e_n in enumerate(ea):
        r = KProblem(s.L, s.n, e_n, n_k, kap, mills, eps, coeffs, n_occ).energies(tau, w)
        assert abs(edn[n] - r["e_d_lt"]) <= 1e-9 * abs(r["e_d_lt"])
        assert abs(exn[n] - r["e_x_lt"]) <= 1e-9 * abs(r["e_x_lt"])


@pytest.mark.parametrize("prec", [0, 2])
def test_c1_mesh_vs_stored_oracle(torch_cuda, prec):
    path = os.path.join(HERE, "golden", "c1_kmesh2.json")
    ref = json.load(open(path))
    n_k, n_occ = ref["n_k"], ref["n_occ"]
    kap, mills, eps, coeffs = make_cell_kmesh(C1, n_k)
    tau, w = np.array(ref["tau"]), np.array(ref["w"])
    _say("small workload cell, k mesh 2, prec", prec)
    with _kctx(C1, n_k, mills, eps, coeffs, n_occ, tau, w, prec=prec) as ctx:
        ed, ex, pt, qe = ctx.energy()
        info = ctx.info
    print(f"[c1 kmesh prec={prec}] n_grid={info.n_grid} n_g={info.n_g} n_pw={info.n_pw} "
          f"dE_d={ed - ref['e_d_lt']:.3e} dE_x={ex - ref['e_x_lt']:.3e}")
    assert abs(info.x_min - ref["x_min"]) <= 1e-12 and abs(info.x_max - ref["x_max"]) <= 1e-12
    if prec == 0:
        assert abs(ed - ref["e_d_lt"]) <= 1e-9 * abs(ref["e_d_lt"])
        assert abs(ex - ref["e_x_lt"]) <= 1e-9 * abs(ref["e_x_lt"])
        assert np.allclose(pt[:, 0], ref["per_tau_d"], rtol=1e-9, atol=0)
        assert np.allclose(pt[:, 1], ref["per_tau_x"], rtol=1e-9, atol=0)
    else:
        tol = n_k ** 3 * n_occ * 1e-6
        assert abs(ed - ref["e_d_lt"]) < tol and abs(ex - ref["e_x_lt"]) < tol
