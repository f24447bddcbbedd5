"""Pins of the k-point oracle (CPU only).

oracle.kpoints evaluates Eqs. 2eIPLWV / OverlapDens / MP2direct /
MP2ex_spinrestr with crystal momentum conservation on the unit-cell grid.
Pinned here against (a) the Gamma-only oracle for a 1-point mesh; (b) the
Gamma-only oracle on the Born-von Karman supercell, where the Bloch states
become ordinary supercell orbitals (Miller index n_k m + kappa, unchanged
coefficients) and the supercell energy is N times the energy per cell --
a route with no mesh bookkeeping, no q-dependent Coulomb kernel and no
lattice-vector shifts; (c) time-reversal and Laplace-bound properties.
"""
import dataclasses

import numpy as np
import pytest

from synthetic import make_cell_kmesh, tiny_spec, kpoint_miller
from oracle.kpoints import KProblem
from oracle.mp2 import Problem
from oracle.quadrature import minimax_laplace


def _kcase(n_k, amp=1.0, n_occ=1, seed=3):
    s = dataclasses.replace(tiny_spec(seed=seed, L=5.0, n=8, ecut=2.5, eaux=2.0, n_occ=n_occ),
                            amp=amp)
    kap, mills, eps, coeffs = make_cell_kmesh(s, n_k)
    K = KProblem(s.L, s.n, s.eaux, n_k, kap, mills, eps, coeffs, n_occ)
    return s, kap, mills, eps, coeffs, K


def _supercell(s, n_k, kap, mills, eps, coeffs, n_occ):
    """Bloch states as orbitals of the n_k^3 supercell (plain re-indexing)."""
    ms = np.concatenate([n_k * mills[t].astype(np.int64) + kap[t][None, :]
                         for t in range(len(kap))])
    order = np.lexsort((ms[:, 2], ms[:, 1], ms[:, 0]))
    ms = ms[order]
    pos = {tuple(v): c for c, v in enumerate(ms.tolist())}
    nb = eps.shape[1]
    C = np.zeros((len(kap) * nb, len(ms)), complex)
    E = np.zeros(len(kap) * nb)
    for t in range(len(kap)):
        cols = [pos[tuple(v)] for v in (n_k * mills[t].astype(np.int64) + kap[t]).tolist()]
        C[t * nb:(t + 1) * nb][:, cols] = coeffs[t]
        E[t * nb:(t + 1) * nb] = eps[t]
    o = np.argsort(E, kind="stable")
    return ms, E[o], C[o]


def test_single_point_mesh_is_gamma_only():
    s, kap, mills, eps, coeffs, K = _kcase(1, amp=0.3, n_occ=2)
    P = Problem(s.L, s.n, s.eaux, mills[0], eps[0], coeffs[0], 2)
    tau, w, _ = minimax_laplace(*P.x_range(), 6)
    a, b = K.energies(tau, w), P.energies(tau, w)
    for k in ("e_d", "e_x", "e_d_lt", "e_x_lt"):
        assert abs(a[k] - b[k]) <= 1e-12 * abs(b[k]), k


@pytest.mark.parametrize("n_occ,amp", [(1, 1.0), (2, 1.0)])
def test_mesh_equals_born_von_karman_supercell(n_occ, amp):
    n_k = 2
    s, kap, mills, eps, coeffs, K = _kcase(n_k, amp=amp, n_occ=n_occ)
    gap = eps[:, n_occ].min() - eps[:, n_occ - 1].max()
    assert gap > 0
    ms, E, C = _supercell(s, n_k, kap, mills, eps, coeffs, n_occ)
    P = Problem(n_k * s.L, n_k * s.n, s.eaux, ms, E, C, n_k ** 3 * n_occ)
    lo, hi = K.x_range()
    assert np.allclose(P.x_range(), (lo, hi), rtol=1e-14)
    tau, w, _ = minimax_laplace(lo, hi, 6)
    a, b = K.energies(tau, w), P.energies(tau, w)
    N = n_k ** 3
    for k in ("e_d", "e_x", "e_d_lt", "e_x_lt"):
        assert abs(a[k] - b[k] / N) <= 1e-11 * abs(a[k]), (k, a[k], b[k] / N)
    assert np.allclose(a["per_tau_d"], b["per_tau_d"] / N, rtol=1e-11, atol=0)
    assert np.allclose(a["per_tau_x"], b["per_tau_x"] / N, rtol=1e-11, atol=0)
    assert b["imag_x"] < 1e-12 * abs(b["e_x"])


def test_time_reversal_partners_and_bound():
    # the mesh is closed under k -> -k with equal energies; the Laplace error
    # of the direct term stays inside the quadrature's relative bound
    s, kap, mills, eps, coeffs, K = _kcase(2, amp=1.0, n_occ=1)
    for t, k in enumerate(kap):
        tp = K.k_index(-k)
        assert np.allclose(eps[t], eps[tp], rtol=0, atol=1e-12)
    for nt in (4, 6):
        tau, w, delta = minimax_laplace(*K.x_range(), nt)
        r = K.energies(tau, w)
        assert abs(r["e_d_lt"] - r["e_d"]) <= delta * abs(r["e_d"]) * (1 + 1e-9)
        assert r["e_d"] < 0


def test_k_miller_sphere():
    # the union of the per-k spheres is the supercell sphere |b_s M|^2 < 2 E_cut
    s = tiny_spec(seed=3, L=5.0, n=8, ecut=2.5)
    n_k = 2
    ms = []
    for kx in range(n_k):
        for ky in range(n_k):
            for kz in range(n_k):
                m = kpoint_miller(s.L, s.n, s.ecut, (kx, ky, kz), n_k).astype(np.int64)
                ms.append(n_k * m + np.array([kx, ky, kz]))
    ms = np.concatenate(ms)
    bs = 2 * np.pi / (n_k * s.L)
    assert (0.5 * bs * bs * (ms * ms).sum(1) < s.ecut).all()
    r = np.arange(-12, 13)
    mx, my, mz = np.meshgrid(r, r, r, indexing="ij")
    allm = np.stack([mx.ravel(), my.ravel(), mz.ravel()], 1)
    ref = allm[0.5 * bs * bs * (allm * allm).sum(1) < s.ecut * (1 - 1e-12)]
    assert len(ms) == len(ref) == len({tuple(v) for v in ms.tolist()})
