"""Pins of the spin-unrestricted oracle (CPU only).

The oracle sums Eqs. MP2direct / MP2exchange channel by channel.  It is
pinned here against (a) the textbook spin-orbital form of second-order
energy, 1/4 sum |<IJ||AB>|^2 / D over spin orbitals with antisymmetrised
integrals, evaluated by real-space double sums (no FFT, no pair densities);
(b) the spin-restricted oracle when both channels are the same; (c) the
symmetry under exchanging the channels; (d) the Laplace error bound of the
common quadrature; (e) its Green's-function forms per Laplace point.
"""
import numpy as np
import pytest

from synthetic import make_cell, make_cell_spin, tiny_spec
from oracle import brute
from oracle.mp2 import Problem
from oracle.quadrature import minimax_laplace
from oracle.unrestricted import UProblem


@pytest.fixture(scope="module")
def tiny_spin():
    s = tiny_spec(seed=3, L=5.0, n=8, ecut=2.5, eaux=2.0, n_occ=3)
    m, e1, c1, e2, c2 = make_cell_spin(s, n_occ_b=2, split=0.15, split_seed=11)
    U = UProblem(s.L, s.n, s.eaux, m, e1, c1, 3, e2, c2, 2)
    return s, m, e1, c1, e2, c2, U


def _spin_orbital_mp2(s, m, chans, aux, v):
    """1/4 sum_{IJAB} |<IJ|AB> - <IJ|BA>|^2 / (e_I + e_J - e_A - e_B) over spin
    orbitals, with <IJ|AB> = dV^2 sum_{r r'} phi_I* phi_A(r) K(r - r')
    phi_J* phi_B(r') when I, A share a spin and J, B share a spin, else 0.
    Returns (total, opposite-spin part)."""
    K = brute.coulomb_matrix(s.L, s.n, aux, v)
    dV = s.L ** 3 / s.n ** 3
    occ, vir = [], []  # (spin, orbital on the grid, energy)
    for sp, (eps, coeff, no) in enumerate(chans):
        psi = brute.orbitals(s.L, s.n, m, coeff)
        occ += [(sp, psi[i], eps[i]) for i in range(no)]
        vir += [(sp, psi[a], eps[a]) for a in range(no, len(eps))]
    nI, nA = len(occ), len(vir)
    rho = np.zeros((nI, nA, K.shape[0]), complex)
    for I, (si, pi, _) in enumerate(occ):
        for A, (sa, pa, _) in enumerate(vir):
            if si == sa:
                rho[I, A] = np.conj(pi) * pa
    R = rho.reshape(nI * nA, -1)
    M = ((R @ K @ R.T) * dV ** 2).reshape(nI, nA, nI, nA)   # <IJ|AB> at [I, A, J, B]
    ijab = np.transpose(M, (0, 2, 1, 3))                     # [I, J, A, B]
    anti = ijab - np.transpose(ijab, (0, 1, 3, 2))
    eo = np.array([x[2] for x in occ])
    ev = np.array([x[2] for x in vir])
    D = eo[:, None, None, None] + eo[None, :, None, None] - ev[None, None, :, None] \
        - ev[None, None, None, :]
    T = 0.25 * np.abs(anti) ** 2 / D
    so = np.array([x[0] for x in occ])
    opp = so[:, None] != so[None, :]
    return float(T.sum()), float(T[opp].sum())


def test_spin_orbital_brute_force(tiny_spin):
    # the channel sums equal the antisymmetrised spin-orbital energy, and the
    # opposite-spin part of the latter is the cross-channel direct term
    s, m, e1, c1, e2, c2, U = tiny_spin
    r = U.energies()
    tot, opp = _spin_orbital_mp2(s, m, [(e1, c1, 3), (e2, c2, 2)], U.ch[0].aux, U.v)
    assert abs(r["e_d"] + r["e_x"] - tot) <= 1e-12 * abs(tot)
    assert abs(r["e_d_os"] - opp) <= 1e-12 * abs(opp)
    assert r["e_d"] < 0 and r["e_x"] > 0 and r["e_d_os"] < 0


def test_identical_channels_reduce_to_restricted():
    s = tiny_spec(seed=5, L=5.0, n=8, ecut=2.5, eaux=2.0, n_occ=3)
    m, e, c = make_cell(s)
    P = Problem(s.L, s.n, s.eaux, m, e, c, 3)
    U = UProblem(s.L, s.n, s.eaux, m, e, c, 3, e, c, 3)
    tau, w, _ = minimax_laplace(*P.x_range(), 6)
    rp, ru = P.energies(tau, w), U.energies(tau, w)
    for k in ("e_d", "e_x", "e_d_lt", "e_x_lt"):
        assert abs(rp[k] - ru[k]) <= 1e-13 * abs(rp[k]), k
    assert np.allclose(rp["per_tau_d"], ru["per_tau_d"], rtol=1e-13, atol=0)
    assert np.allclose(rp["per_tau_x"], ru["per_tau_x"], rtol=1e-13, atol=0)
    # with identical channels half of the direct term is opposite-spin
    assert abs(ru["e_d_os"] - 0.5 * ru["e_d"]) <= 1e-13 * abs(ru["e_d"])


def test_channel_swap_symmetry(tiny_spin):
    s, m, e1, c1, e2, c2, U = tiny_spin
    V = UProblem(s.L, s.n, s.eaux, m, e2, c2, 2, e1, c1, 3)
    tau, w, _ = minimax_laplace(*U.x_range(), 6)
    a, b = U.energies(tau, w), V.energies(tau, w)
    for k in ("e_d", "e_x", "e_d_os", "e_d_lt", "e_x_lt"):
        assert abs(a[k] - b[k]) <= 1e-13 * abs(a[k]), k


def test_common_quadrature_error_bound(tiny_spin):
    # one quadrature on [2 min gap, 2 max spread] covers every denominator of
    # both channels and their cross pairs: |E^LT - E| <= delta * sum |terms|
    s, m, e1, c1, e2, c2, U = tiny_spin
    xmin, xmax = U.x_range()
    lo = 2 * min(e1[3] - e1[2], e2[2] - e2[1])
    hi = 2 * max(e1[-1] - e1[0], e2[-1] - e2[0])
    assert abs(xmin - lo) < 1e-14 and abs(xmax - hi) < 1e-14
    for nt in (6, 8):
        tau, w, delta = minimax_laplace(xmin, xmax, nt)
        r = U.energies(tau, w)
        bx = 0.5 * sum(p.energies()["bound_x"] for p in U.ch)
        assert abs(r["e_d_lt"] - r["e_d"]) <= delta * abs(r["e_d"]) * (1 + 1e-9)
        assert abs(r["e_x_lt"] - r["e_x"]) <= delta * bx * (1 + 1e-9)


def test_green_function_forms_per_tau(tiny_spin):
    # -1/2 v v |chi_1 + chi_2|^2 and 1/2 (X_1 + X_2) equal the integral sums
    s, m, e1, c1, e2, c2, U = tiny_spin
    tau = np.array([0.4, 2.5])
    r = U.energies(tau, np.ones(2))
    for k, t in enumerate(tau):
        assert abs(U.direct_trace(t) - r["per_tau_d"][k]) <= 1e-12 * abs(r["per_tau_d"][k])
        x = U.exchange_tau(t)
        assert abs(x.imag) < 1e-14
        assert abs(x.real - r["per_tau_x"][k]) <= 1e-12 * abs(r["per_tau_x"][k])
