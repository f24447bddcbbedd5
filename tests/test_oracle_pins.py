"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test would fail under a plausible mistake in the oracle: a dropped
Coulomb factor, a wrong sign or conjugation, a transposed operand, a wrong
prefactor of the direct or exchange term, or a broken Laplace weight.
"""
import math

import numpy as np
import pytest

from synthetic import make_cell, tiny_spec, random_unitary, C1
from oracle.mp2 import Problem
from oracle import brute
from oracle.quadrature import minimax_laplace


def _tiny(seed=3, **kw):
    s = tiny_spec(seed=seed, **kw)
    m, e, c = make_cell(s)
    return s, m, e, c, Problem(s.L, s.n, s.eaux, m, e, c, s.n_occ)


@pytest.fixture(scope="module")
def tiny():
    return _tiny(seed=3, L=5.0, n=8, ecut=2.5, eaux=2.0, n_occ=3)


@pytest.fixture(scope="module")
def c1():
    m, e, c = make_cell(C1)
    P = Problem(C1.L, C1.n, C1.eaux, m, e, c, C1.n_occ)
    return m, e, c, P


def test_counts_c1(c1):
    # basis and auxiliary sizes of the small workload (cutoffs: strict / inclusive)
    m, e, c, P = c1
    assert m.shape[0] == 365
    assert len(P.aux) == 178


def test_overlap_densities_orthogonality(tiny):
    # n_pq(0) = <p|q> = delta_pq on the grid (discrete Parseval)
    s, m, e, c, P = tiny
    psi = P.cell.orbitals(m, c)
    n0 = P.cell.pair_densities(psi, psi, np.zeros((1, 3), np.int64))[:, :, 0]
    assert np.allclose(n0, np.eye(len(e)), atol=1e-12)


def test_brute_integrals(tiny):
    # P1(a): FFT pair densities x Coulomb sum == real-space double sums
    s, m, e, c, P = tiny
    psi = brute.orbitals(s.L, s.n, m, c)
    K = brute.coulomb_matrix(s.L, s.n, P.aux, P.v)
    ijab, abji = brute.integrals(s.L, s.n, psi, P.occ, P.vir, K)
    for i in range(s.n_occ):
        for j in range(s.n_occ):
            Kij, Xij = P.pair_integrals(i, j)
            assert np.abs(Kij - ijab[i, j]).max() < 1e-13
            assert np.abs(Xij - abji[i, j]).max() < 1e-13


def test_brute_four_point_per_tau(tiny):
    # P1(b,c): per-tau exchange and direct terms == O(N_r^4) real-space forms
    s, m, e, c, P = tiny
    tau = np.array([0.3, 1.7, 6.0])
    out = P.energies(tau, np.ones(3))
    psi = brute.orbitals(s.L, s.n, m, c)
    K = brute.coulomb_matrix(s.L, s.n, P.aux, P.v)
    for k, t in enumerate(tau):
        Go, Gv = brute.green(psi, e, P.occ, P.vir, P.mu, t)
        ex = brute.exchange_four_point(s.L, s.n, Go, Gv, K)
        ed = brute.direct_four_point(s.L, s.n, Go, Gv, K)
        assert abs(ex.imag) < 1e-14 and abs(ed.imag) < 1e-14
        assert abs(ex.real - out["per_tau_x"][k]) <= 1e-12 * abs(ex.real)
        assert abs(ed.real - out["per_tau_d"][k]) <= 1e-12 * abs(ed.real)


def test_chi_trace_and_fock_factorisation(tiny):
    # Green's-function direct route and the paper's transformed-state exchange route
    # reproduce the per-tau Laplace terms exactly
    s, m, e, c, P = tiny
    tau = np.array([0.5, 2.5])
    out = P.energies(tau, np.ones(2))
    for k, t in enumerate(tau):
        assert abs(P.direct_trace(t) - out["per_tau_d"][k]) <= 1e-12 * abs(out["per_tau_d"][k])
        ex = P.exchange_tau(t)
        assert abs(ex.imag) < 1e-14
        assert abs(ex.real - out["per_tau_x"][k]) <= 1e-12 * abs(out["per_tau_x"][k])


def test_chi_hermitian_psd(tiny):
    # P6: chi(G, G') is Hermitian and positive semidefinite, so E_d(tau) <= 0
    s, m, e, c, P = tiny
    C = P.chi_GG(1.1)
    assert np.abs(C - C.conj().T).max() < 1e-14 * np.abs(C).max()
    ev = np.linalg.eigvalsh(0.5 * (C + C.conj().T))
    assert ev.min() > -1e-12 * ev.max()
    assert P.direct_trace(1.1) < 0


def test_alias_free_pair_density_is_exact_convolution():
    # P2: on an alias-free grid the FFT pair density equals the continuum
    # plane-wave convolution sum_G1 c_i*(G1) c_a(G1 + G)
    s, m, e, c, P = _tiny(seed=5, L=5.0, n=12, ecut=2.0, eaux=1.5, n_occ=2)
    mmax = np.abs(m).max()
    maux = np.abs(P.aux).max()
    assert s.n > 2 * mmax + maux
    pos = {tuple(v): k for k, v in enumerate(m.tolist())}
    n_ov = P.n_ov
    for i in range(2):
        for a in [0, 3, 7]:
            for g, G in enumerate(P.aux.tolist()):
                ref = 0.0
                for k1, G1 in enumerate(m.tolist()):
                    k2 = pos.get((G1[0] + G[0], G1[1] + G[1], G1[2] + G[2]))
                    if k2 is not None:
                        ref += np.conj(c[P.occ[i], k1]) * c[P.vir[a], k2]
                assert abs(n_ov[i, a, g] - ref) < 1e-13


def test_laplace_bound_and_convergence(c1):
    # P3: |E_d^LT - E_d| <= delta |E_d| (all direct terms share a sign);
    # |E_x^LT - E_x| <= delta sum |<ij|ab><ab|ji>| / |D|; and E^LT -> E
    m, e, c, P = c1
    xmin, xmax = P.x_range()
    prev = None
    for nt in (4, 8, 12):
        tau, w, d = minimax_laplace(xmin, xmax, nt)
        out = P.energies(tau, w)
        assert abs(out["e_d_lt"] - out["e_d"]) <= d * abs(out["e_d"]) * (1 + 1e-9)
        assert abs(out["e_x_lt"] - out["e_x"]) <= d * out["bound_x"] * (1 + 1e-9)
        err = abs(out["e_d_lt"] + out["e_x_lt"] - out["e_d"] - out["e_x"])
        if prev is not None:
            assert err < prev
        prev = err
    assert out["imag_x"] <= 1e-12 * abs(out["e_x"])
    assert out["e_d"] < 0 < out["e_x"]


def test_phase_invariance(tiny):
    # P4(i): random phases on every orbital leave energies, G_occ and chi fixed
    s, m, e, c, P = tiny
    rng = np.random.default_rng(11)
    ph = np.exp(1j * rng.uniform(0, 2 * np.pi, len(e)))
    Q = Problem(s.L, s.n, s.eaux, m, e, c * ph[:, None], s.n_occ)
    a = P.energies([0.7], [1.0])
    b = Q.energies([0.7], [1.0])
    for k in ("e_d", "e_x", "per_tau_d", "per_tau_x"):
        assert np.allclose(a[k], b[k], rtol=1e-12, atol=0)
    Ga, _ = P.green(0.7)
    Gb, _ = Q.green(0.7)
    assert np.abs(Ga - Gb).max() < 1e-13
    assert np.abs(P.chi_GG(0.7) - Q.chi_GG(0.7)).max() < 1e-13


def test_occupied_rotation_invariance(tiny):
    # P4(ii): psi' = psi U with non-canonical F_oo = U^H diag(e_o) U; the
    # occupied Green's function built with expm(tau (F_oo - mu)) is unchanged,
    # and re-diagonalising F_oo recovers the canonical energies
    s, m, e, c, P = tiny
    no = s.n_occ
    U = random_unitary(no, 7)
    co = U.T @ c[:no]                       # rows: rotated occupied states
    F = U.conj().T @ np.diag(e[:no]) @ U
    tau = 1.3
    psi_r = P.cell.orbitals(m, co).reshape(no, -1)
    lam, V = np.linalg.eigh(F - P.mu * np.eye(no))
    Ef = V @ np.diag(np.exp(lam * tau)) @ V.conj().T
    Go_rot = psi_r.T @ Ef @ np.conj(psi_r)
    Go, _ = P.green(tau)
    assert np.abs(Go_rot - Go).max() < 1e-12
    ev, W = np.linalg.eigh(F)
    c_back = np.concatenate([W.T @ co, c[no:]])
    Q = Problem(s.L, s.n, s.eaux, m, np.concatenate([ev, e[no:]]), c_back, no)
    a = P.energies()
    b = Q.energies()
    assert abs(a["e_d"] - b["e_d"]) < 1e-13 and abs(a["e_x"] - b["e_x"]) < 1e-13


def test_single_occupied_exchange_is_minus_half_direct():
    # P5: with one occupied orbital <ab|ji> = <ab|ii> = conj<ii|ab> for real
    # orbitals... in general E_x = -E_d / 2 exactly (same integrals, K X = |K|^2)
    s, m, e, c, P = _tiny(seed=4, L=5.0, n=8, ecut=2.5, eaux=2.0, n_occ=1)
    out = P.energies([0.4, 2.0], [1.0, 1.0])
    assert abs(out["e_x"] + 0.5 * out["e_d"]) < 1e-14 * abs(out["e_d"])
    assert np.allclose(out["per_tau_x"], -0.5 * out["per_tau_d"], rtol=1e-13)


def test_pair_symmetry(tiny):
    # P6: swapping the two electrons maps pair (i, j) onto (j, i)
    s, m, e, c, P = tiny
    K01, X01 = P.pair_integrals(0, 1)
    K10, X10 = P.pair_integrals(1, 0)
    assert np.abs(K01 - K10.T).max() < 1e-14
    assert np.abs(X01 - X10.T).max() < 1e-14


@pytest.mark.parametrize("L,n", [(16.0, 100), (20.0, 128)])
def test_coulomb_kernel_absolute_normalisation(L, n):
    # Appendix "Two-electron integrals in the plane wave basis": the periodic
    # Coulomb energy of a charge density is (1/2) sum_{G != 0} v(G) |rho(G)|^2
    # with v(G) = 4 pi / (Omega |G|^2).  For a neutral pair of unit Gaussian
    # charges (exponent alpha, distance d) in a cubic cell that energy is the
    # isolated pair's sqrt(2 alpha / pi) - erf(sqrt(alpha / 2) d) / d, minus
    # the cubic-cell dipole term 2 pi d^2 / (3 Omega) that dropping G = 0
    # implies, up to O(d^4 / L^5).  The densities are built twice: in closed
    # form and on the grid through the oracle's pair densities (dV sum_r
    # e^{-iG.r}).  A wrong 4 pi, Omega power or dV fails by orders of
    # magnitude; the residual must fall like L^-5.
    from scipy.special import erf
    from oracle.planewave import Cell
    alpha, d = 2.0, 1.0
    cell = Cell(L, n)
    aux = cell.aux_miller(160.0)
    v = cell.coulomb(aux)
    G = cell.b * aux.astype(float)
    R1 = np.array([L / 2 - d / 2, L / 2, L / 2])
    R2 = R1 + np.array([d, 0.0, 0.0])
    rho = np.exp(-(G * G).sum(1) / (4 * alpha)) * (np.exp(-1j * G @ R1) - np.exp(-1j * G @ R2))
    e_pw = 0.5 * float((v * np.abs(rho) ** 2).sum())
    omega = L ** 3
    e_cf = (math.sqrt(2 * alpha / math.pi) - erf(math.sqrt(alpha / 2) * d) / d
            - 2 * math.pi * d * d / (3 * omega))
    resid_20 = 1.0e-6                       # O(L^-5) multipole residual at L = 20
    bound = 2.0 * resid_20 * (20.0 / L) ** 5
    assert abs(e_pw - e_cf) <= bound, (e_pw, e_cf)
    x = np.arange(n) * L / n
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")

    def gauss(R):
        dx, dy, dz = ((A - c + L / 2) % L - L / 2 for A, c in zip((X, Y, Z), R))
        return (alpha / math.pi) ** 1.5 * np.exp(-alpha * (dx * dx + dy * dy + dz * dz))

    rg = gauss(R1) - gauss(R2)
    nd = cell.pair_densities(np.ones((1, n, n, n)), rg[None], aux)[0, 0]
    e_grid = 0.5 * float((v * np.abs(nd) ** 2).sum())
    assert abs(e_grid - e_cf) <= bound, (e_grid, e_cf)


def test_extrapolation_line_fit_recovers_the_decay_law():
    # y = a + b E^(-3/2) sampled at the cutoff array is fitted exactly; a
    # noisy sample is fitted to within its noise (least squares)
    from oracle.extrapolation import cutoffs, extrapolate
    e = cutoffs(5.0)
    assert np.allclose(e, [5.0 / 1.05 ** k for k in range(8)], rtol=1e-15)
    a, b = extrapolate(e, -1.25 + 0.37 * e ** -1.5)
    assert abs(a + 1.25) < 1e-13 and abs(b - 0.37) < 1e-12
    rng = np.random.default_rng(4)
    y = -1.25 + 0.37 * e ** -1.5 + rng.normal(0, 1e-9, e.size)
    a, b = extrapolate(e, y)
    X = np.stack([np.ones_like(e), e ** -1.5], 1)
    ref = np.linalg.lstsq(X, y, rcond=None)[0]
    assert abs(a - ref[0]) < 1e-12 and abs(b - ref[1]) < 1e-10


def test_extrapolation_cutoff_energies_nested():
    # the direct term sums non-negative contributions over nested auxiliary
    # sets: E_d[n] is non-decreasing in n (less negative for smaller sets),
    # and E[1] is the energy at the user-given cutoff
    from oracle.extrapolation import energies_at_cutoffs
    spec = tiny_spec(seed=2, L=6.0, n=10, ecut=3.0, eaux=3.0, n_occ=2)
    m, e, c = make_cell(spec)
    P = Problem(spec.L, spec.n, spec.eaux, m, e, c, spec.n_occ)
    tau, w, _ = minimax_laplace(*P.x_range(), 6)
    ed, ex = energies_at_cutoffs(spec.L, spec.n, spec.eaux, m, e, c, spec.n_occ, tau, w)
    full = P.energies(tau, w)
    assert abs(ed[0] - full["e_d_lt"]) < 1e-14 and abs(ex[0] - full["e_x_lt"]) < 1e-14
    assert np.all(np.diff(ed) >= -1e-15) and ed[-1] > ed[0]
