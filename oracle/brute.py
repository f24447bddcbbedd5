"""Oracle: real-space brute force for tiny cells (no FFT anywhere).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Used to pin the FFT-based oracle.  Everything is an explicit sum over grid
points and plane waves:
  * psi_p(r) = Omega^(-1/2) sum_G c_p(G) exp(i G.r) as an explicit matrix;
  * Coulomb kernel on the grid K(d) = sum_{G in aux} v(G) exp(i G.d)
    (the G-sum of the Coulomb Fourier series, Appendix A, at k = 0);
  * <ij|ab> = dV^2 sum_{r,r'} psi_i* psi_a (r) K(r - r') psi_j* psi_b (r');
  * exchange at one Laplace point as the four-point contraction
    dV^4 sum K(r1-r2) K(r3-r4) G_occ(r4,r1) G_occ(r3,r2) G_vir(r1,r3) G_vir(r2,r4);
  * direct at one Laplace point as -2 dV^4 Tr[chi K chi K].
"""

from __future__ import annotations

import math

import numpy as np


def grid_points(L, n):
    k = np.arange(n)
    kx, ky, kz = np.meshgrid(k, k, k, indexing="ij")
    return (L / n) * np.stack([kx.ravel(), ky.ravel(), kz.ravel()], axis=1)


def plane_waves(L, n, miller):
    """[N_r, N_G] matrix exp(i G.r) with G = (2 pi / L) m."""
    r = grid_points(L, n)
    G = (2.0 * math.pi / L) * np.asarray(miller, float)
    return np.exp(1j * r @ G.T)


def orbitals(L, n, miller, coeff):
    """psi[p, r] by explicit plane-wave sums."""
    return (plane_waves(L, n, miller) @ np.asarray(coeff).T).T / math.sqrt(L ** 3)


def coulomb_matrix(L, n, aux, v):
    """K[r, r'] = sum_G v(G) exp(i G.(r - r'))."""
    P = plane_waves(L, n, aux)
    return (P * v[None, :]) @ np.conj(P).T


def integrals(L, n, psi, occ, vir, K):
    """<ij|ab>[i,j,a,b] and <ab|ji>[i,j,a,b] by double sums over the grid."""
    dV = L ** 3 / n ** 3
    po = psi[occ]
    pv = psi[vir]
    rho = np.conj(po)[:, None, :] * pv[None, :, :]           # psi_i* psi_a  [I, A, r]
    nI, nA = rho.shape[:2]
    R = rho.reshape(nI * nA, -1)
    M = (R @ K @ R.T).reshape(nI, nA, nI, nA) * dV ** 2      # <ij|ab> at [i,a,j,b]
    ijab = np.transpose(M, (0, 2, 1, 3))
    rho2 = np.conj(pv)[:, None, :] * po[None, :, :]           # psi_a* psi_j  [A, J, r]
    R2 = rho2.reshape(nA * nI, -1)
    M2 = (R2 @ K @ R2.T).reshape(nA, nI, nA, nI) * dV ** 2    # <ab|ji> at [a,j,b,i]
    abji = np.transpose(M2, (3, 1, 0, 2))
    return ijab, abji


def green(psi, eps, occ, vir, mu, tau):
    po = psi[occ]
    pv = psi[vir]
    fo = np.exp((eps[occ] - mu) * tau)
    fv = np.exp(-(eps[vir] - mu) * tau)
    Go = (po.T * fo[None, :]) @ np.conj(po)
    Gv = (pv.T * fv[None, :]) @ np.conj(pv)
    return Go, Gv


def exchange_four_point(L, n, Go, Gv, K):
    """dV^4 sum_{r1..r4} K12 K34 Go(r4,r1) Go(r3,r2) Gv(r1,r3) Gv(r2,r4)."""
    dV = L ** 3 / n ** 3
    total = 0.0 + 0.0j
    nr = Go.shape[0]
    for r1 in range(nr):
        U = Go.T * Gv[r1][None, :]          # U[r2, r3] = Go(r3, r2) Gv(r1, r3)
        V = Gv * Go[:, r1][None, :]         # V[r2, r4] = Go(r4, r1) Gv(r2, r4)
        total += (K[r1] * np.einsum("ij,ij->i", U @ K, V)).sum()
    return total * dV ** 4


def direct_four_point(L, n, Go, Gv, K):
    """-2 dV^4 Tr[chi K chi K] with chi(r, r') = Go(r, r') Gv(r', r)."""
    dV = L ** 3 / n ** 3
    chi = Go * Gv.T
    M = chi @ K
    return -2.0 * np.trace(M @ M) * dV ** 4
