"""Oracle: plane-wave grid objects for a Gamma-only cubic cell.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Definitions follow the Theory section ("Reducing the computational cost"):
  * plane wave <r|G> = Omega^(-1/2) exp(i G.r), so an orbital is
    psi_p(r) = Omega^(-1/2) sum_{G in B} c_p(G) exp(i G.r)  (inverse FFT);
  * overlap density <p| exp(-i G r) |q> = int psi_p* psi_q exp(-i G.r)
    (Eq. SCHovrlp), on the grid  n_pq(G) = dV sum_r psi_p*(r) psi_q(r) e^{-iG.r};
  * Coulomb kernel of Eq. SCH2EI: 4 pi / (Omega |G|^2) on the auxiliary set
    G != 0 with |G|^2 / 2 <= E_aux (auxiliary cutoff, ENCUTGW); the G = 0
    term is absent (n_pq(0) = <p|q> = 0 for p != q on the grid anyway).
The grid point r_k = L k / n, dV = Omega / n^3; G.r_k = 2 pi m.k / n.
"""

from __future__ import annotations

import math

import numpy as np


class Cell:
    """Geometry of one cubic cell with an n^3 FFT grid."""

    def __init__(self, L: float, n: int):
        self.L = float(L)
        self.n = int(n)
        self.omega = self.L ** 3
        self.b = 2.0 * math.pi / self.L
        self.nr = self.n ** 3
        self.dV = self.omega / self.nr

    def aux_miller(self, eaux: float) -> np.ndarray:
        """Auxiliary set: m != 0 with |b m|^2 / 2 <= eaux (inclusive)."""
        lim = int(math.floor(2.0 * eaux / (self.b * self.b) + 1e-9))
        mm = int(math.isqrt(lim))
        r = np.arange(-mm, mm + 1)
        mx, my, mz = np.meshgrid(r, r, r, indexing="ij")
        m = np.stack([mx.ravel(), my.ravel(), mz.ravel()], axis=1)
        m2 = (m * m).sum(1)
        m = m[(m2 <= lim) & (m2 > 0)]
        if np.any(2 * np.abs(m) >= self.n):
            raise ValueError("auxiliary sphere does not fit inside the FFT grid")
        return m.astype(np.int64)

    def coulomb(self, miller: np.ndarray) -> np.ndarray:
        """v(G) = 4 pi / (Omega |G|^2)."""
        g2 = self.b * self.b * (miller * miller).sum(1)
        return 4.0 * math.pi / (self.omega * g2)

    def grid_index(self, miller: np.ndarray):
        """Index tuple of each m on the n^3 FFT array (m mod n)."""
        m = np.mod(miller, self.n)
        return m[:, 0], m[:, 1], m[:, 2]

    def orbitals(self, miller: np.ndarray, coeff: np.ndarray) -> np.ndarray:
        """psi[p, x, y, z] = Omega^(-1/2) sum_G c_p(G) e^{i G.r} (complex)."""
        n = self.n
        ix, iy, iz = self.grid_index(miller)
        out = np.empty((coeff.shape[0], n, n, n), complex)
        A = np.zeros((n, n, n), complex)
        for p in range(coeff.shape[0]):
            A[:] = 0.0
            A[ix, iy, iz] = coeff[p]
            out[p] = np.fft.ifftn(A) * (self.nr / math.sqrt(self.omega))
        return out

    def pair_densities(self, psi_p: np.ndarray, psi_q: np.ndarray,
                       miller: np.ndarray) -> np.ndarray:
        """n[p, q, G] = dV sum_r psi_p*(r) psi_q(r) e^{-i G.r} for G in miller."""
        ix, iy, iz = self.grid_index(miller)
        out = np.empty((psi_p.shape[0], psi_q.shape[0], miller.shape[0]), complex)
        for a in range(psi_p.shape[0]):
            cp = np.conj(psi_p[a])
            for b in range(psi_q.shape[0]):
                F = np.fft.fftn(cp * psi_q[b])
                out[a, b] = self.dV * F[ix, iy, iz]
        return out


def negate_index(miller: np.ndarray) -> np.ndarray:
    """Permutation k -> index of -m_k within the same (symmetric) set."""
    pos = {tuple(v): k for k, v in enumerate(np.asarray(miller).tolist())}
    return np.array([pos[(-a, -b, -c)] for a, b, c in np.asarray(miller).tolist()])
