"""Oracle: canonical and Laplace-transformed MP2 for a Gamma-only cell.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Spin-restricted, closed shell, Hartree atomic units.  With spin sums done
(direct: Eq. MP2direct with sum_{ss'} -> 4 and the prefactor 1/2; exchange:
Eq. MP2ex_spinrestr, sum_s -> 2):

  E_d =  2 sum_{ijab} |<ij|ab>|^2 / D_ijab
  E_x = -  sum_{ijab} <ij|ab> <ab|ji> / D_ijab,   D = e_i + e_j - e_a - e_b < 0

with <ij|ab> = sum_{G in aux} v(G) n_ia(G) n_jb(-G) (Eq. SCH2EI) and
<ab|ji> = sum_G v(G) n_aj(G) n_bi(-G).  The Laplace transform of 1/D
(Eq. SCHLT) with a quadrature (tau_n, w_n) gives

  E_d^LT = -2 sum_n w_n sum_{ijab} |<ij|ab>|^2 exp(D tau_n)
  E_x^LT = +  sum_n w_n sum_{ijab} <ij|ab><ab|ji> exp(D tau_n).

The Green's-function quantities (occupied / virtual imaginary-time Green's
functions, chi = G_occ(r,r') G_vir(r',r), its double Fourier transform) and
the transformed states of Eqs. SCHnewstate / SCHtransmatrix with the
Fock-like contraction (Eq. SCHfocklike, discrete form with v on both Coulomb
lines) are written out from their definitions for intermediate checks.
Energies are shifted by mu = (e_HOMO + e_LUMO) / 2 inside the Green's
functions only (the shift cancels in every product that enters an energy).
"""

from __future__ import annotations

import math

import numpy as np

from .planewave import Cell, negate_index


class Problem:
    """One cell: orbitals on the grid, auxiliary set, Coulomb kernel.

    occ: indices of the occupied orbitals used (default: the first n_occ);
    every orbital with index >= n_occ is virtual.
    """

    def __init__(self, L, n, eaux, miller, eps, coeff, n_occ, occ=None):
        self.cell = Cell(L, n)
        self.miller = np.asarray(miller, np.int64)
        self.eps = np.asarray(eps, float)
        self.coeff = np.asarray(coeff, complex)
        self.n_occ = int(n_occ)
        self.occ = np.arange(self.n_occ) if occ is None else np.asarray(occ)
        self.vir = np.arange(self.n_occ, self.eps.shape[0])
        self.aux = self.cell.aux_miller(eaux)
        self.v = self.cell.coulomb(self.aux)
        self.neg = negate_index(self.aux)
        self.mu = 0.5 * (self.eps[self.n_occ - 1] + self.eps[self.n_occ])
        self._psi_o = None
        self._psi_v = None
        self._n_ov = None
        self._n_vo = None

    # --- orbitals and overlap densities -------------------------------------
    @property
    def psi_o(self):
        if self._psi_o is None:
            self._psi_o = self.cell.orbitals(self.miller, self.coeff[self.occ])
        return self._psi_o

    @property
    def psi_v(self):
        if self._psi_v is None:
            self._psi_v = self.cell.orbitals(self.miller, self.coeff[self.vir])
        return self._psi_v

    @property
    def n_ov(self):
        """n_ia(G) [I, A, G]."""
        if self._n_ov is None:
            self._n_ov = self.cell.pair_densities(self.psi_o, self.psi_v, self.aux)
        return self._n_ov

    @property
    def n_vo(self):
        """n_aj(G) [A, J, G]."""
        if self._n_vo is None:
            self._n_vo = self.cell.pair_densities(self.psi_v, self.psi_o, self.aux)
        return self._n_vo

    def x_range(self):
        """[x_min, x_max] bounding -D over all (i, j, a, b)."""
        eo = self.eps[self.occ]
        ev = self.eps[self.vir]
        return 2.0 * (ev.min() - eo.max()), 2.0 * (ev.max() - eo.min())

    # --- integrals and energies ---------------------------------------------
    def pair_integrals(self, i, j):
        """(K, X) with K[a,b] = <ij|ab>, X[a,b] = <ab|ji> (local indices)."""
        v = self.v
        K = (self.n_ov[i] * v[None, :]) @ self.n_ov[j][:, self.neg].T
        X = (self.n_vo[:, j] * v[None, :]) @ self.n_vo[:, i][:, self.neg].T
        return K, X

    def denominators(self, i, j):
        eo = self.eps[self.occ]
        ev = self.eps[self.vir]
        return eo[i] + eo[j] - ev[:, None] - ev[None, :]

    def energies(self, tau=None, w=None):
        """Canonical (O1) and, if (tau, w) is given, Laplace (O2) energies.

        Returns a dict with e_d, e_x (canonical) and, for the quadrature,
        e_d_lt, e_x_lt, per_tau_d [N_tau], per_tau_x [N_tau] (unweighted
        per-point values), plus the absolute-value sums that bound the
        Laplace error and the largest imaginary part seen in the exchange.
        """
        nI = len(self.occ)
        ed = ex = 0.0
        bound_x = 0.0
        imag_x = 0.0
        nt = 0 if tau is None else len(tau)
        pd = np.zeros(nt)
        px = np.zeros(nt)
        for i in range(nI):
            for j in range(nI):
                K, X = self.pair_integrals(i, j)
                D = self.denominators(i, j)
                KK = (K * np.conj(K)).real
                KX = K * X
                ed += 2.0 * (KK / D).sum()
                cx = (KX / D).sum()
                ex += -cx.real
                imag_x = max(imag_x, abs(cx.imag))
                bound_x += (np.abs(KX) / np.abs(D)).sum()
                for n in range(nt):
                    f = np.exp(D * tau[n])
                    pd[n] += -2.0 * (KK * f).sum()
                    px[n] += (KX * f).sum().real
        out = dict(e_d=ed, e_x=ex, bound_x=bound_x, imag_x=imag_x)
        if nt:
            out.update(per_tau_d=pd, per_tau_x=px,
                       e_d_lt=float(np.dot(w, pd)), e_x_lt=float(np.dot(w, px)))
        return out

    # --- Green's functions (small cells only) -------------------------------
    def green(self, tau):
        """G_occ(r, r') and G_vir(r, r') as dense [N_r, N_r] matrices."""
        po = self.psi_o.reshape(len(self.occ), -1)
        pv = self.psi_v.reshape(len(self.vir), -1)
        fo = np.exp((self.eps[self.occ] - self.mu) * tau)
        fv = np.exp(-(self.eps[self.vir] - self.mu) * tau)
        Go = (po.T * fo[None, :]) @ np.conj(po)
        Gv = (pv.T * fv[None, :]) @ np.conj(pv)
        return Go, Gv

    def chi_rr(self, tau):
        """chi(r, r') = G_occ(r, r') G_vir(r', r)."""
        Go, Gv = self.green(tau)
        return Go * Gv.T

    def chi_GG(self, tau):
        """chi(G, G') = dV^2 sum_{r,r'} e^{-iG.r} chi(r,r') e^{+iG'.r'} on aux x aux."""
        n = self.cell.n
        c = self.chi_rr(tau).reshape(n, n, n, n, n, n)
        c = np.fft.fftn(c, axes=(0, 1, 2))
        c = np.fft.ifftn(c, axes=(3, 4, 5)) * self.cell.nr
        ix, iy, iz = self.cell.grid_index(self.aux)
        out = c[ix, iy, iz][:, ix, iy, iz]
        return out * self.cell.dV ** 2

    def direct_trace(self, tau):
        """E_d(tau) = -2 sum_{G,G'} v(G) v(G') |chi(G,G')|^2."""
        C = self.chi_GG(tau)
        return -2.0 * float((self.v[:, None] * self.v[None, :] * np.abs(C) ** 2).sum())

    # --- transformed states and the Fock-like factorisation ------------------
    def transformed_states(self, tau, g):
        """w_j^{(G')}(r) for all occupied j at G' = aux[g] [J, n, n, n].

        C_ja = exp((e_j - mu) tau) exp(-(e_a - mu) tau) <a|e^{-iG'r}|j>
        (Eq. SCHtransmatrix), w_j = sum_a C_ja psi_a (Eq. SCHnewstate).
        """
        fo = np.exp((self.eps[self.occ] - self.mu) * tau)
        fv = np.exp(-(self.eps[self.vir] - self.mu) * tau)
        C = fo[:, None] * fv[None, :] * self.n_vo[:, :, g].T      # [J, A]
        return np.tensordot(C, self.psi_v, axes=(1, 0))

    def fock_overlaps(self, tau, g):
        """A[i, j, G] = dV sum_r psi_i*(r) w_j^{(G')}(r) e^{-iG.r}."""
        w = self.transformed_states(tau, g)
        return self.cell.pair_densities(self.psi_o, w, self.aux)

    def exchange_partial(self, tau, g):
        """S_x(G') = sum_G v(G) sum_ij A^{G'}_ij(G) A^{-G'}_ji(-G)."""
        A = self.fock_overlaps(tau, g)
        B = self.fock_overlaps(tau, self.neg[g])
        Bt = np.transpose(B, (1, 0, 2))[:, :, self.neg]
        return complex((A * Bt * self.v[None, None, :]).sum())

    def exchange_tau(self, tau):
        """E_x(tau) = sum_{G'} v(G') S_x(G') (all G' of the auxiliary set)."""
        return sum(self.v[g] * self.exchange_partial(tau, g) for g in range(len(self.aux)))

    def direct_partial(self, tau, g, chi=None):
        """S_d(G') = sum_G v(G) |chi(G, G')|^2 for G' = aux[g]."""
        C = self.chi_GG(tau) if chi is None else chi
        return float((self.v * np.abs(C[:, g]) ** 2).sum())
