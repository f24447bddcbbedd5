"""Oracle: spin-unrestricted MP2 for a Gamma-only cell.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this.

Theory section, Eqs. MP2direct and MP2exchange at the Gamma point (N = 1,
one k-point): the Coulomb operator keeps each electron's spin, so an
integral <ij|ab> is nonzero only when a has i's spin and b has j's.  With
D = e_i + e_j - e_a - e_b < 0 and the two channels s, s' in {1, 2}:

  E_d =  1/2 sum_{s s'} sum_{i,a in s} sum_{j,b in s'} |<ij|ab>|^2 / D
  E_x = -1/2 sum_s      sum_{i,j,a,b in s}  <ij|ab> <ab|ji> / D

where <ij|ab> = sum_{G in aux} v(G) n_ia(G) n_jb(-G) (Eq. SCH2EI) with each
overlap density taken from its own channel's orbitals.  The Laplace
transform of 1/D (Eq. SCHLT) with one quadrature (tau_n, w_n) for both
channels gives

  E_d^LT = -1/2 sum_n w_n sum_{s s'} sum |<ij|ab>|^2 exp(D tau_n)
  E_x^LT = +1/2 sum_n w_n sum_s      sum <ij|ab><ab|ji> exp(D tau_n).

Green's-function forms (for intermediate checks): chi_s(r, r') of each
channel as in the spin-restricted oracle; the direct value at one Laplace
point is -1/2 sum_{G G'} v(G) v(G') |chi_1(G, G') + chi_2(G, G')|^2 (the
sum over s s' of the cross traces), and the exchange value is 1/2 the sum of
the two channels' spin-restricted exchange values.
"""

from __future__ import annotations

import numpy as np

from .mp2 import Problem


class UProblem:
    """Two spin channels on one basis and one auxiliary set."""

    def __init__(self, L, n, eaux, miller, eps_1, coeff_1, n_occ_1, eps_2, coeff_2, n_occ_2):
        self.ch = (Problem(L, n, eaux, miller, eps_1, coeff_1, n_occ_1),
                   Problem(L, n, eaux, miller, eps_2, coeff_2, n_occ_2))
        self.v = self.ch[0].v
        self.neg = self.ch[0].neg

    def x_range(self):
        """[x_min, x_max] bounding -D over both channels and their pairs."""
        lo = [p.x_range()[0] for p in self.ch]
        hi = [p.x_range()[1] for p in self.ch]
        return min(lo), max(hi)

    def integrals(self, s, t, i, j):
        """<ij|ab> [a, b] for i, a of channel s and j, b of channel t."""
        P, Q = self.ch[s], self.ch[t]
        return (P.n_ov[i] * self.v[None, :]) @ Q.n_ov[j][:, self.neg].T

    def exchange_integrals(self, s, i, j):
        """<ab|ji> [a, b], all four states of channel s."""
        P = self.ch[s]
        return (P.n_vo[:, j] * self.v[None, :]) @ P.n_vo[:, i][:, self.neg].T

    def denominators(self, s, t, i, j):
        P, Q = self.ch[s], self.ch[t]
        eo_s, ev_s = P.eps[P.occ], P.eps[P.vir]
        eo_t, ev_t = Q.eps[Q.occ], Q.eps[Q.vir]
        return eo_s[i] + eo_t[j] - ev_s[:, None] - ev_t[None, :]

    def energies(self, tau=None, w=None):
        """Canonical and, with (tau, w), Laplace energies.

        Returns e_d, e_x, e_d_os (the part of e_d with s != s'), and for the
        quadrature e_d_lt, e_x_lt, per_tau_d, per_tau_x (unweighted).
        """
        nt = 0 if tau is None else len(tau)
        ed = ex = ed_os = 0.0
        pd = np.zeros(nt)
        px = np.zeros(nt)
        for s in range(2):
            for t in range(2):
                for i in range(len(self.ch[s].occ)):
                    for j in range(len(self.ch[t].occ)):
                        K = self.integrals(s, t, i, j)
                        D = self.denominators(s, t, i, j)
                        KK = (K * np.conj(K)).real
                        term = 0.5 * (KK / D).sum()
                        ed += term
                        if s != t:
                            ed_os += term
                        for n in range(nt):
                            pd[n] += -0.5 * (KK * np.exp(D * tau[n])).sum()
                        if s == t:
                            KX = K * self.exchange_integrals(s, i, j)
                            ex += -0.5 * (KX / D).sum().real
                            for n in range(nt):
                                px[n] += 0.5 * (KX * np.exp(D * tau[n])).sum().real
        out = dict(e_d=ed, e_x=ex, e_d_os=ed_os)
        if nt:
            out.update(per_tau_d=pd, per_tau_x=px,
                       e_d_lt=float(np.dot(w, pd)), e_x_lt=float(np.dot(w, px)))
        return out

    # --- Green's-function forms (small cells only) --------------------------
    def chi_GG(self, tau):
        """chi_1(G, G') + chi_2(G, G') over the auxiliary set."""
        return self.ch[0].chi_GG(tau) + self.ch[1].chi_GG(tau)

    def direct_trace(self, tau):
        C = self.chi_GG(tau)
        return -0.5 * float((self.v[:, None] * self.v[None, :] * np.abs(C) ** 2).sum())

    def exchange_tau(self, tau):
        return 0.5 * (self.ch[0].exchange_tau(tau) + self.ch[1].exchange_tau(tau))
