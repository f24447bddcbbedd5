"""Oracle: spin-restricted MP2 with k-point sampling of the Brillouin zone.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this.

Theory section, "MP2 for periodic systems" and "LTMP2 in the plane wave
basis": N unit cells of volume Omega_0 with Born-von Karman boundaries give
the Gamma-centred mesh k = b kappa / n_k (kappa in {0..n_k-1}^3, N = n_k^3).
Bloch states phi_{pk}(r) = Omega^(-1/2) e^{ik.r} u_{pk}(r) (Eq. BlochOrbital)
with u_{pk}(r) = sum_m c_{pk}(m) e^{i b m.r}, so that int_{Omega_0} |u|^2 =
Omega_0 and <pk|p'k'> = delta (Eq. BlochNorm), Omega = N Omega_0.

Two-electron integrals (Eq. 2eIPLWV), nonzero only when T(k1 - k3) =
T(k4 - k2) =: q (crystal momentum conservation):

  <ik1, jk2|ak3, bk4> = (1/Omega) sum_G 4 pi / |G + q|^2
                        <ik1| e^{+i(G + q).r} |ak3>_0  <jk2| e^{-i(G + q).r} |bk4>_0

with the overlap densities of Eq. OverlapDens,
<pk| e^{-iK.r} |p'k'>_0 = N int_{Omega_0} phi*_{pk} phi_{p'k'} e^{-iK.r}
= (1/Omega_0) int_{Omega_0} u*_{pk} u_{p'k'} e^{i(k' - k - K).r}, evaluated on
the unit-cell grid as a plain average over its points.  T(k) is taken as the
mesh label mod n_k; any representative gives the same integral because G runs
over the whole lattice.  The G sum runs over the auxiliary set of q,
{G : |G + q|^2 / 2 <= E_aux, G + q != 0} (the cutoff acts on the Coulomb
wavevector G + q).

Energies per unit cell with spin sums done (Eq. MP2direct with
sum_{ss'} -> 4 and the prefactor 1/2; Eq. MP2ex_spinrestr), k4 fixed by
momentum conservation, D = e_ik1 + e_jk2 - e_ak3 - e_bk4 < 0:

  E_d =  (2/N) sum_{k1 k2 k3} sum_{ijab} |<ik1, jk2|ak3, bk4>|^2 / D
  E_x = -(1/N) sum_{k1 k2 k3} sum_{ijab} <ik1, jk2|ak3, bk4> <ak3, bk4|jk2, ik1> / D

and their Laplace forms (Eq. LTMP2): 1/D -> -sum_n w_n exp(D tau_n).
"""

from __future__ import annotations

import math

import numpy as np


class KProblem:
    """One cell on an n_k^3 mesh: Bloch states per k, n_occ occupied bands."""

    def __init__(self, L, n, eaux, n_k, kappas, millers, eps, coeffs, n_occ):
        self.L, self.n, self.eaux, self.n_k = float(L), int(n), float(eaux), int(n_k)
        self.b = 2.0 * math.pi / self.L
        self.omega0 = self.L ** 3
        self.N = self.n_k ** 3
        self.kap = np.asarray(kappas, np.int64)
        self.index = {tuple(k): t for t, k in enumerate(self.kap.tolist())}
        assert len(self.index) == self.N
        self.eps = np.asarray(eps, float)
        self.n_occ = int(n_occ)
        nb = self.eps.shape[1]
        self.u = np.empty((self.N, nb, n, n, n), complex)
        for t in range(self.N):
            self.u[t] = self._periodic_parts(np.asarray(millers[t], np.int64),
                                             np.asarray(coeffs[t], complex))
        self._rho = {}
        self._aux = {}

    # --- states and grids ----------------------------------------------------
    def _periodic_parts(self, miller, coeff):
        """u_p(r) = sum_m c_p(m) e^{i b m.r} on the unit-cell grid."""
        n = self.n
        m = np.mod(miller, n)
        out = np.empty((coeff.shape[0], n, n, n), complex)
        A = np.zeros((n, n, n), complex)
        for p in range(coeff.shape[0]):
            A[:] = 0.0
            A[m[:, 0], m[:, 1], m[:, 2]] = coeff[p]
            out[p] = np.fft.ifftn(A) * self.n ** 3
        return out

    def k_index(self, kappa):
        return self.index[tuple(int(x) % self.n_k for x in kappa)]

    def q_label(self, t1, t2):
        """Mesh label of T(k_t1 - k_t2)."""
        return np.mod(self.kap[t1] - self.kap[t2], self.n_k)

    def aux(self, ql):
        """(G Miller indices, 4 pi / |G + q|^2) of the auxiliary set of q."""
        key = tuple(int(x) for x in ql)
        if key not in self._aux:
            f = np.asarray(ql, float) / self.n_k
            mm = int(math.sqrt(2.0 * self.eaux) / self.b) + 2
            r = np.arange(-mm, mm + 1)
            mx, my, mz = np.meshgrid(r, r, r, indexing="ij")
            m = np.stack([mx.ravel(), my.ravel(), mz.ravel()], axis=1)
            g = self.b * (m + f[None, :])
            g2 = (g * g).sum(1)
            lim = 2.0 * self.eaux
            keep = (g2 <= lim * (1 + 1e-12)) & (g2 > 1e-12 * lim)
            m, g2 = m[keep], g2[keep]
            self._aux[key] = (m, 4.0 * math.pi / g2)
        return self._aux[key]

    def rho(self, ta, tb, sa, sb):
        """<p ka| e^{+i(G + q).r} |p' kb>_0 for p in band slice sa, p' in sb,
        q = T(ka - kb), over the auxiliary set of q:
        (1/Omega_0) int u*_{p ka} u_{p' kb} e^{i(G + q - ka + kb).r}."""
        key = (ta, tb, sa.start, sa.stop, sb.start, sb.stop)
        if key not in self._rho:
            ql = self.q_label(ta, tb)
            g0 = (ql - self.kap[ta] + self.kap[tb]) // self.n_k   # lattice vector
            m, _ = self.aux(ql)
            K = np.mod(m + g0[None, :], self.n)
            ua, ub = self.u[ta][sa], self.u[tb][sb]
            out = np.empty((ua.shape[0], ub.shape[0], m.shape[0]), complex)
            for p in range(ua.shape[0]):
                cp = np.conj(ua[p])
                for p2 in range(ub.shape[0]):
                    F = np.fft.ifftn(cp * ub[p2])      # (1/N_r) sum_r f(r) e^{+iK.r}
                    out[p, p2] = F[K[:, 0], K[:, 1], K[:, 2]]
            self._rho[key] = out
        return self._rho[key]

    # --- integrals and energies ---------------------------------------------
    def integrals(self, t1, t2, t3, t4, s1, s2, s3, s4):
        """<p1 k1, p2 k2|p3 k3, p4 k4> [p1, p2, p3, p4] over band slices."""
        ql = self.q_label(t1, t3)
        assert np.array_equal(ql, self.q_label(t4, t2))
        _, v = self.aux(ql)
        A = self.rho(t1, t3, s1, s3)               # <p1 k1| e^{+i(G+q)r} |p3 k3>
        B = np.conj(self.rho(t4, t2, s4, s2))      # <p2 k2| e^{-i(G+q)r} |p4 k4>
        T = np.tensordot(A * v[None, None, :], B, axes=([2], [2]))    # [p1, p3, p4, p2]
        return np.transpose(T, (0, 3, 1, 2)) / (self.N * self.omega0)

    def x_range(self):
        eo = self.eps[:, :self.n_occ]
        ev = self.eps[:, self.n_occ:]
        return 2.0 * (ev.min() - eo.max()), 2.0 * (ev.max() - eo.min())

    def energies(self, tau=None, w=None):
        """Canonical E_d, E_x per unit cell and, with (tau, w), the Laplace
        forms (e_d_lt, e_x_lt, per_tau_d, per_tau_x unweighted)."""
        no = self.n_occ
        so, sv = slice(0, no), slice(no, self.eps.shape[1])
        nt = 0 if tau is None else len(tau)
        ed = ex = 0.0
        pd = np.zeros(nt)
        px = np.zeros(nt)
        for t1 in range(self.N):
            for t2 in range(self.N):
                for t3 in range(self.N):
                    t4 = self.k_index(self.kap[t1] + self.kap[t2] - self.kap[t3])
                    K = self.integrals(t1, t2, t3, t4, so, so, sv, sv)    # [i, j, a, b]
                    X = self.integrals(t3, t4, t2, t1, sv, sv, so, so)    # [a, b, j, i]
                    X = np.transpose(X, (3, 2, 0, 1))                      # [i, j, a, b]
                    eo1, eo2 = self.eps[t1, so], self.eps[t2, so]
                    ev3, ev4 = self.eps[t3, sv], self.eps[t4, sv]
                    D = (eo1[:, None, None, None] + eo2[None, :, None, None]
                         - ev3[None, None, :, None] - ev4[None, None, None, :])
                    KK = (K * np.conj(K)).real
                    KX = (K * X)
                    ed += 2.0 * (KK / D).sum() / self.N
                    ex += -(KX / D).sum().real / self.N
                    for k in range(nt):
                        f = np.exp(D * tau[k])
                        pd[k] += -2.0 * (KK * f).sum() / self.N
                        px[k] += (KX * f).sum().real / self.N
        out = dict(e_d=ed, e_x=ex)
        if nt:
            out.update(per_tau_d=pd, per_tau_x=px,
                       e_d_lt=float(np.dot(w, pd)), e_x_lt=float(np.dot(w, px)))
        return out
