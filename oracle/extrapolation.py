"""Oracle: internal extrapolation of the auxiliary cutoff.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this.

Implementation section, "Internal cutoff extrapolation": the MP2 energy is
evaluated for nested auxiliary cutoffs

    E_aux[n] = E_aux / alpha^(n - 1),   n = 1 .. n_c   (alpha = 1.05, n_c = 8)

where for each cutoff only auxiliary vectors with |G| <= sqrt(2 E_aux[n])
enter the plane-wave loops (both Coulomb lines), and the energies are fitted
by the straight line y = a + b x with y = E[n], x = E_aux[n]^(-3/2)
(Eq. CutDecay: the error decays like E_aux^(-3/2)); the intercept a is the
extrapolated energy E(E_aux -> infinity).

Here E[n] is, by definition, the oracle's Laplace MP2 energy of the same
orbitals and quadrature with the auxiliary set of E_aux[n]; the fit is the
ordinary least-squares line written out from its normal equations.
"""

from __future__ import annotations

import numpy as np

from .mp2 import Problem


def cutoffs(eaux: float, n_c: int = 8, alpha: float = 1.05) -> np.ndarray:
    """E_aux[n] = E_aux / alpha^(n - 1), n = 1 .. n_c."""
    return np.array([eaux / alpha ** (n - 1) for n in range(1, n_c + 1)])


def energies_at_cutoffs(L, n, eaux, miller, eps, coeff, n_occ, tau, w, n_c=8, alpha=1.05,
                        occ=None):
    """Laplace MP2 (E_d[n], E_x[n]) for every cutoff of the array, each a plain
    oracle evaluation with that auxiliary set."""
    ed, ex = [], []
    for e_n in cutoffs(eaux, n_c, alpha):
        r = Problem(L, n, e_n, miller, eps, coeff, n_occ, occ=occ).energies(tau, w)
        ed.append(r["e_d_lt"])
        ex.append(r["e_x_lt"])
    return np.array(ed), np.array(ex)


def line_fit(x, y):
    """Least-squares (a, b) of y = a + b x (normal equations)."""
    x = np.asarray(x, float)
    y = np.asarray(y, float)
    m = len(x)
    sx, sy = x.sum(), y.sum()
    sxx, sxy = (x * x).sum(), (x * y).sum()
    det = m * sxx - sx * sx
    b = (m * sxy - sx * sy) / det
    a = (sy - b * sx) / m
    return a, b


def extrapolate(e_aux, energies):
    """Intercept and slope of E[n] against E_aux[n]^(-3/2) (Eq. CutDecay)."""
    return line_fit(np.asarray(e_aux, float) ** -1.5, energies)
