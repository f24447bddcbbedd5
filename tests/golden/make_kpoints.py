"""Stored oracle energies of the small workload's cell on a 2 x 2 x 2 k-point
mesh (per unit cell), for the GPU k-point test.

Calls only synthetic/ and oracle/ (oracle.kpoints, the k-point form of
Eqs. 2eIPLWV / MP2direct / MP2ex_spinrestr; about 4 CPU-minutes).
Run from the repository root:  python tests/golden/make_kpoints.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from synthetic import C1, make_cell_kmesh          # noqa: E402
from oracle.kpoints import KProblem                 # noqa: E402
from oracle.quadrature import minimax_laplace       # noqa: E402

N_K, N_OCC = 2, 4


def main():
    kap, mills, eps, coeffs = make_cell_kmesh(C1, N_K)
    K = KProblem(C1.L, C1.n, C1.eaux, N_K, kap, mills, eps, coeffs, N_OCC)
    xmin, xmax = K.x_range()
    tau, w, delta = minimax_laplace(xmin, xmax, C1.n_tau)
    r = K.energies(tau, w)
    out = dict(cell="C1", n_k=N_K, n_occ=N_OCC, n_bands=int(eps.shape[1]), x_min=xmin,
               x_max=xmax, tau=list(map(float, tau)), w=list(map(float, w)),
               e_d=r["e_d"], e_x=r["e_x"], e_d_lt=r["e_d_lt"], e_x_lt=r["e_x_lt"],
               per_tau_d=list(map(float, r["per_tau_d"])),
               per_tau_x=list(map(float, r["per_tau_x"])))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c1_kmesh2.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", path, r["e_d_lt"], r["e_x_lt"])


if __name__ == "__main__":
    main()
