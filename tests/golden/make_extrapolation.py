"""Writes tests/golden/c2_extrapolation.json: the FP64 oracle's Laplace MP2
energies of the 32^3 throughput cell restricted to the occupied subset
{62, 63}, at the eight nested auxiliary cutoffs E_aux / 1.05^(n-1) of the
internal cutoff extrapolation, each an independent oracle evaluation with
that auxiliary set, and the oracle's extrapolation in E_aux^(-3/2).

Calls only the seeded input generator and oracle/ (minutes of CPU time).
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from synthetic import C2, make_cell  # noqa: E402
from oracle.mp2 import Problem  # noqa: E402
from oracle.quadrature import minimax_laplace  # noqa: E402
from oracle.extrapolation import cutoffs, energies_at_cutoffs, extrapolate  # noqa: E402

OCC = [62, 63]


def main():
    m, e, c = make_cell(C2)
    occ = np.array(OCC)
    P = Problem(C2.L, C2.n, C2.eaux, m, e, c, C2.n_occ, occ=occ)
    tau, w, d = minimax_laplace(*P.x_range(), C2.n_tau)
    ed, ex = energies_at_cutoffs(C2.L, C2.n, C2.eaux, m, e, c, C2.n_occ, tau, w, occ=occ)
    ea = cutoffs(C2.eaux)
    out = {"cell": "L=16 bohr, 32^3 grid, E_cut=7.5 Ha, E_aux=5 Ha, N_occ=64, seed 0",
           "occ": OCC, "tau": list(map(float, tau)), "w": list(map(float, w)),
           "e_aux": list(map(float, ea)), "e_d": list(map(float, ed)),
           "e_x": list(map(float, ex)),
           "e_inf": [float(extrapolate(ea, ed + ex)[0]), float(extrapolate(ea, ed)[0]),
                     float(extrapolate(ea, ex)[0])]}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_extrapolation.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path, out["e_inf"])


if __name__ == "__main__":
    main()
