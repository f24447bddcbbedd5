"""Writes tests/golden/c3_subset.json: the FP64 oracle's Laplace MP2 energy of
the 40^3 mixed-precision cell restricted to the occupied subset
{156, 157, 158, 159}, at the oracle's own minimax quadrature.  Calls only the
seeded input generator and oracle/ (several minutes of CPU time)."""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from synthetic import C3, make_cell  # noqa: E402
from oracle.mp2 import Problem  # noqa: E402
from oracle.quadrature import minimax_laplace  # noqa: E402

OCC = [156, 157, 158, 159]


def main():
    m, e, c = make_cell(C3)
    P = Problem(C3.L, C3.n, C3.eaux, m, e, c, C3.n_occ, occ=np.array(OCC))
    tau, w, d = minimax_laplace(*P.x_range(), C3.n_tau)
    ref = P.energies(tau, w)
    out = {"cell": "L=20 bohr, 40^3 grid, E_cut=7.5 Ha, E_aux=5 Ha, N_occ=160, seed 0",
           "occ": OCC, "tau": list(map(float, tau)), "w": list(map(float, w)),
           "quad_delta": float(d), "e_d_lt": float(ref["e_d_lt"]),
           "e_x_lt": float(ref["e_x_lt"]),
           "per_tau_d": list(map(float, ref["per_tau_d"])),
           "per_tau_x": list(map(float, ref["per_tau_x"]))}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_subset.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path, out["e_d_lt"], out["e_x_lt"])


if __name__ == "__main__":
    main()
