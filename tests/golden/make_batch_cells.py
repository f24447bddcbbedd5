"""Writes tests/golden/batch_cells.json: the FP64 oracle's Laplace MP2 energy
of whole cells of the 64-cell batched workload (synthetic.batch_specs()), one
or two cells per internal transform grid the batch uses (12, 15, 18, 20 and
24; the 24 grid is the one whose pair launches run 192-thread workgroups),
each at the oracle's own minimax quadrature for the cell's denominator range.

Calls only the seeded input generator and oracle/ (about a quarter of an
hour of CPU time).
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from synthetic import batch_specs, make_cell  # noqa: E402
from oracle.mp2 import Problem  # noqa: E402
from oracle.quadrature import minimax_laplace  # noqa: E402

# batch index -> internal transform grid of that cell (smallest cells per grid)
CELLS = {11: 12, 1: 15, 36: 18, 34: 18, 22: 20, 50: 24}


def main():
    specs = batch_specs()
    out = {"workload": "batch_specs(): 64 cells, L ~ U[6,14], E_cut 7.5 Ha, E_aux 5 Ha, "
                       "batch seed 0", "cells": []}
    for k, grid in CELLS.items():
        s = specs[k]
        t0 = time.time()
        m, e, c = make_cell(s)
        P = Problem(s.L, s.n, s.eaux, m, e, c, s.n_occ)
        tau, w, d = minimax_laplace(*P.x_range(), s.n_tau)
        ref = P.energies(tau, w)
        out["cells"].append({"index": k, "internal_grid": grid, "n": s.n, "L": s.L,
                             "n_occ": s.n_occ, "n_tau": s.n_tau, "n_pw": int(len(e)),
                             "tau": list(map(float, tau)), "w": list(map(float, w)),
                             "e_d_lt": float(ref["e_d_lt"]), "e_x_lt": float(ref["e_x_lt"]),
                             "oracle_seconds": time.time() - t0})
        print("cell", k, grid, ref["e_d_lt"], ref["e_x_lt"], f"{time.time() - t0:.0f}s",
              flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch_cells.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
