"""Writes tests/golden/{c2,c3}_subset16.json: the FP64 oracle's Laplace MP2
energy of the 32^3 throughput cell and of the 40^3 mixed-precision cell,
each restricted to a seeded, non-contiguous subset I of 16 occupied
orbitals (two 8 x 8 blocks of occupied pairs on the library side), at the
oracle's own minimax quadrature for the subset's denominator range.

Calls only the seeded input generator and oracle/.  CPU time: about 40
minutes for the 32^3 cell, several hours for the 40^3 cell (run with the
cell name as argument to write one file).
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from synthetic import C2, C3, make_cell  # noqa: E402
from oracle.mp2 import Problem  # noqa: E402
from oracle.quadrature import minimax_laplace  # noqa: E402

CELLS = {"c2": (C2, "L=16 bohr, 32^3 grid, E_cut=7.5 Ha, E_aux=5 Ha, N_occ=64, seed 0"),
         "c3": (C3, "L=20 bohr, 40^3 grid, E_cut=7.5 Ha, E_aux=5 Ha, N_occ=160, seed 0")}
SUBSET_SIZE = 16
SUBSET_SEED = 16


def subset(n_occ):
    """Seeded sorted choice of 16 occupied orbitals (the HOMO always in)."""
    rng = np.random.default_rng(SUBSET_SEED)
    pick = rng.choice(n_occ - 1, size=SUBSET_SIZE - 1, replace=False)
    return sorted(int(k) for k in pick) + [n_occ - 1]


def write(name):
    spec, text = CELLS[name]
    t0 = time.time()
    m, e, c = make_cell(spec)
    occ = subset(spec.n_occ)
    P = Problem(spec.L, spec.n, spec.eaux, m, e, c, spec.n_occ, occ=np.array(occ))
    tau, w, d = minimax_laplace(*P.x_range(), spec.n_tau)
    ref = P.energies(tau, w)
    out = {"cell": text, "occ": occ, "tau": list(map(float, tau)), "w": list(map(float, w)),
           "quad_delta": float(d), "e_d_lt": float(ref["e_d_lt"]),
           "e_x_lt": float(ref["e_x_lt"]), "e_d": float(ref["e_d"]), "e_x": float(ref["e_x"]),
           "per_tau_d": list(map(float, ref["per_tau_d"])),
           "per_tau_x": list(map(float, ref["per_tau_x"])),
           "oracle_seconds": time.time() - t0}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_subset16.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path, out["e_d_lt"], out["e_x_lt"], f"{out['oracle_seconds']:.0f}s", flush=True)


if __name__ == "__main__":
    for name in (sys.argv[1:] or ["c2", "c3"]):
        write(name)
