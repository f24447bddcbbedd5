"""Seeded synthetic inputs (plane-wave basis, orbital energies, orbital
coefficients) shared by the CPU oracle and the GPU path.  No MP2 arithmetic
lives here."""
from .model import (CellSpec, C1, C2, C3, orbital_miller, make_cell, make_cell_spin,
                    make_cell_complex, make_cell_kmesh, kmesh_points, kpoint_miller,
                    random_unitary, tiny_spec, hamiltonian, batch_specs, smooth_grid)

__all__ = ["CellSpec", "C1", "C2", "C3", "orbital_miller", "make_cell", "make_cell_spin",
           "make_cell_complex", "make_cell_kmesh", "kmesh_points", "kpoint_miller",
           "random_unitary", "tiny_spec", "hamiltonian", "batch_specs", "smooth_grid"]
