"""CPU FP64 oracle for the Gamma-only LTMP2 hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import anything from this package.
The GPU path never imports, links or executes it, and it imports nothing
from the GPU package: the two share only the seeded input generator in
``synthetic``.

Contents (plain, slow, obviously correct; numpy FFT / matmul / eigh are the
only library primitives used as steps):
  planewave   -- grids, auxiliary set, Coulomb kernel, real-space orbitals,
                 overlap (pair) densities                 (Theory section)
  mp2         -- two-electron integrals, canonical MP2, Laplace-transformed
                 MP2 at given (tau_n, w_n), Green's functions, chi(G, G'),
                 transformed states and the Fock-like factorisation
  quadrature  -- relative-error minimax Laplace quadrature (Remez)
  brute       -- real-space brute force for tiny cells (no FFT)
"""
