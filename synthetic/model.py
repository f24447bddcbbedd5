"""Seeded synthetic inputs for the Gamma-only LTMP2 workloads.

This module produces the *inputs* the method assumes are given (the paper's
Implementation section: Hartree-Fock orbitals and energies for all occupied
and virtual states): plane-wave Miller indices, orbital energies and
orbital coefficients.  It contains none of the MP2 arithmetic: no pair
densities, no Coulomb kernel, no Laplace quadrature, no energy.  Both the
CPU oracle and the GPU path consume its output as plain arrays.

Model problem (a stand-in for the paper's LiH / chabazite HF orbitals, which
need VASP and PAW data that are not available):

* cubic cell of side L (bohr), reciprocal spacing b = 2 pi / L, FFT grid n^3;
* orbital basis B = { G = b m : |G|^2 / 2 < E_cut }, each |m_d| < n / 2
  (plane-wave cutoff, Theory section, "Reducing the computational cost");
* one-particle Hamiltonian H_{GG'} = |G|^2/2 delta_{GG'} + V(G - G') with a
  seeded complex Gaussian potential V(G) = 0.3 exp(-|G|^2/4) xi_G drawn over
  the box of difference vectors, Hermitised so that V(r) is real, V(0) = 0;
* FP64 diagonalisation in the time-reversal-invariant (real-orbital) basis,
  so every orbital psi_p(r) is real on the grid: the Gamma-point form the
  paper's time-reversal subsection relies on (phi* = phi at k = 0).

The random draws use numpy's PCG64 (``numpy.random.default_rng(seed)``).
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class CellSpec:
    """Sizes of one synthetic Gamma-only cell."""

    L: float          # cubic cell side, bohr
    n: int            # FFT grid points per axis
    ecut: float       # orbital cutoff, Ha (strict: |G|^2/2 < ecut)
    eaux: float       # auxiliary cutoff, Ha (inclusive: |G|^2/2 <= eaux)
    n_occ: int        # doubly occupied orbitals
    n_tau: int        # Laplace points
    seed: int = 0     # potential seed
    amp: float = 0.3  # potential amplitude


# The workloads: small oracle case, the throughput case, the large
# mixed-precision case.  E_cut of the two larger cells is a reading (the
# workload text only gives approximate plane-wave counts).
C1 = CellSpec(L=8.0, n=12, ecut=6.0, eaux=4.0, n_occ=4, n_tau=8)
C2 = CellSpec(L=16.0, n=32, ecut=7.5, eaux=5.0, n_occ=64, n_tau=8)
C3 = CellSpec(L=20.0, n=40, ecut=7.5, eaux=5.0, n_occ=160, n_tau=10)


def smooth_grid(m: int) -> int:
    """Smallest integer >= m whose only prime factors are 2, 3 and 5."""
    k = max(int(m), 1)
    while True:
        r = k
        for p in (2, 3, 5):
            while r % p == 0:
                r //= p
        if r == 1:
            return k
        k += 1


def batch_specs(count: int = 64, seed: int = 0, L_range=(6.0, 14.0), ecut: float = 7.5,
                eaux: float = 5.0, n_tau_range=(6, 12)) -> list:
    """Many independent cells of uneven size (the batched workload).

    L ~ U[L_range]; grid n = smallest 2,3,5-smooth integer >= ceil(2L)
    (0.5 bohr spacing as in the larger single cells); N_occ = round(8 +
    5 (L - 6)); N_tau ~ U{n_tau_range}; cell k's potential uses seed
    1000 + k.  All draws come from default_rng(seed).
    """
    rng = np.random.default_rng(seed)
    Ls = rng.uniform(L_range[0], L_range[1], size=count)
    nts = rng.integers(n_tau_range[0], n_tau_range[1] + 1, size=count)
    out = []
    for k in range(count):
        L = float(Ls[k])
        out.append(CellSpec(L=L, n=smooth_grid(math.ceil(2.0 * L)), ecut=ecut, eaux=eaux,
                            n_occ=int(round(8 + 5 * (L - 6.0))), n_tau=int(nts[k]),
                            seed=1000 + k))
    return out


def orbital_miller(L: float, n: int, ecut: float) -> np.ndarray:
    """Miller indices of the orbital sphere |b m|^2 / 2 < ecut, sorted.

    Sorted lexicographically, so -m and m are at mirrored positions.  Raises
    if the sphere does not fit inside the centred FFT range |m_d| < n / 2.
    """
    b = 2.0 * math.pi / L
    mmax = int(math.floor(math.sqrt(2.0 * ecut) / b)) + 1
    r = np.arange(-mmax, mmax + 1)
    mx, my, mz = np.meshgrid(r, r, r, indexing="ij")
    m = np.stack([mx.ravel(), my.ravel(), mz.ravel()], axis=1)
    m2 = (m * m).sum(axis=1)
    keep = 0.5 * b * b * m2 < ecut * (1.0 - 1e-12)
    m = m[keep]
    if np.any(2 * np.abs(m) >= n):
        raise ValueError("orbital sphere does not fit inside the FFT grid")
    order = np.lexsort((m[:, 2], m[:, 1], m[:, 0]))
    return np.ascontiguousarray(m[order].astype(np.int32))


def _real_basis(miller: np.ndarray) -> np.ndarray:
    """Unitary U whose columns are time-reversal-invariant plane-wave pairs.

    Column for G = 0 is e_0; for each pair (G, -G) with G "positive" (first
    non-zero component > 0) the columns are (e_G + e_-G)/sqrt2 and
    i (e_G - e_-G)/sqrt2.  Any vector c = U x with x real satisfies
    c(-G) = conj(c(G)), i.e. its real-space function is real.
    """
    npw = miller.shape[0]
    index = {tuple(v): k for k, v in enumerate(miller.tolist())}
    cols = []
    for k, v in enumerate(miller.tolist()):
        t = tuple(v)
        if t == (0, 0, 0):
            e = np.zeros(npw, complex)
            e[k] = 1.0
            cols.append(e)
            continue
        first = next(c for c in t if c != 0)
        if first < 0:
            continue
        kp = index[(-t[0], -t[1], -t[2])]
        e1 = np.zeros(npw, complex)
        e1[k] = 1.0 / math.sqrt(2.0)
        e1[kp] = 1.0 / math.sqrt(2.0)
        e2 = np.zeros(npw, complex)
        e2[k] = 1j / math.sqrt(2.0)
        e2[kp] = -1j / math.sqrt(2.0)
        cols.append(e1)
        cols.append(e2)
    U = np.stack(cols, axis=1)
    assert U.shape == (npw, npw)
    return U


def _real_basis_sparse(miller: np.ndarray):
    """The unitary of _real_basis as a sparse matrix (two entries per column)."""
    import scipy.sparse as sp
    U = _real_basis(miller) if miller.shape[0] <= 64 else None
    if U is not None:
        return sp.csc_matrix(U)
    npw = miller.shape[0]
    index = {tuple(v): k for k, v in enumerate(miller.tolist())}
    rows, cols, vals = [], [], []
    col = 0
    s = 1.0 / math.sqrt(2.0)
    for k, v in enumerate(miller.tolist()):
        t = tuple(v)
        if t == (0, 0, 0):
            rows.append(k); cols.append(col); vals.append(1.0)
            col += 1
            continue
        first = next(c for c in t if c != 0)
        if first < 0:
            continue
        kp = index[(-t[0], -t[1], -t[2])]
        rows += [k, kp, k, kp]
        cols += [col, col, col + 1, col + 1]
        vals += [s, s, 1j * s, -1j * s]
        col += 2
    assert col == npw
    return sp.csc_matrix((np.array(vals, complex), (rows, cols)), shape=(npw, npw))


def potential_box(miller: np.ndarray, L: float, seed: int, amp: float):
    """Seeded Hermitised potential V on the box of difference vectors.

    Returns (V, M) with V indexed as V[m + 2M] for m in [-2M, 2M]^3.
    """
    M = int(np.abs(miller).max())
    K = 4 * M + 1
    rng = np.random.default_rng(seed)
    xi = (rng.standard_normal((K, K, K)) + 1j * rng.standard_normal((K, K, K))) / math.sqrt(2.0)
    b = 2.0 * math.pi / L
    r = np.arange(-2 * M, 2 * M + 1)
    mx, my, mz = np.meshgrid(r, r, r, indexing="ij")
    g2 = b * b * (mx * mx + my * my + mz * mz)
    V = amp * np.exp(-g2 / 4.0) * xi
    V = 0.5 * (V + np.conj(V[::-1, ::-1, ::-1]))   # V(-m) sits at the mirrored index
    V[2 * M, 2 * M, 2 * M] = 0.0
    return V, M


def hamiltonian(miller: np.ndarray, L: float, seed: int, amp: float) -> np.ndarray:
    """H_{GG'} = |G|^2/2 delta + V(G - G') in the orbital basis (complex)."""
    V, M = potential_box(miller, L, seed, amp)
    b = 2.0 * math.pi / L
    npw = miller.shape[0]
    H = np.empty((npw, npw), complex)
    m = miller.astype(np.int64)
    for i0 in range(0, npw, 512):
        d = m[i0:i0 + 512, None, :] - m[None, :, :] + 2 * M
        H[i0:i0 + 512] = V[d[..., 0], d[..., 1], d[..., 2]]
    kin = 0.5 * b * b * (m * m).sum(axis=1)
    H[np.arange(npw), np.arange(npw)] += kin
    return H


def make_cell(spec: CellSpec):
    """Generate (miller, eps, coeff) for one cell.

    miller: int32 [n_pw, 3]; eps: float64 [n_pw] ascending;
    coeff: complex128 [n_pw states, n_pw], row p = c_p(G), unit norm,
    time-reversal invariant (c_p(-G) = conj(c_p(G))).
    """
    miller = orbital_miller(spec.L, spec.n, spec.ecut)
    H = hamiltonian(miller, spec.L, spec.seed, spec.amp)
    eps, coeff = _real_eigh(miller, H)
    return miller, eps, coeff


def make_cell_spin(spec: CellSpec, n_occ_b: int, split: float = 0.1, split_seed: int = 1000):
    """Two spin channels of one cell (a spin-polarised stand-in).

    Channel 1 sees H + dV, channel 2 sees H - dV, with dV a second seeded
    potential of amplitude `split` (seed `split_seed`), the way an exchange
    splitting separates the two channels of an open-shell mean field.
    Channel 1 holds spec.n_occ electrons, channel 2 n_occ_b.  Returns
    (miller, eps_1, coeff_1, eps_2, coeff_2), each channel as make_cell's.
    """
    miller = orbital_miller(spec.L, spec.n, spec.ecut)
    H = hamiltonian(miller, spec.L, spec.seed, spec.amp)
    dV = hamiltonian(miller, spec.L, split_seed, split)
    kin = np.diag(np.diag(dV).copy())
    dV = dV - kin  # potential part only
    e1, c1 = _real_eigh(miller, H + dV)
    e2, c2 = _real_eigh(miller, H - dV)
    assert 1 <= n_occ_b < e2.shape[0]
    return miller, e1, c1, e2, c2


def _real_eigh(miller: np.ndarray, H: np.ndarray):
    """Eigenpairs of a time-reversal-invariant H in the real basis, with
    coefficients in the plane-wave basis (state-major)."""
    U = _real_basis_sparse(miller)
    Hr = np.asarray((U.conj().T @ (U.T @ H.T).T))
    if np.abs(Hr.imag).max() > 1e-10 * max(1.0, np.abs(Hr.real).max()):
        raise RuntimeError("Hamiltonian is not time-reversal invariant")
    Hr = 0.5 * (Hr.real + Hr.real.T)
    eps, R = np.linalg.eigh(Hr)
    # deterministic sign: largest component of each eigenvector positive
    piv = np.argmax(np.abs(R), axis=0)
    sgn = np.sign(R[piv, np.arange(R.shape[1])])
    R = R * sgn[None, :]
    coeff = (U @ R).T.copy()
    return eps.copy(), coeff


def kmesh_points(n_k: int) -> np.ndarray:
    """Integer labels kappa of the Gamma-centred n_k^3 mesh, k = b kappa / n_k,
    in the order kappa_x-major (index (kx n_k + ky) n_k + kz)."""
    r = np.arange(n_k)
    kx, ky, kz = np.meshgrid(r, r, r, indexing="ij")
    return np.stack([kx.ravel(), ky.ravel(), kz.ravel()], axis=1)


def kpoint_miller(L: float, n: int, ecut: float, kappa, n_k: int) -> np.ndarray:
    """Miller indices m of the sphere |b (m + kappa / n_k)|^2 / 2 < ecut
    (plane waves e^{i (G + k).r}), sorted lexicographically."""
    b = 2.0 * math.pi / L
    f = np.asarray(kappa, float) / n_k
    mmax = int(math.floor(math.sqrt(2.0 * ecut) / b)) + 2
    r = np.arange(-mmax, mmax + 1)
    mx, my, mz = np.meshgrid(r, r, r, indexing="ij")
    m = np.stack([mx.ravel(), my.ravel(), mz.ravel()], axis=1)
    q = m + f[None, :]
    keep = 0.5 * b * b * (q * q).sum(axis=1) < ecut * (1.0 - 1e-12)
    m = m[keep]
    if np.any(2 * np.abs(m) >= n):
        raise ValueError("orbital sphere does not fit inside the FFT grid")
    order = np.lexsort((m[:, 2], m[:, 1], m[:, 0]))
    return np.ascontiguousarray(m[order].astype(np.int32))


def make_cell_kmesh(spec: CellSpec, n_k: int, n_bands: int | None = None):
    """Bloch states of one cell on the Gamma-centred n_k^3 mesh.

    The cell and potential are spec's; at each k the Hamiltonian
    H_k = |G + k|^2 / 2 delta + V(G - G') is diagonalised in the sphere of
    kpoint_miller.  Time reversal is exact: for the mesh point k' = -k (mod
    the mesh) the states are the complex conjugates, c_{k'}(m') =
    conj(c_k(-m' - g0)) with k' + k = b g0.  Returns (kappas [N_k, 3],
    millers [N_k] int32 arrays, eps [N_k, n_bands], coeffs [N_k] complex
    arrays [n_bands, n_pw_k]); n_bands defaults to the smallest basis.
    """
    kap = kmesh_points(n_k)
    b = 2.0 * math.pi / spec.L
    mills = [kpoint_miller(spec.L, spec.n, spec.ecut, k, n_k) for k in kap]
    nb = min(m.shape[0] for m in mills) if n_bands is None else int(n_bands)
    allm = np.concatenate(mills)
    V, M = potential_box(allm, spec.L, spec.seed, spec.amp)
    index = {tuple(k): t for t, k in enumerate(kap.tolist())}
    eps = np.zeros((len(kap), nb))
    coeffs = [None] * len(kap)
    for t, k in enumerate(kap):
        kp = tuple(int(x) for x in (-k) % n_k)
        tp = index[kp]
        if tp < t:  # time-reversal partner done: conjugate its states
            g0 = (np.asarray(kp) + k) // n_k
            pos = {tuple(v): c for c, v in enumerate(mills[tp].tolist())}
            src = np.array([pos[tuple(v)] for v in (-mills[t] - g0[None, :]).tolist()])
            eps[t] = eps[tp]
            coeffs[t] = np.conj(coeffs[tp][:, src])
            continue
        m = mills[t].astype(np.int64)
        d = m[:, None, :] - m[None, :, :] + 2 * M
        H = V[d[..., 0], d[..., 1], d[..., 2]].astype(complex)
        q = m + k[None, :] / n_k
        H[np.arange(len(m)), np.arange(len(m))] += 0.5 * b * b * (q * q).sum(axis=1)
        e, U = np.linalg.eigh(H)
        eps[t] = e[:nb]
        coeffs[t] = U[:, :nb].T.copy()
    return kap, mills, eps, coeffs


def make_cell_complex(spec: CellSpec, phase_seed: int | None = None):
    """(miller, eps, coeff) from a plain complex Hermitian eigensolver.

    H is diagonalised as given (no real basis), so each state carries
    whatever phase the eigensolver returns; with phase_seed, every state is
    further multiplied by a seeded random phase e^{i theta_p}.  The orbitals
    are real on the grid only up to these phases.
    """
    miller = orbital_miller(spec.L, spec.n, spec.ecut)
    H = hamiltonian(miller, spec.L, spec.seed, spec.amp)
    eps, V = np.linalg.eigh(H)
    coeff = V.T.copy()
    if phase_seed is not None:
        th = np.random.default_rng(phase_seed).uniform(0.0, 2.0 * math.pi, size=coeff.shape[0])
        coeff *= np.exp(1j * th)[:, None]
    return miller, eps.copy(), coeff


def random_unitary(k: int, seed: int) -> np.ndarray:
    """Haar-like random unitary (QR of a complex Gaussian), seeded."""
    rng = np.random.default_rng(seed)
    z = (rng.standard_normal((k, k)) + 1j * rng.standard_normal((k, k))) / math.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    return q * (d / np.abs(d))[None, :]


def tiny_spec(seed: int = 0, L: float = 4.5, n: int = 6, ecut: float = 2.5,
              eaux: float = 2.0, n_occ: int = 2) -> CellSpec:
    """Tiny cells for brute-force checks (tens of plane waves)."""
    return CellSpec(L=L, n=n, ecut=ecut, eaux=eaux, n_occ=n_occ, n_tau=8, seed=seed)
