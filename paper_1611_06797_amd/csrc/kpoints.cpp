// Host-side unfolding of a k-point mesh onto its Born-von Karman supercell.
//
// With N = n_k^3 unit cells and Born-von Karman boundaries (Theory section,
// "LTMP2 in the plane wave basis"), the crystal wavevectors form the mesh
// k = b kappa / n_k (b = 2 pi / L, kappa in {0..n_k-1}^3), and a Bloch state
//   phi_{pk}(r) = Omega^(-1/2) sum_m c_{pk}(m) e^{i (b m + k).r},  Omega = N L^3,
// is, letter for letter, a plane-wave orbital of the cubic supercell of side
// n_k L, whose reciprocal spacing is b / n_k: its plane waves are the supercell
// Miller indices M = n_k m + kappa, with the same coefficients and the same
// normalisation.  Every two-electron integral of the mesh (Eq. 2eIPLWV) is
// the supercell integral of these orbitals: the supercell's Coulomb
// wavevectors b M / n_k are exactly the G + q of the mesh, the supercell's
// auxiliary sphere is the mesh's cutoff on |G + q|, and the supercell sum over
// M != 0 is the mesh sum over (q, G) without the q = G = 0 term.  Momentum
// conservation is the supercell's orthogonality of plane waves.  So the MP2
// energy per unit cell of the mesh (Eqs. MP2direct, MP2ex_spinrestr) is the
// supercell's Gamma-point energy divided by N, and the Gamma-point path
// computes it unchanged.
//
// Time reversal (phi*_{pk} = phi_{p,-k}, the time-reversal subsection) makes
// the supercell orbitals real up to rotations within each pair of partners
// k, -k of equal energy; the real-orbital preparation then finds the real
// basis of each such pair.
#include <algorithm>
#include <cstdint>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/ltmp2.h"

namespace ltmp2 {

ltmp2_status unfold_kmesh(int n_k, int n_bands, int n_occ, const int32_t* n_pw_k,
                          const int32_t* miller, const double* eps, const double* coeff,
                          std::vector<int32_t>& miller_s, std::vector<double>& eps_s,
                          std::vector<double>& coeff_s, std::string& err) {
  if (n_k < 1 || n_k > 6) {
    err = "n_k must be in [1, 6]";
    return LTMP2_EINVAL;
  }
  const int nk = n_k * n_k * n_k;
  if (n_bands < 2 || n_occ < 1 || n_occ >= n_bands) {
    err = "need 1 <= n_occ < n_states (bands per k-point)";
    return LTMP2_EINVAL;
  }
  std::vector<long> off(nk + 1, 0);
  for (int t = 0; t < nk; ++t) {
    if (n_pw_k[t] < n_bands) {
      err = "k-point " + std::to_string(t) + ": fewer plane waves than bands";
      return LTMP2_EINVAL;
    }
    off[t + 1] = off[t] + n_pw_k[t];
  }
  const long npw = off[nk];
  const long nst = long(nk) * n_bands;
  if (npw > (1L << 16) || double(nst) * double(npw) > double(1L << 30)) {
    err = "supercell too large for the unfolded coefficient table";
    return LTMP2_EINVAL;
  }
  // bands ascending per k, and a gap common to the mesh: the lowest
  // N * n_occ supercell states must be the occupied bands of every k
  double occ_max = -1e300, vir_min = 1e300;
  for (int t = 0; t < nk; ++t) {
    const double* e = eps + long(t) * n_bands;
    for (int p = 0; p + 1 < n_bands; ++p)
      if (!(e[p] <= e[p + 1])) {
        err = "k-point " + std::to_string(t) + ": energies not ascending";
        return LTMP2_EINVAL;
      }
    occ_max = std::max(occ_max, e[n_occ - 1]);
    vir_min = std::min(vir_min, e[n_occ]);
  }
  if (!(vir_min - occ_max > 1e-8)) {
    err = "occupied and virtual bands of the mesh overlap (no gap)";
    return LTMP2_EGAP;
  }
  // supercell plane waves M = n_k m + kappa, kappa of mesh index
  // t = (kappa_x n_k + kappa_y) n_k + kappa_z
  miller_s.resize(3 * size_t(npw));
  for (int t = 0; t < nk; ++t) {
    const int kap[3] = {t / (n_k * n_k), (t / n_k) % n_k, t % n_k};
    for (long g = off[t]; g < off[t + 1]; ++g)
      for (int d = 0; d < 3; ++d) {
        const long M = long(n_k) * miller[3 * g + d] + kap[d];
        if (M < -32768 || M > 32767) {
          err = "Miller index out of range";
          return LTMP2_EINVAL;
        }
        miller_s[3 * g + d] = int32_t(M);
      }
  }
  // states in ascending energy (stable: k index, then band)
  std::vector<long> order(nst);
  std::iota(order.begin(), order.end(), 0L);
  std::stable_sort(order.begin(), order.end(), [&](long a, long c) { return eps[a] < eps[c]; });
  eps_s.resize(nst);
  coeff_s.assign(2 * size_t(nst) * npw, 0.0);
  long coff = 0;
  std::vector<long> cstart(nk);
  for (int t = 0; t < nk; ++t) {
    cstart[t] = coff;
    coff += 2L * n_bands * n_pw_k[t];
  }
  for (long s = 0; s < nst; ++s) {
    const long src = order[s];
    const int t = int(src / n_bands), p = int(src % n_bands);
    eps_s[s] = eps[src];
    const double* c = coeff + cstart[t] + 2L * p * n_pw_k[t];
    std::copy(c, c + 2L * n_pw_k[t], coeff_s.begin() + 2 * (s * npw + off[t]));
  }
  return LTMP2_OK;
}

}  // namespace ltmp2
