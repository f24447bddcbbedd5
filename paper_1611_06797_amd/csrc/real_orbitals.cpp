// Host-side preparation of the orbital coefficients: bring orbitals that are
// real only up to a phase to real form on the grid.
//
// At the Gamma point of a cell with a real potential, time reversal
// (complex conjugation, the time-reversal subsection of the paper: phi* = phi
// at k = 0) maps every eigenstate to an eigenstate of the same energy.  A
// non-degenerate state is therefore real up to a phase,
//   c_p(G) = e^{i theta} r(G),  r(-G) = conj r(G),
// and the phase follows from z = sum_G c_p(-G) c_p(G) = e^{2 i theta}.  A
// degenerate block is only time-reversal invariant as a whole; its span then
// has an orthonormal basis of real functions, built here from the invariant
// combinations (c + Tc)/2 and (c - Tc)/(2i) of each member (Tc(G) =
// conj c(-G)) by Gram-Schmidt with pivoting: inner products of invariant
// vectors are real, so real combinations keep them invariant.  Rotating
// within a block of equal energies leaves every energy of the method
// unchanged (the Green's functions depend on the block only through its
// projector).
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/ltmp2.h"
#include "ctx.h"

namespace ltmp2 {
namespace {

using cd = std::complex<double>;

constexpr double kPhaseTol = 1e-9;    // | |z| - 1 | for a state real up to a phase
constexpr double kRealTol = 1e-10;    // residual of c(-G) = conj c(G) after the fix
constexpr double kSpanTol = 1e-7;     // residual norm of a vector outside the span

double degeneracy_tol(double e) { return 1e-9 * std::max(1.0, std::fabs(e)); }

}  // namespace

// On success `out` holds the coefficients to use ([n_states][n_pw] complex,
// state-major) and *changed tells whether any state was modified; if no
// state needs a change, `out` is left empty.
ltmp2_status real_orbitals(int npw, const int32_t* miller, int nst, const double* eps, int nocc,
                           const double* coeff, std::vector<double>& out, bool* changed,
                           std::string& err) {
  *changed = false;
  out.clear();
  std::map<std::tuple<int, int, int>, int> pos;
  for (int k = 0; k < npw; ++k)
    pos[std::make_tuple(miller[3 * k], miller[3 * k + 1], miller[3 * k + 2])] = k;
  std::vector<int> neg(npw);
  for (int k = 0; k < npw; ++k) {
    auto it = pos.find(std::make_tuple(-miller[3 * k], -miller[3 * k + 1], -miller[3 * k + 2]));
    if (it == pos.end()) {
      err = "basis not closed under G -> -G";
      return LTMP2_EINVAL;
    }
    neg[k] = it->second;
  }
  auto cof = [&](int s, int k) {
    const double* c = coeff + 2 * (size_t(s) * npw + k);
    return cd(c[0], c[1]);
  };
  auto asym = [&](const cd* v) {
    double a = 0.0;
    for (int k = 0; k < npw; ++k) a = std::max(a, std::abs(v[neg[k]] - std::conj(v[k])));
    return a;
  };
  // per state: phase z, or flagged for the block treatment
  std::vector<cd> fix(nst, cd(1.0, 0.0));
  std::vector<char> bad(nst, 0);
  bool any = false;
  std::vector<cd> tmp(npw);
  for (int s = 0; s < nst; ++s) {
    for (int k = 0; k < npw; ++k) tmp[k] = cof(s, k);
    if (asym(tmp.data()) <= kRealTol) continue;  // already real: no change
    cd z(0.0, 0.0);
    for (int k = 0; k < npw; ++k) z += cof(s, neg[k]) * cof(s, k);
    const double az = std::abs(z);
    if (std::fabs(az - 1.0) <= kPhaseTol) {
      const cd half = std::sqrt(z / az);  // e^{i theta}, principal branch
      for (int k = 0; k < npw; ++k) tmp[k] = cof(s, k) * std::conj(half);
      if (asym(tmp.data()) <= kRealTol) {
        fix[s] = std::conj(half);
        any = true;
        continue;
      }
    }
    bad[s] = 1;
    any = true;
  }
  if (!any) return LTMP2_OK;
  out.assign(2 * size_t(nst) * npw, 0.0);
  for (int s = 0; s < nst; ++s) {
    if (bad[s]) continue;
    for (int k = 0; k < npw; ++k) {
      const cd v = cof(s, k) * fix[s];
      // enforce c(-G) = conj c(G) exactly: average the state with its image
      const cd vn = cof(s, neg[k]) * fix[s];
      const cd sym = 0.5 * (v + std::conj(vn));
      out[2 * (size_t(s) * npw + k)] = sym.real();
      out[2 * (size_t(s) * npw + k) + 1] = sym.imag();
    }
  }
  // degenerate blocks
  for (int s = 0; s < nst; ++s) {
    if (bad[s] != 1) continue;
    int b0 = s, b1 = s + 1;
    while (b0 > 0 && eps[b0] - eps[b0 - 1] <= degeneracy_tol(eps[b0])) --b0;
    while (b1 < nst && eps[b1] - eps[b1 - 1] <= degeneracy_tol(eps[b1])) ++b1;
    const int kb = b1 - b0;
    if (kb == 1) {
      err = "orbital " + std::to_string(s) +
            " is not real on the grid up to a phase (c(-G) != e^{2i theta} conj c(G)) and has "
            "no degenerate partner";
      return LTMP2_EINVAL;
    }
    if (b0 < nocc && b1 > nocc) {
      err = "degenerate block " + std::to_string(b0) + ".." + std::to_string(b1 - 1) +
            " spans the occupied and virtual spaces";
      return LTMP2_EGAP;
    }
    // 2 kb invariant candidates
    std::vector<std::vector<cd>> cand;
    for (int p = b0; p < b1; ++p) {
      std::vector<cd> u(npw), v(npw);
      for (int k = 0; k < npw; ++k) {
        const cd c = cof(p, k), tc = std::conj(cof(p, neg[k]));
        u[k] = 0.5 * (c + tc);
        v[k] = (c - tc) / cd(0.0, 2.0);
      }
      cand.push_back(std::move(u));
      cand.push_back(std::move(v));
    }
    auto dot = [&](const std::vector<cd>& a, const std::vector<cd>& b) {
      double r = 0.0;  // real for invariant vectors
      for (int k = 0; k < npw; ++k) r += (std::conj(a[k]) * b[k]).real();
      return r;
    };
    std::vector<std::vector<cd>> basis;
    std::vector<char> used(cand.size(), 0);
    for (int it = 0; it < kb; ++it) {
      int best = -1;
      double bn = 0.0;
      for (size_t q = 0; q < cand.size(); ++q) {
        if (used[q]) continue;
        const double nq = std::sqrt(dot(cand[q], cand[q]));
        if (nq > bn) {
          bn = nq;
          best = int(q);
        }
      }
      if (best < 0 || bn < 1e-3) {
        err = "degenerate block " + std::to_string(b0) + ".." + std::to_string(b1 - 1) +
              " has no real basis (not time-reversal invariant)";
        return LTMP2_EINVAL;
      }
      used[best] = 1;
      std::vector<cd> e = cand[best];
      for (auto& x : e) x /= bn;
      for (size_t q = 0; q < cand.size(); ++q) {
        if (used[q]) continue;
        const double d = dot(e, cand[q]);
        for (int k = 0; k < npw; ++k) cand[q][k] -= d * e[k];
      }
      basis.push_back(std::move(e));
    }
    for (size_t q = 0; q < cand.size(); ++q)
      if (!used[q] && std::sqrt(dot(cand[q], cand[q])) > kSpanTol) {
        err = "degenerate block " + std::to_string(b0) + ".." + std::to_string(b1 - 1) +
              " is not time-reversal invariant";
        return LTMP2_EINVAL;
      }
    for (int p = b0; p < b1; ++p) {
      const std::vector<cd>& e = basis[p - b0];
      if (asym(e.data()) > 1e-8) {
        err = "degenerate block " + std::to_string(b0) + ".." + std::to_string(b1 - 1) +
              ": real basis failed";
        return LTMP2_ENUMERIC;
      }
      for (int k = 0; k < npw; ++k) {
        const cd sym = 0.5 * (e[k] + std::conj(e[neg[k]]));
        out[2 * (size_t(p) * npw + k)] = sym.real();
        out[2 * (size_t(p) * npw + k) + 1] = sym.imag();
      }
      bad[p] = 2;
    }
  }
  *changed = true;
  return LTMP2_OK;
}

}  // namespace ltmp2

extern "C" ltmp2_status ltmp2_real_orbitals(int n_pw, const int32_t* miller, int n_states,
                                            const double* eps, int n_occ, const double* coeff_in,
                                            double* coeff_out) {
  if (n_pw < 1 || n_states < 1 || n_occ < 0 || n_occ > n_states || !miller || !eps ||
      !coeff_in || !coeff_out)
    return LTMP2_EINVAL;
  std::vector<double> out;
  bool changed = false;
  std::string err;
  const ltmp2_status s =
      ltmp2::real_orbitals(n_pw, miller, n_states, eps, n_occ, coeff_in, out, &changed, err);
  if (s) {
    ltmp2::set_setup_error(err);
    return s;
  }
  const double* src = changed ? out.data() : coeff_in;
  if (src != coeff_out) std::memmove(coeff_out, src, sizeof(double) * 2 * size_t(n_states) * n_pw);
  return LTMP2_OK;
}
