// Relative-error minimax Laplace quadrature, host FP64.
//
// The energy denominator is replaced by 1/x = int_0^inf exp(-x tau) dtau
// (Eq. SCHLT) evaluated with a few tau points (LTMP2 subsection; the paper
// cites Haser 1992 and Kaltak 2014 for the quadrature).  The fit minimises
// max_x |x sum_n w_n exp(-x tau_n) - 1| on [x_min, x_max] by the Remez
// exchange for exponential sums (Takatsuka, Ten-no, Hackbusch, J. Chem.
// Phys. 129, 044112 (2008)):
//   * unit interval y = x / x_min in [1, R]; alpha_n = e^{p_n}, beta_n = e^{q_n};
//   * start at R_s(N) = max(10, exp(1.25 (N - 1) - 2)) from a uniform layout
//     of s = -log alpha on [-1, log R_s + 1] with trapezoid weights, refined by
//     damped Gauss-Newton (Levenberg-Marquardt) and Lawson reweighting;
//   * exchange: alternating extrema (grid bracketing + Newton on de/dt = 0),
//     Newton solve of e(y_k) = (-1)^k E, repeat until the levels agree;
//   * continuation in R with adaptive log-steps, reference stretched in log y;
//   * N >= 9: the fit is made on [1, max(R, R_floor(N))], R_floor =
//     exp(0.5 (N - 10) + 3.8), where the minimax error reaches ~1e-8 and the
//     Newton system stops being solvable in double precision.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "quadrature.h"
#include "reference_table.h"

namespace ltmp2 {
namespace {

using Vec = std::vector<double>;

// e(y) = y sum_n beta_n exp(-alpha_n y) - 1
double err1(double y, const Vec& p, const Vec& q) {
  double s = 0.0;
  for (size_t n = 0; n < p.size(); ++n) s += std::exp(q[n] - std::exp(p[n]) * y);
  return y * s - 1.0;
}

// de/dt and d2e/dt2 at t = log y
void derivs_t(double t, const Vec& p, const Vec& q, double& d1, double& d2) {
  const double y = std::exp(t);
  double s0 = 0, s1 = 0, s2 = 0;
  for (size_t n = 0; n < p.size(); ++n) {
    const double a = std::exp(p[n]);
    const double E = std::exp(q[n] - a * y);
    s0 += E;
    s1 -= a * E;
    s2 += a * a * E;
  }
  const double g1 = s0 + y * s1, g2 = 2.0 * s1 + y * s2;
  d1 = y * g1;
  d2 = y * g1 + y * y * g2;
}

// Row of the Jacobian of e(y) w.r.t. (p, q).
void jac_row(double y, const Vec& p, const Vec& q, double* row) {
  const size_t N = p.size();
  for (size_t n = 0; n < N; ++n) {
    const double a = std::exp(p[n]);
    const double E = std::exp(q[n] - a * y);
    row[n] = -y * y * a * E;
    row[N + n] = y * E;
  }
}

// Solve A x = b (n x n, row-major) by Gaussian elimination with partial
// pivoting.  Returns false if singular.
bool lu_solve(std::vector<double> A, std::vector<double> b, int n, std::vector<double>& x) {
  for (int c = 0; c < n; ++c) {
    int piv = c;
    double best = std::fabs(A[c * n + c]);
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > best) {
        best = std::fabs(A[r * n + c]);
        piv = r;
      }
    if (!(best > 0.0) || !std::isfinite(best)) return false;
    if (piv != c) {
      for (int k = 0; k < n; ++k) std::swap(A[c * n + k], A[piv * n + k]);
      std::swap(b[c], b[piv]);
    }
    for (int r = c + 1; r < n; ++r) {
      const double f = A[r * n + c] / A[c * n + c];
      if (f == 0.0) continue;
      for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
      b[r] -= f * b[c];
    }
  }
  x.assign(n, 0.0);
  for (int r = n - 1; r >= 0; --r) {
    double s = b[r];
    for (int k = r + 1; k < n; ++k) s -= A[r * n + k] * x[k];
    x[r] = s / A[r * n + r];
  }
  for (double v : x)
    if (!std::isfinite(v)) return false;
  return true;
}

struct Ref {
  Vec y, e;
  double emax = 0.0;
};

thread_local int g_ngrid = 20000;  // bracketing grid of the extremum search

// Alternating extrema of e on [1, R].
Ref alternation(int N, double R, const Vec& p, const Vec& q) {
  const int ngrid = g_ngrid;
  const double T = std::log(R);
  const double h = T / (ngrid - 1);
  Vec e(ngrid);
  double emax = 0.0;
  for (int k = 0; k < ngrid; ++k) {
    e[k] = err1(std::exp(k * h), p, q);
    emax = std::max(emax, std::fabs(e[k]));
  }
  Vec ts{0.0};
  for (int k = 1; k < ngrid - 1; ++k) {
    const double a = e[k] - e[k - 1], b = e[k + 1] - e[k];
    if (a * b < 0.0) {
      double t = k * h;
      for (int it = 0; it < 30; ++it) {
        double d1, d2;
        derivs_t(t, p, q, d1, d2);
        if (d2 == 0.0) break;
        const double st = std::clamp(-d1 / d2, -h, h);
        t += st;
        if (std::fabs(st) < 1e-15 * std::max(1.0, T)) break;
      }
      ts.push_back(std::clamp(t, 0.0, T));
    }
  }
  ts.push_back(T);
  Ref out;
  for (double t : ts) {
    const double y = std::exp(t), v = err1(y, p, q);
    if (!out.y.empty() && ((v > 0) == (out.e.back() > 0))) {
      if (std::fabs(v) > std::fabs(out.e.back())) {
        out.y.back() = y;
        out.e.back() = v;
      }
    } else {
      out.y.push_back(y);
      out.e.push_back(v);
    }
  }
  while ((int)out.y.size() > 2 * N + 1) {
    if (std::fabs(out.e.front()) < std::fabs(out.e.back())) {
      out.y.erase(out.y.begin());
      out.e.erase(out.e.begin());
    } else {
      out.y.pop_back();
      out.e.pop_back();
    }
  }
  out.emax = emax;
  return out;
}

// Damped Newton on e(y_k) - (-1)^k E = 0 for (p, q, E).
bool newton_reference(int N, const Vec& ys, Vec& p, Vec& q, double E) {
  const int m = 2 * N + 1;
  auto resid = [&](const Vec& pp, const Vec& qq, double EE, Vec& F) {
    F.resize(m);
    for (int k = 0; k < m; ++k) F[k] = err1(ys[k], pp, qq) - ((k & 1) ? -EE : EE);
  };
  Vec F;
  resid(p, q, E, F);
  for (int it = 0; it < 40; ++it) {
    std::vector<double> J(m * m), row(2 * N);
    for (int k = 0; k < m; ++k) {
      jac_row(ys[k], p, q, row.data());
      for (int c = 0; c < 2 * N; ++c) J[k * m + c] = row[c];
      J[k * m + 2 * N] = (k & 1) ? 1.0 : -1.0;
    }
    Vec rhs(m), step;
    for (int k = 0; k < m; ++k) rhs[k] = -F[k];
    if (!lu_solve(J, rhs, m, step)) return false;
    double f0 = 0.0;
    for (double v : F) f0 = std::max(f0, std::fabs(v));
    double lam = 1.0;
    Vec pn(N), qn(N), Fn;
    double En;
    while (true) {
      for (int n = 0; n < N; ++n) {
        pn[n] = p[n] + lam * step[n];
        qn[n] = q[n] + lam * step[N + n];
      }
      En = E + lam * step[2 * N];
      resid(pn, qn, En, Fn);
      double f1 = 0.0;
      bool finite = true;
      for (double v : Fn) {
        if (!std::isfinite(v)) finite = false;
        f1 = std::max(f1, std::fabs(v));
      }
      if (finite && f1 <= f0) break;
      lam *= 0.5;
      if (lam < 1e-8) return f0 <= 1e-3 * std::fabs(E);  // at the noise floor
    }
    p = pn;
    q = qn;
    E = En;
    F = Fn;
    double f1 = 0.0;
    for (double v : F) f1 = std::max(f1, std::fabs(v));
    if (f1 <= std::max(1e-13 * std::fabs(E), 2e-16)) break;
  }
  return true;
}

void sort_pq(Vec& p, Vec& q) {
  std::vector<int> idx(p.size());
  for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int)i;
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return p[a] < p[b]; });
  Vec p2(p.size()), q2(q.size());
  for (size_t i = 0; i < idx.size(); ++i) {
    p2[i] = p[idx[i]];
    q2[i] = q[idx[i]];
  }
  p = p2;
  q = q2;
}

struct State {
  Vec p, q, ref;
  double delta = 0.0;
};

// Remez exchange; ref (optional) is a starting reference.
bool remez(int N, double R, State& s, const Vec* ref, double tol = 1e-8, int maxit = 60) {
  Vec p = s.p, q = s.q;
  if (ref) {
    double mean = 0.0;
    for (double y : *ref) mean += std::fabs(err1(y, p, q));
    mean /= ref->size();
    const double sg = err1((*ref)[0], p, q) < 0 ? -1.0 : 1.0;
    if (!newton_reference(N, *ref, p, q, sg * mean)) return false;
  }
  for (int it = 0; it < maxit; ++it) {
    Ref r = alternation(N, R, p, q);
    if ((int)r.y.size() < 2 * N + 1) return false;
    double lo = 1e300, hi = 0.0, mean = 0.0;
    for (double v : r.e) {
      lo = std::min(lo, std::fabs(v));
      hi = std::max(hi, std::fabs(v));
      mean += std::fabs(v);
    }
    mean /= r.e.size();
    if ((hi - lo) / lo <= std::max(tol, 4e-15 / lo)) {
      s.p = p;
      s.q = q;
      s.delta = r.emax;
      s.ref = r.y;
      return true;
    }
    if (!newton_reference(N, r.y, p, q, (r.e[0] < 0 ? -1.0 : 1.0) * mean)) return false;
    sort_pq(p, q);
  }
  return false;
}

// Levenberg-Marquardt on sum (w_k e(y_k))^2.
void lm_fit(int N, const Vec& y, const Vec& wt, Vec& p, Vec& q, int iters) {
  const int n2 = 2 * N;
  const size_t m = y.size();
  auto cost = [&](const Vec& pp, const Vec& qq, Vec& r) {
    r.resize(m);
    double f = 0.0;
    for (size_t k = 0; k < m; ++k) {
      r[k] = wt[k] * err1(y[k], pp, qq);
      f += r[k] * r[k];
    }
    return f;
  };
  Vec r;
  double f = cost(p, q, r), lam = 1e-2;
  std::vector<double> row(n2);
  for (int it = 0; it < iters; ++it) {
    std::vector<double> A(n2 * n2, 0.0);
    Vec g(n2, 0.0);
    for (size_t k = 0; k < m; ++k) {
      jac_row(y[k], p, q, row.data());
      for (int a = 0; a < n2; ++a) {
        const double ja = wt[k] * row[a];
        g[a] += ja * r[k];
        for (int b = 0; b < n2; ++b) A[a * n2 + b] += ja * wt[k] * row[b];
      }
    }
    bool moved = false;
    Vec pn(N), qn(N), rn;
    double fn = 0.0;
    for (int t = 0; t < 60; ++t) {
      std::vector<double> M = A;
      for (int a = 0; a < n2; ++a) M[a * n2 + a] += lam * std::max(A[a * n2 + a], 1e-30);
      Vec rhs(n2), st;
      for (int a = 0; a < n2; ++a) rhs[a] = -g[a];
      if (lu_solve(M, rhs, n2, st)) {
        for (int n = 0; n < N; ++n) {
          pn[n] = p[n] + st[n];
          qn[n] = q[n] + st[N + n];
        }
        fn = cost(pn, qn, rn);
        if (std::isfinite(fn) && fn < f) {
          moved = true;
          break;
        }
      }
      lam *= 3.0;
    }
    if (!moved) break;
    const double gain = (f - fn) / f;
    p = pn;
    q = qn;
    r = rn;
    f = fn;
    lam = std::max(lam / 3.0, 1e-15);
    if (gain < 1e-14) break;
  }
}

bool start_fit(int N, double& Rs, State& s) {
  Rs = std::max(10.0, std::exp(1.25 * (N - 1) - 2.0));
  const double T = std::log(Rs);
  s.p.assign(N, 0.0);
  s.q.assign(N, 0.0);
  if (N == 1) {
    s.p[0] = -T / 2.0;
    s.q[0] = s.p[0] + 1.4;
  } else {
    const double h = (T + 2.0) / (N - 1);
    for (int n = 0; n < N; ++n) {
      const double sv = -1.0 + n * h;
      s.p[n] = -sv;
      s.q[n] = -sv + std::log(h);
    }
    const int m = 3000;
    Vec y(m), wt(m, 1.0);
    for (int k = 0; k < m; ++k) y[k] = std::exp(T * k / (m - 1));
    lm_fit(N, y, wt, s.p, s.q, 500);
    Vec W(m, 1.0);  // Lawson weights; residual weights are sqrt(W)
    for (int rep = 0; rep < 30; ++rep) {
      double emax = 0.0;
      Vec e(m);
      for (int k = 0; k < m; ++k) {
        e[k] = std::fabs(err1(y[k], s.p, s.q));
        emax = std::max(emax, e[k]);
      }
      double wmax = 0.0;
      for (int k = 0; k < m; ++k) {
        W[k] = W[k] * std::sqrt(e[k] / emax) + 1e-300;
        wmax = std::max(wmax, W[k]);
      }
      for (int k = 0; k < m; ++k) {
        W[k] /= wmax;
        wt[k] = std::sqrt(W[k]);
      }
      lm_fit(N, y, wt, s.p, s.q, 100);
    }
  }
  return remez(N, Rs, s, nullptr);
}

bool walk(int N, double R0, State& s, double R) {
  double cur = R0, lf = 0.25;
  int steps = 0;
  while (std::fabs(std::log(cur / R)) > 1e-13) {
    const double dl = std::log(R / cur);
    double nxt = cur * std::exp(std::clamp(dl, -lf, lf));
    if (std::fabs(std::log(nxt / R)) < 1e-13) nxt = R;
    Vec ref(s.ref.size());
    for (size_t k = 0; k < ref.size(); ++k)
      ref[k] = std::exp(std::log(s.ref[k]) * std::log(nxt) / std::log(cur));
    State t = s;
    if (++steps > 2000) return false;
    if (remez(N, nxt, t, &ref)) {
      s = t;
      cur = nxt;
      lf = std::min(0.4, lf * 1.5);
    } else {
      lf *= 0.5;
      if (lf < 1e-4) return false;
    }
  }
  return true;
}

std::mutex g_mu;
std::map<int, std::pair<double, State>> g_start;

}  // namespace

double quad_r_floor(int n) { return n <= 8 ? 1.0 : std::exp(0.5 * (n - 10) + 3.8); }

int minimax_quadrature(double x_min, double x_max, int n, double* tau, double* w,
                       double* delta) {
  if (!(x_min > 0.0) || !(x_max > x_min) || !std::isfinite(x_max) || n < 1 || n > 16) return 1;
  const double R = std::max(x_max / x_min, quad_r_floor(n));
  double R0;
  State s;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_start.find(n);
    if (it == g_start.end()) {
      if (!start_fit(n, R0, s)) return 2;
      g_start[n] = {R0, s};
    } else {
      R0 = it->second.first;
      s = it->second.second;
    }
  }
  if (!walk(n, R0, s, R)) return 2;
  sort_pq(s.p, s.q);
  for (int k = 0; k < n; ++k) {
    tau[k] = std::exp(s.p[k]) / x_min;
    w[k] = std::exp(s.q[k]) / x_min;
  }
  if (delta) *delta = s.delta;
  return 0;
}

// Remez polish from a proposal (tau, w) on [x_min, x_max]: `steps` exchange
// passes (extrema + Newton) without continuation.  Returns 0 and the
// certified spread test in *certified (1 if the 2n + 1 extrema agree to
// cert_tol relative).
int remez_polish(double x_min, double x_max, int n, int steps, double cert_tol, double* tau,
                 double* w, double* delta, int* certified) {
  if (!(x_min > 0.0) || !(x_max > x_min) || n < 1 || n > 16) return 1;
  const double R = std::max(x_max / x_min, quad_r_floor(n));
  Vec p(n), q(n);
  for (int k = 0; k < n; ++k) {
    if (!(tau[k] > 0.0) || !(w[k] > 0.0)) return 1;
    p[k] = std::log(tau[k] * x_min);
    q[k] = std::log(w[k] * x_min);
  }
  sort_pq(p, q);
  // A proposal whose error is far above the optimum shows too few
  // alternations for the exchange to start.  Solve the equioscillation system
  // first at a model reference: the normalised alternation points
  // t_k = log y_k / log R of plain fits, tabulated for N <= 12 at four ratios
  // and interpolated in log R (they depend only weakly on R); the solution
  // alternates at those points by construction.
  if (n <= 12) {
    const double T = std::log(R);
    const double* rr = kRefR[n - 1];
    int i0 = 0;
    while (i0 < 2 && R > rr[i0 + 1]) ++i0;
    double u = (std::log(R) - std::log(rr[i0])) / (std::log(rr[i0 + 1]) - std::log(rr[i0]));
    u = std::clamp(u, 0.0, 1.0);
    Vec ref(2 * n + 1);
    for (int k = 0; k <= 2 * n; ++k) {
      const double t = (1.0 - u) * kRefT[n - 1][i0][k] + u * kRefT[n - 1][i0 + 1][k];
      ref[k] = std::exp(t * T);
    }
    double mean = 0.0;
    for (double y : ref) mean += std::fabs(err1(y, p, q));
    mean /= ref.size();
    Vec p2 = p, q2 = q;
    if (newton_reference(n, ref, p2, q2, (err1(ref[0], p, q) < 0 ? -1.0 : 1.0) * mean)) {
      sort_pq(p2, q2);
      bool ok = true;
      for (int k = 0; k < n; ++k) ok = ok && std::isfinite(p2[k]) && std::isfinite(q2[k]);
      if (ok) {
        p = p2;
        q = q2;
      }
    }
  }
  for (int it = 0; it < steps; ++it) {
    Ref r = alternation(n, R, p, q);
    if ((int)r.y.size() < 2 * n + 1) break;
    double mean = 0.0;
    for (double v : r.e) mean += std::fabs(v);
    mean /= r.e.size();
    Vec p2 = p, q2 = q;
    if (!newton_reference(n, r.y, p2, q2, (r.e[0] < 0 ? -1.0 : 1.0) * mean)) break;
    sort_pq(p2, q2);
    bool ok = true;
    for (int k = 0; k < n; ++k) ok = ok && std::isfinite(p2[k]) && std::isfinite(q2[k]);
    if (!ok) break;
    p = p2;
    q = q2;
  }
  Ref r = alternation(n, R, p, q);
  int cert = 0;
  if ((int)r.y.size() == 2 * n + 1) {
    double lo = 1e300, hi = 0.0;
    for (double v : r.e) {
      lo = std::min(lo, std::fabs(v));
      hi = std::max(hi, std::fabs(v));
    }
    cert = ((hi - lo) / lo <= std::max(cert_tol, 4e-15 / lo)) ? 1 : 0;
  }
  for (int k = 0; k < n; ++k) {
    tau[k] = std::exp(p[k]) / x_min;
    w[k] = std::exp(q[k]) / x_min;
  }
  if (delta) *delta = r.emax;
  if (certified) *certified = cert;
  return 0;
}

int quadrature_table(int n, int count, const double* R, double* alpha, double* beta,
                     double* delta) {
  if (n < 1 || n > 16 || count < 0) return 1;
  for (int k = 1; k < count; ++k)
    if (!(R[k] >= R[k - 1])) return 1;
  if (count == 0) return 0;
  if (!(R[0] > 1.0)) return 1;
  const int saved = g_ngrid;
  g_ngrid = 4000;
  double R0;
  State s;
  bool have = false;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_start.find(n);
    if (it != g_start.end()) {
      R0 = it->second.first;
      s = it->second.second;
      have = true;
    }
  }
  if (!have) {
    g_ngrid = 20000;
    if (!start_fit(n, R0, s)) {
      g_ngrid = saved;
      return 2;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    g_start[n] = {R0, s};
  }
  g_ngrid = 4000;
  const double fl = quad_r_floor(n);
  double cur = R0;
  for (int k = 0; k < count; ++k) {
    const double target = std::max(R[k], fl);
    if (std::fabs(std::log(target / cur)) > 1e-13) {
      State keep = s;
      if (!walk(n, cur, s, target)) {
        // near the double-precision floor the coarse bracketing grid can
        // miss an extremum: repeat the step with the fine grid
        s = keep;
        g_ngrid = 20000;
        const bool ok = walk(n, cur, s, target);
        g_ngrid = 4000;
        if (!ok) {
          g_ngrid = saved;
          return 2;
        }
      }
      cur = target;
    }
    Vec p = s.p, q = s.q;
    sort_pq(p, q);
    for (int t = 0; t < n; ++t) {
      alpha[size_t(k) * n + t] = std::exp(p[t]);
      beta[size_t(k) * n + t] = std::exp(q[t]);
    }
    if (delta) delta[k] = s.delta;
  }
  g_ngrid = saved;
  return 0;
}

}  // namespace ltmp2
