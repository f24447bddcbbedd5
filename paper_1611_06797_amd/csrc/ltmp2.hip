// libltmp2: host side of the C ABI (validation, tables, device memory,
// per-Laplace-point drivers).  The device work is in kernels_*.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/ltmp2.h"
#include "ctx.h"
#include "dispatch.h"
#include "quadrature.h"

using namespace ltmp2;

// Spin sums of a two-channel (spin-unrestricted) cell, from the spin-orbital
// energy (Theory section, "MP2 for periodic systems"): the direct term is
// -1/2 sum_n w_n Tr[((chi_a + chi_b) v)^2], i.e. 1/4 of the spin-restricted
// trace formula (-2 Tr[(chi v)^2]) applied to chi_a + chi_b; the exchange
// term is 1/2 of the spin-restricted formula summed over the two channels.
constexpr double kSpinDirect = 0.25, kSpinExchange = 0.5;

namespace {

thread_local std::string g_setup_error;

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace



namespace {

ltmp2_status fail(ltmp2_ctx* c, ltmp2_status s, const std::string& msg) {
  if (c) {
    c->err = msg;
    if (s == LTMP2_EDEVICE) c->failed = true;
  } else {
    g_setup_error = msg;
  }
  return s;
}

#define HIPCHK(ctx, call)                                                              \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(ctx, e_ == hipErrorOutOfMemory ? LTMP2_ENOMEM : LTMP2_EDEVICE,       \
                  std::string(#call) + ": " + hipGetErrorString(e_));                  \
  } while (0)

bool smooth235(int n) {
  for (int f : {2, 3, 5})
    while (n % f == 0) n /= f;
  return n == 1;
}

bool positive_half(int a, int b, int c) {
  if (a != 0) return a > 0;
  if (b != 0) return b > 0;
  return c > 0;
}

template <class T>
ltmp2_status dalloc(ltmp2_ctx* c, T** p, size_t count) {
  void* q = nullptr;
  const size_t b = std::max<size_t>(count, 1) * sizeof(T);
  hipError_t e = hipMalloc(&q, b);
  if (e != hipSuccess)
    return fail(c, e == hipErrorOutOfMemory ? LTMP2_ENOMEM : LTMP2_EDEVICE,
                "hipMalloc(" + std::to_string(b) + " bytes): " + hipGetErrorString(e));
  c->owned.push_back(q);
  c->bytes += b;
  *p = reinterpret_cast<T*>(q);
  return LTMP2_OK;
}

ltmp2_status dalloc_bytes(ltmp2_ctx* c, void** p, size_t bytes) {
  void* q = nullptr;
  const size_t b = std::max<size_t>(bytes, 1);
  hipError_t e = hipMalloc(&q, b);
  if (e != hipSuccess)
    return fail(c, e == hipErrorOutOfMemory ? LTMP2_ENOMEM : LTMP2_EDEVICE,
                "hipMalloc(" + std::to_string(b) + " bytes): " + hipGetErrorString(e));
  c->owned.push_back(q);
  c->bytes += b;
  *p = q;
  return LTMP2_OK;
}

template <class T>
ltmp2_status upload(ltmp2_ctx* c, T** p, const std::vector<T>& v) {
  ltmp2_status s = dalloc(c, p, v.size());
  if (s) return s;
  if (!v.empty()) HIPCHK(c, hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return LTMP2_OK;
}

// Validation of everything the host receives, before any device call.
ltmp2_status validate(const ltmp2_params* p, const int32_t* miller, const double* eps,
                      const double* coeff, const double* tau, const double* w) {
  if (!p) return fail(nullptr, LTMP2_EINVAL, "params is NULL");
  if (!(p->L > 0.0) || !std::isfinite(p->L)) return fail(nullptr, LTMP2_EINVAL, "L must be > 0");
  if (p->n_fft < 4 || p->n_fft > 64 || !smooth235(p->n_fft))
    return fail(nullptr, LTMP2_EINVAL, "n_fft must be a 2,3,5-smooth size in [4, 64]");
  if (!grid_supported(p->n_fft))
    return fail(nullptr, LTMP2_EINVAL, "n_fft " + std::to_string(p->n_fft) + " is not compiled in");
  if (!(p->ecut > 0.0) || !std::isfinite(p->ecut) || !(p->eaux > 0.0) || !std::isfinite(p->eaux))
    return fail(nullptr, LTMP2_EINVAL, "ecut and eaux must be > 0");
  if (p->n_pw < 2) return fail(nullptr, LTMP2_EINVAL, "n_pw must be >= 2");
  const int nst = p->n_states ? p->n_states : p->n_pw;
  if (nst < 2 || nst > p->n_pw) return fail(nullptr, LTMP2_EINVAL, "n_states must be in [2, n_pw]");
  if (p->n_occ < 1 || p->n_occ >= nst)
    return fail(nullptr, LTMP2_EINVAL, "n_occ must be in [1, n_states - 1]");
  if (p->n_tau < 1 || p->n_tau > 16) return fail(nullptr, LTMP2_EINVAL, "n_tau must be in [1, 16]");
  if (p->prec < 0 || p->prec > 2) return fail(nullptr, LTMP2_EINVAL, "unknown precision");
  if (p->quad_mode < 0 || p->quad_mode > 2) return fail(nullptr, LTMP2_EINVAL, "unknown quad_mode");
  if (p->quad_mode == LTMP2_QUAD_LEARNED && p->n_tau > 12)
    return fail(nullptr, LTMP2_EINVAL, "learned quadrature covers n_tau <= 12");
  if (p->n_extrap < 0 || p->n_extrap == 1 || p->n_extrap > kMaxShells)
    return fail(nullptr, LTMP2_EINVAL, "n_extrap must be 0 or in [2, 8]");
  if (p->n_extrap && p->extrap_alpha != 0.0 &&
      !(p->extrap_alpha > 1.0 && std::isfinite(p->extrap_alpha)))
    return fail(nullptr, LTMP2_EINVAL, "extrap_alpha must be > 1 (or 0 for 1.05)");
  if (!miller || !eps || !coeff) return fail(nullptr, LTMP2_EINVAL, "NULL input array");
  if (p->quad_mode == LTMP2_QUAD_GIVEN) {
    if (!tau || !w) return fail(nullptr, LTMP2_EINVAL, "tau and w required with LTMP2_QUAD_GIVEN");
    for (int k = 0; k < p->n_tau; ++k)
      if (!(tau[k] > 0.0) || !(w[k] > 0.0) || !std::isfinite(tau[k]) || !std::isfinite(w[k]))
        return fail(nullptr, LTMP2_EINVAL, "tau and w must be positive and finite");
  } else if (tau || w) {
    return fail(nullptr, LTMP2_EINVAL, "tau / w given but quad_mode is not LTMP2_QUAD_GIVEN");
  }
  const int n = p->n_fft, npw = p->n_pw;
  const double b = 2.0 * M_PI / p->L;
  std::map<std::tuple<int, int, int>, int> pos;
  for (int k = 0; k < npw; ++k) {
    const int a = miller[3 * k], bb = miller[3 * k + 1], c = miller[3 * k + 2];
    if (2 * std::abs(a) >= n || 2 * std::abs(bb) >= n || 2 * std::abs(c) >= n)
      return fail(nullptr, LTMP2_EINVAL, "basis vector outside the centred FFT grid");
    const double g2 = b * b * double(a * a + bb * bb + c * c);
    if (!(0.5 * g2 < p->ecut)) return fail(nullptr, LTMP2_EINVAL, "basis vector beyond ecut");
    if (!pos.emplace(std::make_tuple(a, bb, c), k).second)
      return fail(nullptr, LTMP2_EINVAL, "duplicate Miller index");
  }
  for (int k = 0; k < npw; ++k)
    if (!pos.count(std::make_tuple(-miller[3 * k], -miller[3 * k + 1], -miller[3 * k + 2])))
      return fail(nullptr, LTMP2_EINVAL, "basis not closed under G -> -G");
  // the transforms walk each (ky, kz) column of the sphere as a run of
  // consecutive kx: a basis with a hole inside a column is rejected
  {
    std::map<std::pair<int, int>, std::vector<int>> cols;
    for (int k = 0; k < npw; ++k)
      cols[{miller[3 * k + 1], miller[3 * k + 2]}].push_back(miller[3 * k]);
    for (auto& kv : cols) {
      std::vector<int>& xs = kv.second;
      std::sort(xs.begin(), xs.end());
      if (xs.back() - xs.front() + 1 != int(xs.size()))
        return fail(nullptr, LTMP2_EINVAL,
                    "basis column (ky, kz) = (" + std::to_string(kv.first.first) + ", " +
                        std::to_string(kv.first.second) + ") is not a run of consecutive kx");
    }
  }
  for (int k = 0; k < nst; ++k) {
    if (!std::isfinite(eps[k])) return fail(nullptr, LTMP2_EINVAL, "non-finite orbital energy");
    if (k > 0 && eps[k] < eps[k - 1]) return fail(nullptr, LTMP2_EINVAL, "eps must be ascending");
  }
  if (!(eps[p->n_occ] - eps[p->n_occ - 1] > 1e-8))
    return fail(nullptr, LTMP2_EGAP, "HOMO-LUMO gap <= 1e-8 Ha");
  for (int s = 0; s < nst; ++s) {
    const double* c = coeff + 2 * size_t(s) * npw;
    double nrm = 0.0;
    for (int k = 0; k < npw; ++k) {
      if (!std::isfinite(c[2 * k]) || !std::isfinite(c[2 * k + 1]))
        return fail(nullptr, LTMP2_EINVAL, "non-finite coefficient");
      nrm += c[2 * k] * c[2 * k] + c[2 * k + 1] * c[2 * k + 1];
    }
    if (std::fabs(nrm - 1.0) > 1e-8) return fail(nullptr, LTMP2_EINVAL, "state not normalised");
  }
  return LTMP2_OK;
}

// Validation, then the orbitals brought to real form (real_orbitals.cpp):
// *use points at the caller's coefficients or at `store`.
ltmp2_status validate_and_realise(const ltmp2_params* p, const int32_t* miller, const double* eps,
                                  const double* coeff, const double* tau, const double* w,
                                  std::vector<double>& store, const double** use) {
  ltmp2_status s = validate(p, miller, eps, coeff, tau, w);
  if (s) return s;
  const int nst = p->n_states ? p->n_states : p->n_pw;
  bool changed = false;
  std::string err;
  s = real_orbitals(p->n_pw, miller, nst, eps, p->n_occ, coeff, store, &changed, err);
  if (s) return fail(nullptr, s, err);
  *use = changed ? store.data() : coeff;
  return LTMP2_OK;
}

// Weight file: "LTMP2MLP", uint32 version 1, uint32 count, count floats.
bool read_mlp_weights(const std::string& path, std::vector<float>& out) {
  if (path.empty()) return false;
  FILE* f = std::fopen(path.c_str(), "rb");
  if (!f) return false;
  char magic[8];
  uint32_t ver = 0, cnt = 0;
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "LTMP2MLP", 8) == 0 &&
            std::fread(&ver, 4, 1, f) == 1 && std::fread(&cnt, 4, 1, f) == 1 && ver == 1 &&
            cnt == LTMP2_MLP_NPARAM;
  if (ok) {
    out.resize(cnt);
    ok = std::fread(out.data(), sizeof(float), cnt, f) == cnt;
    char extra;
    ok = ok && std::fread(&extra, 1, 1, f) == 0;
    for (float v : out) ok = ok && std::isfinite(v);
  }
  std::fclose(f);
  return ok;
}

// Launch helpers --------------------------------------------------------------
ltmp2_status check_launch(ltmp2_ctx* c, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    return fail(c, LTMP2_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return LTMP2_OK;
}

hipEvent_t pooled_event(ltmp2_ctx* c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets one launch with events when timing is on.
struct StageTimer {
  ltmp2_ctx* c;
  int stage;
  hipEvent_t a = nullptr;
  StageTimer(ltmp2_ctx* cc, int s) : c(cc), stage(s) {
    if (c->timing && (a = pooled_event(c))) (void)hipEventRecord(a, c->stream);
  }
  ~StageTimer() {
    if (!a) return;
    hipEvent_t b = pooled_event(c);
    if (!b) return;
    (void)hipEventRecord(b, c->stream);
    c->marks.push_back({stage, a, b});
  }
};

void collect_timing(ltmp2_ctx* c) {
  if (c->marks.empty()) return;
  (void)hipStreamSynchronize(c->stream);
  for (auto& m : c->marks) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, m.a, m.b) == hipSuccess) {
      c->stage_ms[m.stage] += ms;
      c->stage_n[m.stage] += 1;
    }
    c->pool.push_back(m.a);
    c->pool.push_back(m.b);
  }
  c->marks.clear();
}

}  // namespace

// ---------------------------------------------------------------------------
extern "C" ltmp2_status ltmp2_quadrature(double x_min, double x_max, int n_tau, double* tau,
                                         double* w, double* delta) {
  if (!tau || !w) return fail(nullptr, LTMP2_EINVAL, "NULL output");
  const int r = minimax_quadrature(x_min, x_max, n_tau, tau, w, delta);
  if (r == 1) return fail(nullptr, LTMP2_EINVAL, "need 0 < x_min < x_max and 1 <= n_tau <= 16");
  if (r != 0) return fail(nullptr, LTMP2_ENUMERIC, "minimax fit did not converge");
  return LTMP2_OK;
}

extern "C" int ltmp2_supported_grids(int* sizes, int cap) {
  std::vector<int> g = supported_grids();
  for (int k = 0; k < (int)g.size() && k < cap; ++k) sizes[k] = g[k];
  return (int)g.size();
}

namespace {

template <class T>
ltmp2_status prepare_cell(ltmp2_ctx* c, const cplx<double>* d_coef) {
  const GridOps<T>* ops = grid_ops<T>(c->n);
  if (!ops) return fail(nullptr, LTMP2_EINVAL, "grid not compiled");
  ltmp2_status s;
  if ((s = ops->orbitals(d_coef, c->nst, c->npw, c->sc, 1.0 / std::sqrt(c->omega),
                         static_cast<T*>(c->d_psi), c->nrp, c->stream)))
    return fail(nullptr, s, "orbital synthesis launch failed");
  if ((s = ops->overlap(static_cast<const T*>(c->d_psi), c->nrp, c->no, c->nv, c->d_gdesc, c->nh,
                        c->kmax_aux, c->dV, static_cast<cplx<T>*>(c->d_nd), c->stream)))
    return fail(nullptr, s, "overlap-density launch failed");
  return LTMP2_OK;
}

ltmp2_status setup_impl(ltmp2_ctx* c, const int32_t* miller, const double* eps,
                        const double* coeff, const double* tau, const double* w) {
  const ltmp2_params& P = c->prm;
  // Transform grid: the smallest compiled grid n' <= n_fft on which every
  // product of two orbital-sphere functions is alias-free at the kept
  // auxiliary wavevectors (n' >= 2 k_orb + k_aux + 1 per axis).  There the
  // grid sums equal the plane-wave integrals, so the energies are those of
  // the n_fft grid to rounding; if n_fft itself is below the bound, n_fft is
  // used (and its aliasing is part of the model).
  int n = P.n_fft;
  {
    int ko = 0;
    for (int k = 0; k < 3 * P.n_pw; ++k) ko = std::max(ko, std::abs(int(miller[k])));
    const double bb = 2.0 * M_PI / P.L;
    const int ka = int(std::sqrt(double(int(std::floor(2.0 * P.eaux / (bb * bb) + 1e-9)))));
    const int need = 2 * ko + ka + 1;
    for (int g : supported_grids())
      if (g >= need && g < n) n = g;
  }
  c->n = n;
  c->nr = n * n * n;
  c->nrp = (c->nr + 127) / 128 * 128;  // whole 128 x 128 Green's-function tiles
  c->npw = P.n_pw;
  c->nst = P.n_states ? P.n_states : P.n_pw;
  c->no = P.n_occ;
  c->nv = c->nst - P.n_occ;
  c->ntau = P.n_tau;
  c->omega = P.L * P.L * P.L;
  c->dV = c->omega / c->nr;
  c->eps.assign(eps, eps + c->nst);
  c->mu = 0.5 * (eps[c->no - 1] + eps[c->no]);
  c->xmin = 2.0 * (eps[c->no] - eps[c->no - 1]);
  c->xmax = 2.0 * (eps[c->nst - 1] - eps[0]);
  if (c->xmax_force > 0.0) {
    c->xmin = c->xmin_force;
    c->xmax = c->xmax_force;
  }
  c->npairs = c->no * (c->no + 1) / 2;
  if (c->npairs > (1 << 22) || c->no >= (1 << 15))
    return fail(nullptr, LTMP2_EINVAL, "too many occupied states");

  // auxiliary set: H (positive half, lexicographic), then -H
  const double b = 2.0 * M_PI / P.L;
  const int lim = int(std::floor(2.0 * P.eaux / (b * b) + 1e-9));
  const int mm = int(std::sqrt(double(lim))) + 1;
  std::vector<std::array<int, 3>> H;
  for (int x = -mm; x <= mm; ++x)
    for (int y = -mm; y <= mm; ++y)
      for (int z = -mm; z <= mm; ++z) {
        const int m2 = x * x + y * y + z * z;
        if (m2 == 0 || m2 > lim || !positive_half(x, y, z)) continue;
        if (2 * std::abs(x) >= n || 2 * std::abs(y) >= n || 2 * std::abs(z) >= n)
          return fail(nullptr, LTMP2_EINVAL, "auxiliary sphere does not fit inside the FFT grid");
        H.push_back({x, y, z});
      }
  if (H.empty()) return fail(nullptr, LTMP2_EINVAL, "auxiliary set is empty");
  c->nh = (int)H.size();
  c->ng = 2 * c->nh;
  if (c->ng > max_outputs()) return fail(nullptr, LTMP2_EINVAL, "auxiliary set too large");
  c->aux.resize(3 * c->ng);
  int km = 0;
  for (int k = 0; k < c->nh; ++k)
    for (int d = 0; d < 3; ++d) {
      c->aux[3 * k + d] = H[k][d];
      c->aux[3 * (k + c->nh) + d] = -H[k][d];
      km = std::max(km, std::abs(H[k][d]));
    }
  c->kmax_aux = km;
  std::vector<int> gdesc(c->ng);
  std::vector<double> v(c->ng);
  for (int k = 0; k < c->ng; ++k) {
    const int x = c->aux[3 * k], y = c->aux[3 * k + 1], z = c->aux[3 * k + 2];
    gdesc[k] = pack_g(((x % n) + n) % n, y + km, z + km);
    v[k] = 4.0 * M_PI / (c->omega * b * b * double(x * x + y * y + z * z));
  }

  // internal cutoff extrapolation: number of nested spheres containing each
  // auxiliary vector (the same inclusive integer test as the auxiliary set)
  std::vector<signed char> shell;
  if (P.n_extrap > 0) {
    c->nb = P.n_extrap;
    c->alpha = P.extrap_alpha > 0.0 ? P.extrap_alpha : 1.05;
    c->eaux_n.resize(c->nb);
    std::vector<int> lims(c->nb);
    for (int q = 0; q < c->nb; ++q) {
      c->eaux_n[q] = P.eaux / std::pow(c->alpha, q);
      lims[q] = int(std::floor(2.0 * c->eaux_n[q] / (b * b) + 1e-9));
    }
    shell.resize(c->ng);
    for (int k = 0; k < c->ng; ++k) {
      const int x = c->aux[3 * k], y = c->aux[3 * k + 1], z = c->aux[3 * k + 2];
      const int m2 = x * x + y * y + z * z;
      int sh = 0;
      while (sh < c->nb && m2 <= lims[sh]) ++sh;
      shell[k] = static_cast<signed char>(sh);
    }
  }

  // orbital sphere in (ky, kz) column order
  int ko = 0;
  for (int k = 0; k < c->npw; ++k)
    for (int d = 0; d < 3; ++d) ko = std::max(ko, std::abs(miller[3 * k + d]));
  c->kmax_orb = ko;
  std::vector<int> order(c->npw);
  for (int k = 0; k < c->npw; ++k) order[k] = k;
  std::sort(order.begin(), order.end(), [&](int a, int bq) {
    auto key = [&](int i) {
      return std::make_tuple(miller[3 * i + 1], miller[3 * i + 2], miller[3 * i]);
    };
    return key(a) < key(bq);
  });
  std::vector<int> cdesc, cstart, ckx(c->npw);
  for (int e = 0; e < c->npw; ++e) {
    const int i = order[e];
    const int ky = miller[3 * i + 1], kz = miller[3 * i + 2];
    if (e == 0 || ky != miller[3 * order[e - 1] + 1] || kz != miller[3 * order[e - 1] + 2]) {
      cdesc.push_back((ky + ko) | ((kz + ko) << 8));
      cstart.push_back(e);
    }
    ckx[e] = miller[3 * i];
  }
  cstart.push_back(c->npw);
  // real basis of the coefficients: q = 0 for G = 0, (2k+1, 2k+2) for the
  // k-th basis vector of the positive half (in input order)
  std::map<std::tuple<int, int, int>, int> qre;
  int nq = 1, zero_idx = -1;
  for (int k = 0; k < c->npw; ++k) {
    const int x = miller[3 * k], y = miller[3 * k + 1], z = miller[3 * k + 2];
    if (x == 0 && y == 0 && z == 0) zero_idx = k;
    if (positive_half(x, y, z)) {
      qre[std::make_tuple(x, y, z)] = nq;
      nq += 2;
    }
  }
  if (zero_idx < 0 || nq != c->npw)
    return fail(nullptr, LTMP2_EINVAL, "basis must contain G = 0 and be symmetric");
  std::vector<int> wq(c->npw);
  std::vector<signed char> wsgn(c->npw);
  for (int e = 0; e < c->npw; ++e) {
    const int i = order[e];
    const int x = miller[3 * i], y = miller[3 * i + 1], z = miller[3 * i + 2];
    if (x == 0 && y == 0 && z == 0) {
      wq[e] = 0;
      wsgn[e] = 1;
    } else if (positive_half(x, y, z)) {
      const int q = qre[std::make_tuple(x, y, z)];
      wq[e] = q | ((q + 1 + 1) << 16);
      wsgn[e] = 1;
    } else {
      const int q = qre[std::make_tuple(-x, -y, -z)];
      wq[e] = q | ((q + 1 + 1) << 16);
      wsgn[e] = -1;
    }
  }
  // coefficients in column order, and the real basis of the virtual ones
  std::vector<double> coef_col(2 * size_t(c->nst) * c->npw);
  c->ldbpw = (c->npw + 3) / 4 * 4;  // 16-byte aligned rows
  std::vector<double> bpw(size_t(c->nv) * c->ldbpw, 0.0);
  for (int s = 0; s < c->nst; ++s) {
    const double* cs = coeff + 2 * size_t(s) * c->npw;
    for (int e = 0; e < c->npw; ++e) {
      coef_col[2 * (size_t(s) * c->npw + e)] = cs[2 * order[e]];
      coef_col[2 * (size_t(s) * c->npw + e) + 1] = cs[2 * order[e] + 1];
    }
    if (s >= c->no) {
      double* row = bpw.data() + size_t(s - c->no) * c->ldbpw;
      row[0] = cs[2 * zero_idx];
      for (int k = 0; k < c->npw; ++k) {
        const int x = miller[3 * k], y = miller[3 * k + 1], z = miller[3 * k + 2];
        if (!positive_half(x, y, z)) continue;
        const int q = qre[std::make_tuple(x, y, z)];
        row[q] = cs[2 * k];
        row[q + 1] = cs[2 * k + 1];
      }
    }
  }
  // pairs i <= j in blocks of (i, j): the workgroups resident on one XCD take
  // consecutive items and share the block's orbitals and transformed states
  // in that XCD's L2 and the Infinity Cache.  8 x 8 blocks; 16 x 16 for the
  // wide 512-thread pair form (auxiliary sets above 2304 vectors), measured
  // 2 % faster there.
  std::vector<int> pairs;
  const int kPairBlock = (P.prec != LTMP2_FP64 && c->ng > 9 * kThreads) ? 16 : 8;
  for (int bi = 0; bi < c->no; bi += kPairBlock)
    for (int bj = bi; bj < c->no; bj += kPairBlock)
      for (int i = bi; i < std::min(bi + kPairBlock, c->no); ++i)
        for (int j = std::max(i, bj); j < std::min(bj + kPairBlock, c->no); ++j)
          pairs.push_back(i | (j << 16));

  // quadrature
  c->tau.resize(c->ntau);
  c->w.resize(c->ntau);
  if (P.quad_mode == LTMP2_QUAD_GIVEN) {
    c->tau.assign(tau, tau + c->ntau);
    c->w.assign(w, w + c->ntau);
    double d = 0.0;
    const int ng = 20000;
    for (int k = 0; k < ng; ++k) {
      const double x = c->xmin * std::exp(std::log(c->xmax / c->xmin) * k / (ng - 1));
      double s = 0.0;
      for (int t = 0; t < c->ntau; ++t) s += c->w[t] * std::exp(-x * c->tau[t]);
      d = std::max(d, std::fabs(x * s - 1.0));
    }
    c->quad_delta = d;
  } else if (P.quad_mode == LTMP2_QUAD_LEARNED) {
    std::vector<float> prm;
    if (!read_mlp_weights(c->mlp_path, prm)) {
      c->quad_flags = 4 | 2;
      const int r = minimax_quadrature(c->xmin, c->xmax, c->ntau, c->tau.data(), c->w.data(),
                                       &c->quad_delta);
      if (r != 0) return fail(nullptr, LTMP2_ENUMERIC, "minimax quadrature did not converge");
    } else {
      ltmp2_status q = ltmp2_learned_quadrature(prm.data(), c->xmin, c->xmax, c->ntau, 3, 1e-6,
                                                c->tau.data(), c->w.data(), &c->quad_delta,
                                                &c->quad_flags, c->stream);
      if (q) return fail(nullptr, q, std::string("learned quadrature: ") + ltmp2_mlp_last_error());
    }
  } else {
    const int r = minimax_quadrature(c->xmin, c->xmax, c->ntau, c->tau.data(), c->w.data(),
                                     &c->quad_delta);
    if (r != 0) return fail(nullptr, LTMP2_ENUMERIC, "minimax quadrature did not converge");
  }
  std::vector<double> fo(size_t(c->ntau) * c->no), fv(size_t(c->ntau) * c->nv);
  for (int t = 0; t < c->ntau; ++t) {
    for (int i = 0; i < c->no; ++i) fo[size_t(t) * c->no + i] = std::exp((eps[i] - c->mu) * c->tau[t]);
    for (int a = 0; a < c->nv; ++a)
      fv[size_t(t) * c->nv + a] = std::exp(-(eps[c->no + a] - c->mu) * c->tau[t]);
  }

  // device footprint and G'-block size
  const size_t nrp = c->nrp;
  c->esz = (P.prec == LTMP2_FP64) ? sizeof(double) : sizeof(float);
  const size_t es = c->esz;
  size_t fixed = es * (size_t(c->nst) * nrp + 2 * size_t(c->nv) * c->nh * c->no +
                       size_t(c->nv) * c->ldbpw +
                       (c->own_scratch ? nrp * nrp + 2 * size_t(c->nh) * nrp : 0)) +
                 sizeof(double) * (size_t(c->nh) + size_t(c->nh) * c->npairs) +
                 sizeof(double) * 2 * size_t(c->nst) * c->npw;
  if (c->nb)
    fixed += sizeof(double) * size_t(c->nb) *
             (2 * size_t(c->nh) + size_t(c->nh) * c->npairs + 2 * size_t(c->ntau));
  if (P.prec == LTMP2_BF16X3) {
    c->kpo = (c->no + 63) / 64 * 64;
    c->kpv = (c->nv + 63) / 64 * 64;
    c->ldnd3 = (2L * c->nh * c->no + 127) / 128 * 128 + 128;
    c->ldb3 = (c->npw + 127) / 128 * 128;
    fixed += 4 * (size_t(c->kpo + c->kpv) * nrp + size_t(c->kpv) * c->ldnd3 +
                  size_t(c->kpv) * c->ldb3);
  }
  const size_t per_g = es * (2 * size_t(c->no) * c->npw + 2 * size_t(c->no) * nrp);
  size_t budget = size_t(8) << 30;
  if (P.workspace_cap) {
    if (fixed + per_g > P.workspace_cap)
      return fail(nullptr, LTMP2_ENOMEM, "workspace cap below the minimum device footprint");
    budget = std::min(budget, P.workspace_cap - fixed);
  }
  c->gblock = (int)std::max<size_t>(1, std::min<size_t>(c->nh, budget / per_g));

  // the inverse transforms pack a column's first entry into 16 bits
  if (ckx.size() >= 65536)
    return fail(nullptr, LTMP2_EINVAL, "orbital sphere above 65535 plane waves");
  // device allocations and uploads
  ltmp2_status s;
  if ((s = upload(c, &c->d_cdesc, cdesc)) || (s = upload(c, &c->d_cstart, cstart)) ||
      (s = upload(c, &c->d_ckx, ckx)) || (s = upload(c, &c->d_wq, wq)) ||
      (s = upload(c, &c->d_wsgn, wsgn)) || (s = upload(c, &c->d_gdesc, gdesc)) ||
      (s = upload(c, &c->d_pairs, pairs)) || (s = upload(c, &c->d_v, v)) ||
      (s = upload(c, &c->d_fo, fo)) || (s = upload(c, &c->d_fv, fv)))
    return s;
  if (es == sizeof(double)) {
    double* d = nullptr;
    if ((s = upload(c, &d, bpw))) return s;
    c->d_bpw = d;
  } else {
    std::vector<float> bf(bpw.begin(), bpw.end());
    float* d = nullptr;
    if ((s = upload(c, &d, bf))) return s;
    c->d_bpw = d;
  }
  c->sc = SphereCols{(int)cdesc.size(), ko, c->d_cdesc, c->d_cstart, c->d_ckx};
  double* d_coef = nullptr;
  if ((s = upload(c, &d_coef, coef_col))) return s;
  if ((s = dalloc_bytes(c, &c->d_psi, es * size_t(c->nst) * nrp)) ||
      (s = dalloc_bytes(c, &c->d_nd, es * 2 * size_t(c->nv) * c->nh * c->no)) ||
      (c->own_scratch && (s = dalloc_bytes(c, &c->d_chi, es * nrp * nrp))) ||
      (c->own_scratch && (s = dalloc_bytes(c, &c->d_chihat, es * 2 * size_t(c->nh) * nrp))) ||
      (s = dalloc(c, &c->d_pd, c->nh)) ||
      (s = dalloc(c, &c->d_xpart, size_t(c->nh) * c->npairs)) ||
      (s = dalloc(c, &c->d_xrow, size_t(c->nh))) ||
      (s = dalloc(c, &c->d_scal, 2 * size_t(c->ntau) + 8)))
    return s;
  if (P.prec == LTMP2_BF16X3) {
    const size_t bp = 2 * size_t(c->kpo + c->kpv) * nrp, bn = 2 * size_t(c->kpv) * c->ldnd3,
                 bb = 2 * size_t(c->kpv) * c->ldb3;
    if ((s = dalloc_bytes(c, &c->d_psi3h, bp)) || (s = dalloc_bytes(c, &c->d_psi3l, bp)) ||
        (s = dalloc_bytes(c, &c->d_nd3h, bn)) || (s = dalloc_bytes(c, &c->d_nd3l, bn)) ||
        (s = dalloc_bytes(c, &c->d_b3h, bb)) || (s = dalloc_bytes(c, &c->d_b3l, bb)))
      return s;
    HIPCHK(c, hipMemsetAsync(c->d_nd3h, 0, bn, c->stream));
    HIPCHK(c, hipMemsetAsync(c->d_nd3l, 0, bn, c->stream));
    HIPCHK(c, hipMemsetAsync(c->d_b3h, 0, bb, c->stream));
    HIPCHK(c, hipMemsetAsync(c->d_b3l, 0, bb, c->stream));
  }
  if (c->nb) {
    if ((s = upload(c, &c->d_shell, shell)) || (s = dalloc(c, &c->d_pdb, size_t(c->nh) * c->nb)) ||
        (s = dalloc(c, &c->d_xb, size_t(c->nh) * c->npairs * c->nb)) ||
        (s = dalloc(c, &c->d_xrowb, size_t(c->nh) * c->nb)) ||
        (s = dalloc(c, &c->d_scalb, 2 * size_t(c->ntau) * c->nb)))
      return s;
    HIPCHK(c, hipMemsetAsync(c->d_scalb, 0, sizeof(double) * 2 * size_t(c->ntau) * c->nb,
                             c->stream));
  }
  // transformed-state buffers last, sized by what the cap leaves
  if (c->own_scratch) {
    if (P.workspace_cap) {
      if (c->bytes + per_g > P.workspace_cap)
        return fail(nullptr, LTMP2_ENOMEM, "device footprint exceeds the workspace cap");
      c->gblock = (int)std::min<size_t>(c->gblock, (P.workspace_cap - c->bytes) / per_g);
    }
    if ((s = dalloc_bytes(c, &c->d_P, es * 2 * size_t(c->gblock) * c->no * c->npw)) ||
        (s = dalloc_bytes(c, &c->d_w, es * 2 * size_t(c->gblock) * c->no * nrp)))
      return s;
  }
  if (P.workspace_cap && c->bytes > P.workspace_cap)
    return fail(nullptr, LTMP2_ENOMEM, "device footprint exceeds the workspace cap");
  HIPCHK(c, hipMemsetAsync(c->d_psi, 0, es * size_t(c->nst) * nrp, c->stream));
  HIPCHK(c, hipMemsetAsync(c->d_scal, 0, sizeof(double) * (2 * size_t(c->ntau) + 8), c->stream));

  // orbitals on the grid, then overlap densities (step (i))
  s = (es == sizeof(double))
          ? prepare_cell<double>(c, reinterpret_cast<const cplx<double>*>(d_coef))
          : prepare_cell<float>(c, reinterpret_cast<const cplx<double>*>(d_coef));
  if (s) return s;
  if (P.prec == LTMP2_BF16X3 &&
      (s = launch_split3(static_cast<const float*>(c->d_nd), 2L * c->nh * c->no, c->nv, c->kpv,
                         2 * c->nh * c->no, c->ldnd3, nullptr, 0, c->d_nd3h, c->d_nd3l, 0,
                         c->stream)))
    return fail(nullptr, s, "overlap-density split launch failed");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LTMP2_OK;
}

ltmp2_status usable(ltmp2_ctx* c, int itau) {
  if (!c) return LTMP2_EINVAL;
  if (c->failed) return fail(c, LTMP2_ESTATE, "context failed earlier: " + c->err);
  if (itau < 0 || itau >= c->ntau) return fail(c, LTMP2_EINVAL, "itau out of range");
  return LTMP2_OK;
}

// chi(r, r') = G_occ(r, r') G_vir(r', r) of context c's orbitals at tau_itau
// into `chi` (added to it when accumulate is set: the second spin channel)
template <class T, int MODE>
ltmp2_status chi_tiles_t(ltmp2_ctx* c, int itau, void* chi, int accumulate) {
  const double* fo = c->d_fo + size_t(itau) * c->no;
  const double* fv = c->d_fv + size_t(itau) * c->nv;
  ltmp2_status s;
  if constexpr (MODE == kBF16x3) {
    const float* psi = static_cast<const float*>(c->d_psi);
    s = launch_split3(psi, c->nrp, c->no, c->kpo, int(c->nrp), c->nrp, fo, 2, c->d_psi3h,
                      c->d_psi3l, 0, c->stream);
    if (!s)
      s = launch_split3(psi + long(c->no) * c->nrp, c->nrp, c->nv, c->kpv, int(c->nrp), c->nrp,
                        fv, 2, c->d_psi3h, c->d_psi3l, c->kpo / 8, c->stream);
    if (!s)
      s = launch_chi3(c->d_psi3h, c->d_psi3l, c->nrp, c->kpo, c->kpv, c->nrp,
                      static_cast<float*>(chi), c->nrp, accumulate, c->stream);
  } else {
    s = launch_gf_chi<MODE>(c->d_psi, c->nrp, c->no, c->nv, fo, fv, chi, c->nrp, c->nrp,
                            accumulate, c->stream);
  }
  return s;
}

// direct term at one Laplace point; value left in d_scal[2 * itau].  With a
// second spin channel (c->beta) chi is the sum of both channels' products.
template <class T, int MODE>
ltmp2_status run_direct_t(ltmp2_ctx* c, int itau, double* chi_out) {
  ltmp2_status s;
  const GridOps<T>* ops = grid_ops<T>(c->n);
  {
    StageTimer tm(c, 0);
    s = chi_tiles_t<T, MODE>(c, itau, c->d_chi, 0);
    if (!s && c->beta) s = chi_tiles_t<T, MODE>(c->beta, itau, c->d_chi, 1);
  }
  if (s) return fail(c, s, "chi tile launch failed");
  {
    StageTimer tm(c, 1);
    s = ops->chi_rows(static_cast<const T*>(c->d_chi), c->nrp, c->nr, c->d_gdesc, c->nh,
                      c->kmax_aux, c->dV, static_cast<cplx<T>*>(c->d_chihat), c->stream);
  }
  if (s) return fail(c, s, "chi row transform launch failed");
  {
    StageTimer tm(c, 2);
    ShellBins bins;
    if (c->nb) bins = ShellBins{c->d_shell, c->nb, c->d_pdb};
    s = ops->chi_cols(static_cast<const cplx<T>*>(c->d_chihat), c->nrp, c->d_gdesc, c->ng, c->nh,
                      c->d_v, c->kmax_aux, c->dV, c->d_pd,
                      reinterpret_cast<cplx<double>*>(chi_out), bins, c->stream);
  }
  if (s) return fail(c, s, "chi column transform launch failed");
  StageTimer tm(c, 6);
  hipLaunchKernelGGL(k_reduce_direct, dim3(1), dim3(256), 0, c->stream, c->d_pd, c->nh,
                     c->d_scal + 2 * itau);
  if (c->nb)
    hipLaunchKernelGGL(k_reduce_direct_bins, dim3(1), dim3(256), 0, c->stream, c->d_pdb, c->nh,
                       c->nb, c->d_scalb + size_t(2 * itau) * c->nb);
  return check_launch(c, "k_reduce_direct");
}

ltmp2_status direct_tau(ltmp2_ctx* c, int itau, double* chi_out) {
  switch (c->prm.prec) {
    case LTMP2_FP64: return run_direct_t<double, kF64>(c, itau, chi_out);
    case LTMP2_FP32: return run_direct_t<float, kF32>(c, itau, chi_out);
    default: return run_direct_t<float, kBF16x3>(c, itau, chi_out);
  }
}

// transformed states of one block of outer G' (GEMM P = C Psi_v, synthesis of w)
template <class T, int MODE>
ltmp2_status block_prepare_t(ltmp2_ctx* c, int itau, int g0, int gb) {
  ltmp2_status s;
  const GridOps<T>* ops = grid_ops<T>(c->n);
  const double* fo = c->d_fo + size_t(itau) * c->no;
  const double* fv = c->d_fv + size_t(itau) * c->nv;
  const long lda = 2L * c->nh * c->no;
  const int M = 2 * gb * c->no;
  // P = C Psi_v in the real basis:  C_ja = fo_j fv_a n_aj(G')
  {
    StageTimer tm(c, 3);
    if constexpr (MODE == kBF16x3) {
      // C_ja Psi_v = fo_j sum_a n_aj (fv_a B_a): the virtual factors go into B
      s = launch_split3(static_cast<const float*>(c->d_bpw), c->ldbpw, c->nv, c->kpv, c->npw,
                        c->ldb3, fv, 1, c->d_b3h, c->d_b3l, 0, c->stream);
      if (!s)
        s = launch_mm3(c->d_nd3h, c->d_nd3l, c->ldnd3, 2L * g0 * c->no, c->d_b3h, c->d_b3l,
                       c->ldb3, static_cast<float*>(c->d_P), c->npw, M, c->npw, c->kpv, fo, 2,
                       c->no, c->stream);
    } else {
      s = launch_gemm_kmajor<MODE>(static_cast<const T*>(c->d_nd) + 2L * g0 * c->no, lda,
                                   c->d_bpw, (long)c->ldbpw, c->d_P, (long)c->npw, M, c->npw,
                                   c->nv, fv, fo, 2, c->no, c->stream);
    }
  }
  if (s) return fail(c, s, "transformed-state GEMM launch failed");
  {
    StageTimer tm(c, 4);
    s = ops->wstates(static_cast<const T*>(c->d_P), c->npw, c->d_wq, c->d_wsgn, c->sc, gb * c->no,
                     1.0 / std::sqrt(c->omega), static_cast<cplx<T>*>(c->d_w), c->nrp, c->stream);
  }
  if (s) return fail(c, s, "transformed-state launch failed");
  return LTMP2_OK;
}

template <class T>
ltmp2_status block_pair_t(ltmp2_ctx* c, int g0, int gb) {
  const GridOps<T>* ops = grid_ops<T>(c->n);
  StageTimer tm(c, 5);
  ltmp2_status s = ops->pair(static_cast<const T*>(c->d_psi), c->nrp,
                             static_cast<const cplx<T>*>(c->d_w), c->no, c->d_pairs, c->npairs, gb,
                             c->d_gdesc, c->ng, c->d_v, c->kmax_aux, c->dV * c->dV,
                             c->d_xpart + size_t(g0) * c->npairs, c->d_shell,
                             c->nb ? c->d_xb + size_t(g0) * c->npairs * c->nb : nullptr, c->nb,
                             g0, c->stream);
  if (s) return fail(c, s, "pair transform launch failed");
  return LTMP2_OK;
}

ltmp2_status reduce_x(ltmp2_ctx* c, int itau, int g_first, int g_count) {
  StageTimer tm(c, 6);
  if (g_count <= 0) return LTMP2_OK;
  hipLaunchKernelGGL(k_reduce_xrows, dim3(g_count), dim3(256), 0, c->stream, c->d_xpart, g_first,
                     c->npairs, c->d_v, c->d_xrow);
  hipLaunchKernelGGL(k_reduce_exchange, dim3(1), dim3(256), 0, c->stream, c->d_xrow, g_first,
                     g_count, c->d_scal + 2 * itau + 1);
  if (c->nb) {
    hipLaunchKernelGGL(k_reduce_xrows_bins, dim3(g_count), dim3(256), 0, c->stream, c->d_xb,
                       g_first, c->npairs, c->nb, c->d_v, c->d_xrowb);
    hipLaunchKernelGGL(k_reduce_exchange_bins, dim3(1), dim3(256), 0, c->stream, c->d_xrowb,
                       g_first, g_count, c->nb, c->d_scalb + size_t(2 * itau + 1) * c->nb);
  }
  return check_launch(c, "k_reduce_exchange");
}

ltmp2_status block_prepare(ltmp2_ctx* c, int itau, int g0, int gb) {
  switch (c->prm.prec) {
    case LTMP2_FP64: return block_prepare_t<double, kF64>(c, itau, g0, gb);
    case LTMP2_FP32: return block_prepare_t<float, kF32>(c, itau, g0, gb);
    default: return block_prepare_t<float, kBF16x3>(c, itau, g0, gb);
  }
}

// exchange term at one Laplace point for G' in H[g_first, g_first + g_count)
ltmp2_status exchange_tau(ltmp2_ctx* c, int itau, int g_first, int g_count) {
  ltmp2_status s;
  for (int g0 = g_first; g0 < g_first + g_count; g0 += c->gblock) {
    const int gb = std::min(c->gblock, g_first + g_count - g0);
    if ((s = block_prepare(c, itau, g0, gb))) return s;
    s = (c->prm.prec == LTMP2_FP64) ? block_pair_t<double>(c, g0, gb) : block_pair_t<float>(c, g0, gb);
    if (s) return s;
  }
  return reduce_x(c, itau, g_first, g_count);
}

// G_occ / G_vir rows into double buffers (float contexts go through chi as scratch)
template <class T, int MODE>
ltmp2_status green_t(ltmp2_ctx* c, int itau, int row0, int nrows, double* gocc, double* gvir) {
  const double* fo = c->d_fo + size_t(itau) * c->no;
  const double* fv = c->d_fv + size_t(itau) * c->nv;
  const T* psi = static_cast<const T*>(c->d_psi);
  for (int which = 0; which < 2; ++which) {
    double* out = which ? gvir : gocc;
    if (!out) continue;
    const T* base = psi + (which ? size_t(c->no) * c->nrp : 0);
    const int K = which ? c->nv : c->no;
    void* dst = (sizeof(T) == sizeof(double)) ? static_cast<void*>(out) : c->d_chi;
    ltmp2_status s = launch_gemm_kmajor<MODE>(base + row0, c->nrp, base, c->nrp, dst, (long)c->nr,
                                              nrows, c->nr, K, which ? fv : fo, nullptr, 1, 1,
                                              c->stream);
    if (s) return fail(c, s, "Green's-function GEMM launch failed");
    if (sizeof(T) != sizeof(double)) {
      const long cnt = long(nrows) * c->nr;
      hipLaunchKernelGGL(k_widen, dim3(unsigned((cnt + 255) / 256)), dim3(256), 0, c->stream,
                         static_cast<const float*>(c->d_chi), out, cnt);
      if ((s = check_launch(c, "k_widen"))) return s;
    }
  }
  return LTMP2_OK;
}

// Split-BF16x3 contexts: the rows come from the same split operands and
// matrix-core kernel family as the chi tiles (sqrt-scaled orbitals split into
// hi / lo BF16, hi*hi + hi*lo + lo*hi in FP32), computed on whole 128-row
// tiles into the chi scratch and widened to double.
ltmp2_status green_split3(ltmp2_ctx* c, int itau, int row0, int nrows, double* gocc,
                          double* gvir) {
  const double* fo = c->d_fo + size_t(itau) * c->no;
  const double* fv = c->d_fv + size_t(itau) * c->nv;
  const float* psi = static_cast<const float*>(c->d_psi);
  ltmp2_status s = launch_split3(psi, c->nrp, c->no, c->kpo, int(c->nrp), c->nrp, fo, 2,
                                 c->d_psi3h, c->d_psi3l, 0, c->stream);
  if (!s)
    s = launch_split3(psi + long(c->no) * c->nrp, c->nrp, c->nv, c->kpv, int(c->nrp), c->nrp, fv,
                      2, c->d_psi3h, c->d_psi3l, c->kpo / 8, c->stream);
  if (s) return fail(c, s, "operand split launch failed");
  // whole 128-row tiles, so every operand row read stays inside the n_rp
  // padded rows of the split arrays
  const long r0 = long(row0) / 128 * 128;
  const int M = int(std::min<long>(c->nrp, (long(row0) + nrows + 127) / 128 * 128) - r0);
  for (int which = 0; which < 2; ++which) {
    double* out = which ? gvir : gocc;
    if (!out) continue;
    const long off = which ? long(c->kpo / 8) * c->nrp * 8 : 0;
    const __bf16* hi = static_cast<const __bf16*>(c->d_psi3h) + off;
    const __bf16* lo = static_cast<const __bf16*>(c->d_psi3l) + off;
    s = launch_mm3(hi, lo, c->nrp, r0, hi, lo, c->nrp, static_cast<float*>(c->d_chi),
                   (long)c->nr, M, c->nr, which ? c->kpv : c->kpo, nullptr, 1, 1, c->stream);
    if (s) return fail(c, s, "Green's-function split GEMM launch failed");
    const long cnt = long(nrows) * c->nr;
    hipLaunchKernelGGL(k_widen, dim3(unsigned((cnt + 255) / 256)), dim3(256), 0, c->stream,
                       static_cast<const float*>(c->d_chi) + (row0 - r0) * long(c->nr), out, cnt);
    if ((s = check_launch(c, "k_widen"))) return s;
  }
  return LTMP2_OK;
}

// Direct term at one Laplace point through the transformed states (the
// Hartree-like step (iv.a)): per block of outer G', the W GEMM and synthesis
// of the exchange path, h = sum_i psi_i w_i, its transform onto the
// auxiliary set and the Coulomb-weighted sum; value in d_scal[2 n_tau].
template <class T>
ltmp2_status hartree_tau_t(ltmp2_ctx* c, int itau) {
  const GridOps<T>* ops = grid_ops<T>(c->n);
  ltmp2_status s;
  cplx<T>* h = static_cast<cplx<T>*>(c->d_chi);  // free outside the chi route
  for (int g0 = 0; g0 < c->nh; g0 += c->gblock) {
    const int gb = std::min(c->gblock, c->nh - g0);
    if ((s = block_prepare(c, itau, g0, gb))) return s;
    if ((s = launch_hsum<T>(static_cast<const T*>(c->d_psi), c->nrp,
                            static_cast<const cplx<T>*>(c->d_w), c->no, c->nr, gb, h, c->stream)))
      return fail(c, s, "state-sum launch failed");
    if ((s = ops->hartree(h, c->nrp, c->d_gdesc, c->ng, c->d_v, c->kmax_aux, c->dV, g0, gb,
                          c->d_pd, c->stream)))
      return fail(c, s, "Hartree-like transform launch failed");
  }
  hipLaunchKernelGGL(k_reduce_direct, dim3(1), dim3(256), 0, c->stream, c->d_pd, c->nh,
                     c->d_scal + 2 * c->ntau);
  return check_launch(c, "k_reduce_direct");
}

}  // namespace

extern "C" ltmp2_status ltmp2_direct_hartree(ltmp2_ctx* c, int itau, double* e_direct_tau) {
  ltmp2_status s = usable(c, itau);
  if (s) return s;
  if (!c->own_scratch || !c->d_chi)
    return fail(c, LTMP2_ESTATE, "the Hartree-like route needs a context of its own (ltmp2_setup)");
  if (c->beta)
    return fail(c, LTMP2_ESTATE, "the Hartree-like route covers spin-restricted cells");
  s = (c->prm.prec == LTMP2_FP64) ? hartree_tau_t<double>(c, itau) : hartree_tau_t<float>(c, itau);
  if (s) return s;
  double v = 0.0;
  HIPCHK(c, hipMemcpyAsync(&v, c->d_scal + 2 * c->ntau, sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (!std::isfinite(v)) return fail(c, LTMP2_ENUMERIC, "non-finite direct term");
  if (e_direct_tau) *e_direct_tau = c->escale * v;
  return LTMP2_OK;
}

namespace ltmp2 {
ltmp2_status run_direct(ltmp2_ctx* c, int itau, double* chi_out) {
  return direct_tau(c, itau, chi_out);
}
ltmp2_status run_exchange(ltmp2_ctx* c, int itau, int g_first, int g_count) {
  return exchange_tau(c, itau, g_first, g_count);
}
ltmp2_status exchange_block_prepare(ltmp2_ctx* c, int itau, int g0, int gb) {
  return block_prepare(c, itau, g0, gb);
}
ltmp2_status exchange_reduce(ltmp2_ctx* c, int itau, int g_first, int g_count) {
  return reduce_x(c, itau, g_first, g_count);
}
ltmp2_status setup_cell(ltmp2_ctx* c, const int32_t* miller, const double* eps,
                        const double* coeff, const double* tau, const double* w) {
  return setup_impl(c, miller, eps, coeff, tau, w);
}
ltmp2_status validate_inputs(const ltmp2_params* p, const int32_t* miller, const double* eps,
                             const double* coeff, const double* tau, const double* w,
                             std::vector<double>& store, const double** use) {
  return validate_and_realise(p, miller, eps, coeff, tau, w, store, use);
}
const std::string& setup_error() { return g_setup_error; }
void set_setup_error(const std::string& msg) { g_setup_error = msg; }
}  // namespace ltmp2

extern "C" ltmp2_status ltmp2_setup(const ltmp2_params* p, const int32_t* miller,
                                    const double* eps, const double* coeff, const double* tau,
                                    const double* w, const char* mlp_weights, void* hip_stream,
                                    ltmp2_ctx** out) {
  if (!out) return fail(nullptr, LTMP2_EINVAL, "out is NULL");
  *out = nullptr;
  std::vector<double> creal;
  ltmp2_status s = validate_and_realise(p, miller, eps, coeff, tau, w, creal, &coeff);
  if (s) return s;
  ltmp2_ctx* c = new ltmp2_ctx();
  c->prm = *p;
  if (mlp_weights) c->mlp_path = mlp_weights;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  s = setup_impl(c, miller, eps, coeff, tau, w);
  if (s) {
    if (!c->err.empty() && g_setup_error.empty()) g_setup_error = c->err;
    ltmp2_destroy(c);
    return s;
  }
  *out = c;
  return LTMP2_OK;
}

extern "C" ltmp2_status ltmp2_setup_unrestricted(const ltmp2_params* p, int n_occ_b,
                                                 const int32_t* miller, const double* eps_a,
                                                 const double* coeff_a, const double* eps_b,
                                                 const double* coeff_b, const double* tau,
                                                 const double* w, const char* mlp_weights,
                                                 void* hip_stream, ltmp2_ctx** out) {
  if (!out) return fail(nullptr, LTMP2_EINVAL, "out is NULL");
  *out = nullptr;
  if (!p) return fail(nullptr, LTMP2_EINVAL, "params is NULL");
  ltmp2_params pb = *p;
  pb.n_occ = n_occ_b;
  std::vector<double> creal_a, creal_b;
  ltmp2_status s = validate_and_realise(p, miller, eps_a, coeff_a, tau, w, creal_a, &coeff_a);
  if (s) return s;
  if ((s = validate_and_realise(&pb, miller, eps_b, coeff_b, tau, w, creal_b, &coeff_b)))
    return fail(nullptr, s, "spin channel 2: " + g_setup_error);
  // common quadrature range: every denominator of either channel
  const int nst = p->n_states ? p->n_states : p->n_pw;
  const double xmin = 2.0 * std::min(eps_a[p->n_occ] - eps_a[p->n_occ - 1],
                                     eps_b[n_occ_b] - eps_b[n_occ_b - 1]);
  const double xmax = 2.0 * std::max(eps_a[nst - 1] - eps_a[0], eps_b[nst - 1] - eps_b[0]);
  ltmp2_ctx* c = new ltmp2_ctx();
  c->prm = *p;
  if (mlp_weights) c->mlp_path = mlp_weights;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  c->xmin_force = xmin;
  c->xmax_force = xmax;
  s = setup_impl(c, miller, eps_a, coeff_a, tau, w);
  if (!s) {
    // channel 2 takes channel 1's quadrature and shares its scratch
    ltmp2_ctx* b = new ltmp2_ctx();
    c->beta = b;
    b->prm = pb;
    b->prm.quad_mode = LTMP2_QUAD_GIVEN;
    b->stream = c->stream;
    b->own_scratch = false;
    b->xmin_force = xmin;
    b->xmax_force = xmax;
    s = setup_impl(b, miller, eps_b, coeff_b, c->tau.data(), c->w.data());
    if (s) {
      if (!b->err.empty() && g_setup_error.empty()) g_setup_error = b->err;
      g_setup_error = "spin channel 2: " + g_setup_error;
    } else {
      // transformed-state blocks of channel 2 in channel 1's P / w buffers
      const long room = long(c->gblock) * c->no;
      if (room >= b->no) {
        b->gblock = int(std::min<long>(b->nh, room / b->no));
        b->d_P = c->d_P;
        b->d_w = c->d_w;
      } else {
        const size_t es = b->esz;
        if ((s = dalloc_bytes(b, &b->d_P, es * 2 * size_t(b->gblock) * b->no * b->npw)) ||
            (s = dalloc_bytes(b, &b->d_w, es * 2 * size_t(b->gblock) * b->no * b->nrp)))
          g_setup_error = "spin channel 2: " + b->err;
      }
      b->d_chi = c->d_chi;  // chi tiles of channel 2 accumulate here
      b->d_chihat = c->d_chihat;
    }
  }
  if (s) {
    if (!c->err.empty() && g_setup_error.empty()) g_setup_error = c->err;
    ltmp2_destroy(c);
    return s;
  }
  *out = c;
  return LTMP2_OK;
}

extern "C" ltmp2_status ltmp2_setup_kpoints(const ltmp2_params* p, int n_k,
                                            const int32_t* n_pw_k, const int32_t* miller,
                                            const double* eps, const double* coeff,
                                            const double* tau, const double* w,
                                            const char* mlp_weights, void* hip_stream,
                                            ltmp2_ctx** out) {
  if (!out) return fail(nullptr, LTMP2_EINVAL, "out is NULL");
  *out = nullptr;
  if (!p || !n_pw_k || !miller || !eps || !coeff)
    return fail(nullptr, LTMP2_EINVAL, "NULL argument");
  if (n_k < 1 || n_k > 6) return fail(nullptr, LTMP2_EINVAL, "n_k must be in [1, 6]");
  const int nk = n_k * n_k * n_k;
  long total = 0;
  for (int t = 0; t < nk; ++t) total += n_pw_k[t];
  if (total != p->n_pw)
    return fail(nullptr, LTMP2_EINVAL, "n_pw must be the sum of the per-k basis sizes");
  if (p->n_states <= 0) return fail(nullptr, LTMP2_EINVAL, "n_states (bands per k) must be set");
  if (!(p->L > 0.0) || p->n_fft <= 0 || p->n_fft * n_k > 4096)
    return fail(nullptr, LTMP2_EINVAL, "bad cell or grid");
  std::vector<int32_t> ms;
  std::vector<double> es, cs;
  std::string err;
  ltmp2_status s = unfold_kmesh(n_k, p->n_states, p->n_occ, n_pw_k, miller, eps, coeff, ms, es,
                                cs, err);
  if (s) return fail(nullptr, s, err);
  // the Born-von Karman supercell as a Gamma-point cell
  ltmp2_params ps = *p;
  ps.L = p->L * n_k;
  ps.n_fft = p->n_fft * n_k;
  ps.n_pw = int(total);
  ps.n_states = nk * p->n_states;
  ps.n_occ = nk * p->n_occ;
  const double* cuse = cs.data();
  std::vector<double> creal;
  if ((s = validate_and_realise(&ps, ms.data(), es.data(), cs.data(), tau, w, creal, &cuse)))
    return fail(nullptr, s, "supercell of the mesh: " + g_setup_error);
  ltmp2_ctx* c = new ltmp2_ctx();
  c->prm = ps;
  c->escale = 1.0 / nk;
  c->n_kmesh = n_k;
  if (mlp_weights) c->mlp_path = mlp_weights;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  s = setup_impl(c, ms.data(), es.data(), cuse, tau, w);
  if (s) {
    if (!c->err.empty() && g_setup_error.empty()) g_setup_error = c->err;
    ltmp2_destroy(c);
    return s;
  }
  *out = c;
  return LTMP2_OK;
}

extern "C" ltmp2_status ltmp2_green(ltmp2_ctx* c, int itau, int row0, int nrows, void* gocc,
                                    void* gvir) {
  ltmp2_status s = usable(c, itau);
  if (s) return s;
  if (row0 < 0 || nrows < 0 || row0 + nrows > c->nr)
    return fail(c, LTMP2_EINVAL, "row range outside [0, n_r)");
  if (nrows == 0) return LTMP2_OK;
  if (c->prm.prec == LTMP2_FP64)
    s = green_t<double, kF64>(c, itau, row0, nrows, static_cast<double*>(gocc),
                              static_cast<double*>(gvir));
  else if (c->prm.prec == LTMP2_FP32)
    s = green_t<float, kF32>(c, itau, row0, nrows, static_cast<double*>(gocc),
                             static_cast<double*>(gvir));
  else
    s = green_split3(c, itau, row0, nrows, static_cast<double*>(gocc),
                     static_cast<double*>(gvir));
  if (s) return s;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LTMP2_OK;
}

extern "C" ltmp2_status ltmp2_chi(ltmp2_ctx* c, int itau, void* chi_GG_dev, double* e_direct_tau) {
  ltmp2_status s = usable(c, itau);
  if (s) return s;
  if ((s = direct_tau(c, itau, reinterpret_cast<double*>(chi_GG_dev)))) return s;
  double v = 0.0;
  HIPCHK(c, hipMemcpyAsync(&v, c->d_scal + 2 * itau, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (!std::isfinite(v)) return fail(c, LTMP2_ENUMERIC, "non-finite direct term");
  if (e_direct_tau) *e_direct_tau = c->escale * (c->beta ? kSpinDirect * v : v);
  return LTMP2_OK;
}

extern "C" ltmp2_status ltmp2_exchange(ltmp2_ctx* c, int itau, int g_first, int g_count,
                                       double* e_exchange_tau) {
  ltmp2_status s = usable(c, itau);
  if (s) return s;
  if (g_count <= 0) {
    g_first = 0;
    g_count = c->nh;
  }
  if (g_first < 0 || g_first + g_count > c->nh) return fail(c, LTMP2_EINVAL, "G' range outside H");
  if ((s = exchange_tau(c, itau, g_first, g_count))) return s;
  if (c->beta && (s = exchange_tau(c->beta, itau, g_first, g_count)))
    return fail(c, s, "spin beta: " + c->beta->err);
  double v = 0.0, vb = 0.0;
  HIPCHK(c, hipMemcpyAsync(&v, c->d_scal + 2 * itau + 1, sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
  if (c->beta)
    HIPCHK(c, hipMemcpyAsync(&vb, c->beta->d_scal + 2 * itau + 1, sizeof(double),
                             hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->beta) v = kSpinExchange * (v + vb);
  if (!std::isfinite(v)) return fail(c, LTMP2_ENUMERIC, "non-finite exchange term");
  if (e_exchange_tau) *e_exchange_tau = c->escale * v;
  return LTMP2_OK;
}

namespace {
// least-squares line y = a + b x; returns a
double line_intercept(const std::vector<double>& x, const std::vector<double>& y) {
  const double m = double(x.size());
  double sx = 0, sy = 0, sxx = 0, sxy = 0;
  for (size_t k = 0; k < x.size(); ++k) {
    sx += x[k];
    sy += y[k];
    sxx += x[k] * x[k];
    sxy += x[k] * y[k];
  }
  const double b = (m * sxy - sx * sy) / (m * sxx - sx * sx);
  return (sy - b * sx) / m;
}
}  // namespace

// Energies of the nested auxiliary cutoffs from the per-tau bin sums (bin b
// holds the terms whose smaller sphere count is b + 1; cutoff n sums bins
// n-1 .. nb-1) and their extrapolation in eaux^(-3/2) (Eq. CutDecay).
static ltmp2_status assemble_extrapolation(ltmp2_ctx* c) {
  const int nb = c->nb;
  std::vector<double> bins(2 * size_t(c->ntau) * nb), bb;
  HIPCHK(c, hipMemcpyAsync(bins.data(), c->d_scalb, sizeof(double) * bins.size(),
                           hipMemcpyDeviceToHost, c->stream));
  if (c->beta) {
    bb.resize(bins.size());
    HIPCHK(c, hipMemcpyAsync(bb.data(), c->beta->d_scalb, sizeof(double) * bb.size(),
                             hipMemcpyDeviceToHost, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->beta)
    for (int t = 0; t < c->ntau; ++t)
      for (int q = 0; q < nb; ++q) {
        bins[(2 * size_t(t)) * nb + q] *= kSpinDirect;
        double& x = bins[(2 * size_t(t) + 1) * nb + q];
        x = kSpinExchange * (x + bb[(2 * size_t(t) + 1) * nb + q]);
      }
  for (double& x : bins) x *= c->escale;
  c->ext_d.assign(nb, 0.0);
  c->ext_x.assign(nb, 0.0);
  for (int t = 0; t < c->ntau; ++t)
    for (int n = 0; n < nb; ++n)
      for (int q = n; q < nb; ++q) {
        c->ext_d[n] += c->w[t] * bins[(2 * size_t(t)) * nb + q];
        c->ext_x[n] += c->w[t] * bins[(2 * size_t(t) + 1) * nb + q];
      }
  std::vector<double> x(nb), yt(nb);
  for (int n = 0; n < nb; ++n) {
    x[n] = std::pow(c->eaux_n[n], -1.5);
    yt[n] = c->ext_d[n] + c->ext_x[n];
  }
  c->ext_inf[0] = line_intercept(x, yt);
  c->ext_inf[1] = line_intercept(x, c->ext_d);
  c->ext_inf[2] = line_intercept(x, c->ext_x);
  for (double v : c->ext_inf)
    if (!std::isfinite(v)) return fail(c, LTMP2_ENUMERIC, "non-finite extrapolation");
  c->ext_valid = true;
  return LTMP2_OK;
}

extern "C" ltmp2_status ltmp2_get_extrapolation(const ltmp2_ctx* c, double* e_aux,
                                                double* e_direct, double* e_exchange,
                                                double* e_inf) {
  if (!c) return LTMP2_EINVAL;
  if (!c->nb || !c->ext_valid) return LTMP2_ESTATE;
  if (e_aux) std::copy(c->eaux_n.begin(), c->eaux_n.end(), e_aux);
  if (e_direct) std::copy(c->ext_d.begin(), c->ext_d.end(), e_direct);
  if (e_exchange) std::copy(c->ext_x.begin(), c->ext_x.end(), e_exchange);
  if (e_inf) std::copy(c->ext_inf, c->ext_inf + 3, e_inf);
  return LTMP2_OK;
}

extern "C" ltmp2_status ltmp2_energy(ltmp2_ctx* c, double* e_direct, double* e_exchange,
                                     double* per_tau, double* quad_err) {
  ltmp2_status s = usable(c, 0);
  if (s) return s;
  for (int t = 0; t < c->ntau; ++t) {
    if ((s = direct_tau(c, t, nullptr))) return s;
    if ((s = exchange_tau(c, t, 0, c->nh))) return s;
    if (c->beta && (s = exchange_tau(c->beta, t, 0, c->nh)))
      return fail(c, s, "spin beta: " + c->beta->err);
  }
  std::vector<double> pt(2 * size_t(c->ntau)), pb;
  HIPCHK(c, hipMemcpyAsync(pt.data(), c->d_scal, sizeof(double) * pt.size(), hipMemcpyDeviceToHost,
                           c->stream));
  if (c->beta) {
    pb.resize(pt.size());
    HIPCHK(c, hipMemcpyAsync(pb.data(), c->beta->d_scal, sizeof(double) * pb.size(),
                             hipMemcpyDeviceToHost, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->beta)  // spin-summed per-tau values of the two channels
    for (int t = 0; t < c->ntau; ++t) {
      pt[2 * t] *= kSpinDirect;
      pt[2 * t + 1] = kSpinExchange * (pt[2 * t + 1] + pb[2 * t + 1]);
    }
  for (double& x : pt) x *= c->escale;  // per unit cell of a k-point mesh
  double ed = 0.0, ex = 0.0;
  for (int t = 0; t < c->ntau; ++t) {
    ed += c->w[t] * pt[2 * t];
    ex += c->w[t] * pt[2 * t + 1];
  }
  if (!std::isfinite(ed) || !std::isfinite(ex)) return fail(c, LTMP2_ENUMERIC, "non-finite energy");
  if (c->nb && (s = assemble_extrapolation(c))) return s;
  if (e_direct) *e_direct = ed;
  if (e_exchange) *e_exchange = ex;
  if (per_tau) std::copy(pt.begin(), pt.end(), per_tau);
  if (quad_err) *quad_err = c->quad_delta;
  return LTMP2_OK;
}

extern "C" ltmp2_status ltmp2_get_quadrature(const ltmp2_ctx* c, double* tau, double* w,
                                             double* delta) {
  if (!c) return LTMP2_EINVAL;
  if (tau) std::copy(c->tau.begin(), c->tau.end(), tau);
  if (w) std::copy(c->w.begin(), c->w.end(), w);
  if (delta) *delta = c->quad_delta;
  return LTMP2_OK;
}

extern "C" ltmp2_status ltmp2_get_info(const ltmp2_ctx* c, ltmp2_info* info) {
  if (!c || !info) return LTMP2_EINVAL;
  info->n_r = c->nr;
  info->n_g = c->ng;
  info->n_h = c->nh;
  info->n_pw = c->npw;
  info->n_occ = c->no;
  info->n_vir = c->nv;
  info->n_tau = c->ntau;
  info->x_min = c->xmin;
  info->x_max = c->xmax;
  info->quad_delta = c->quad_delta;
  info->device_bytes = c->bytes;
  info->quad_flags = c->quad_flags;
  info->n_grid = c->n;
  info->g_block = c->gblock;
  info->n_spin = c->beta ? 2 : 1;
  info->n_k = c->n_kmesh;
  info->n_occ_b = c->beta ? c->beta->no : c->no;
  if (c->beta) info->device_bytes += c->beta->bytes;
  return LTMP2_OK;
}

extern "C" ltmp2_status ltmp2_aux_miller(const ltmp2_ctx* c, int32_t* out) {
  if (!c || !out) return LTMP2_EINVAL;
  std::copy(c->aux.begin(), c->aux.end(), out);
  return LTMP2_OK;
}

extern "C" ltmp2_status ltmp2_set_timing(ltmp2_ctx* c, int on) {
  if (!c) return LTMP2_EINVAL;
  for (ltmp2_ctx* x = c; x; x = x->beta) {
    collect_timing(x);
    x->timing = on != 0;
    for (int k = 0; k < 8; ++k) {
      x->stage_ms[k] = 0.0;
      x->stage_n[k] = 0;
    }
  }
  return LTMP2_OK;
}

extern "C" ltmp2_status ltmp2_get_timing(ltmp2_ctx* c, int stage, double* ms, long* launches) {
  if (!c || stage < 0 || stage > 6) return LTMP2_EINVAL;
  double t = 0.0;
  long n = 0;
  for (ltmp2_ctx* x = c; x; x = x->beta) {  // both spin channels
    collect_timing(x);
    t += x->stage_ms[stage];
    n += x->stage_n[stage];
  }
  if (ms) *ms = t;
  if (launches) *launches = n;
  return LTMP2_OK;
}

extern "C" void ltmp2_destroy(ltmp2_ctx* c) {
  if (!c) return;
  if (c->beta) {
    ltmp2_destroy(c->beta);
    c->beta = nullptr;
  }
  if (c->stream || !c->owned.empty()) (void)hipStreamSynchronize(c->stream);
  collect_timing(c);
  for (hipEvent_t e : c->pool) (void)hipEventDestroy(e);
  for (void* p : c->owned) (void)hipFree(p);
  delete c;
}

extern "C" const char* ltmp2_last_error(const ltmp2_ctx* c) {
  return c ? c->err.c_str() : g_setup_error.c_str();
}
