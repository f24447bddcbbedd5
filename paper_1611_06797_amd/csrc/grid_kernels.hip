// Transform kernels instantiated for one grid size n = LTMP2_N.
#include <hip/hip_runtime.h>

#include "dispatch.h"

#ifndef LTMP2_N
#error "LTMP2_N must be defined"
#endif

namespace ltmp2 {
namespace {

constexpr int N = LTMP2_N;
constexpr size_t kLdsCap = 150 * 1024;

int choose_sx(int nk) {
  int sx = std::min(N, 8);
  while (sx > 1 && slab_lds_bytes<double>(N, nk, sx) > kLdsCap) --sx;
  return sx;
}

template <class K>
ltmp2_status launch(K kern, dim3 grid, size_t lds, hipStream_t st, auto... args) {
  if (lds > kLdsCap) return LTMP2_EINVAL;
  if (grid.x == 0 || grid.y == 0) return LTMP2_OK;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  if (e != hipSuccess) return LTMP2_EDEVICE;
  hipLaunchKernelGGL(kern, grid, dim3(kThreads), lds, st, args...);
  return hipGetLastError() == hipSuccess ? LTMP2_OK : LTMP2_EDEVICE;
}

template <template <int> class F>
ltmp2_status by_opt(int nout, auto&&... a) {
  const int need = (nout + kThreads - 1) / kThreads;
  if (need <= 1) return F<1>::go(a...);
  if (need <= 3) return F<3>::go(a...);
  if (need <= 9) return F<9>::go(a...);
  if (need <= 17) return F<17>::go(a...);
  return LTMP2_EINVAL;
}

ltmp2_status orbitals(const cplx<double>* coef, int nstates, int npw, SphereCols sc, double scale,
                      double* psi, long ld, hipStream_t st) {
  const int nk = 2 * sc.kmax + 1, sx = choose_sx(nk);
  return launch(k_orbitals<double, N>, dim3(nstates), slab_lds_bytes<double>(N, nk, sx), st, coef, npw,
                sc, sx, scale, psi, ld);
}

template <int OPT>
struct OverlapF {
  static ltmp2_status go(const double* psi, long ld, int no, int nv, const int* gdesc, int nh,
                         int kmax, double dV, cplx<double>* nd, hipStream_t st) {
    constexpr int NF = 4;
    const int nk = 2 * kmax + 1, sx = choose_sx(nk);
    return launch(k_overlap<double, N, NF, OPT>, dim3((no + NF - 1) / NF, nv),
                  slab_lds_bytes<double>(N, nk, sx), st, psi, ld, no, gdesc, nh, kmax, sx, dV, nd);
  }
};
ltmp2_status overlap(const double* psi, long ld, int no, int nv, const int* gdesc, int nh,
                     int kmax, double dV, cplx<double>* nd, hipStream_t st) {
  return by_opt<OverlapF>(nh, psi, ld, no, nv, gdesc, nh, kmax, dV, nd, st);
}

template <int OPT>
struct ChiRowsF {
  static ltmp2_status go(const double* chi, long ld, int nr, const int* gdesc, int nh, int kmax,
                         double dV, cplx<double>* chihat, hipStream_t st) {
    constexpr int NF = 2;
    const int nk = 2 * kmax + 1, sx = choose_sx(nk);
    return launch(k_chi_rows<double, N, NF, OPT>, dim3((nr + NF - 1) / NF),
                  slab_lds_bytes<double>(N, nk, sx), st, chi, ld, nr, gdesc, nh, kmax, sx, dV,
                  chihat);
  }
};
ltmp2_status chi_rows(const double* chi, long ld, int nr, const int* gdesc, int nh, int kmax,
                      double dV, cplx<double>* chihat, hipStream_t st) {
  return by_opt<ChiRowsF>(nh, chi, ld, nr, gdesc, nh, kmax, dV, chihat, st);
}

template <int OPT>
struct ChiColsF {
  static ltmp2_status go(const cplx<double>* chihat, long ld, const int* gdesc, int ng, int nh,
                         const double* v, int kmax, double dV, double* pd, cplx<double>* chi_out,
                         hipStream_t st) {
    const int nk = 2 * kmax + 1, sx = choose_sx(nk);
    return launch(k_chi_cols<double, N, OPT>, dim3(nh), slab_lds_bytes<double>(N, nk, sx), st,
                  chihat, ld, gdesc, ng, nh, v, kmax, sx, dV, pd, chi_out);
  }
};
ltmp2_status chi_cols(const cplx<double>* chihat, long ld, const int* gdesc, int ng, int nh,
                      const double* v, int kmax, double dV, double* pd, cplx<double>* chi_out,
                      hipStream_t st) {
  return by_opt<ChiColsF>(ng, chihat, ld, gdesc, ng, nh, v, kmax, dV, pd, chi_out, st);
}

ltmp2_status wstates(const double* P, int npw, const int* wq, const signed char* wsgn,
                     SphereCols sc, int nitems, double scale, cplx<double>* w, long ld,
                     hipStream_t st) {
  const int nk = 2 * sc.kmax + 1, sx = choose_sx(nk);
  return launch(k_wstates<double, N>, dim3(nitems), slab_lds_bytes<double>(N, nk, sx), st, P, npw,
                wq, wsgn, sc, sx, scale, w, ld);
}

template <int OPT>
struct PairF {
  static ltmp2_status go(const double* psi, long ld, const cplx<double>* w, int no,
                         const int* pairs, int npairs, int gb, const int* gdesc, int ng,
                         const double* v, int kmax, double dV2, double* xpart, hipStream_t st) {
    const int nk = 2 * kmax + 1, sx = choose_sx(nk);
    return launch(k_pair<double, N, OPT>, dim3(npairs, gb), slab_lds_bytes<double>(N, nk, sx), st,
                  psi, ld, w, no, pairs, npairs, gdesc, ng, v, kmax, sx, dV2, xpart);
  }
};
ltmp2_status pair(const double* psi, long ld, const cplx<double>* w, int no, const int* pairs,
                  int npairs, int gb, const int* gdesc, int ng, const double* v, int kmax,
                  double dV2, double* xpart, hipStream_t st) {
  return by_opt<PairF>(ng, psi, ld, w, no, pairs, npairs, gb, gdesc, ng, v, kmax, dV2, xpart, st);
}

}  // namespace

#define LTMP2_CAT2(a, b) a##b
#define LTMP2_CAT(a, b) LTMP2_CAT2(a, b)
#if !defined(__HIP_DEVICE_COMPILE__)
extern const GridOps LTMP2_CAT(kGridOps_, LTMP2_N);
const GridOps LTMP2_CAT(kGridOps_, LTMP2_N) = {orbitals, overlap, chi_rows, chi_cols, wstates, pair};
#endif

}  // namespace ltmp2
