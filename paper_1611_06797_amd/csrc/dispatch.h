// Launchers of the grid-size-templated transform kernels, one translation
// unit per compiled grid size n (grid_kernels.hip built with -DLTMP2_N=n).
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/ltmp2.h"
#include "kernels_fft.hpp"

namespace ltmp2 {

// Largest auxiliary set a transform kernel can hold in registers.
constexpr int kMaxOpt = 17;
inline int max_outputs() { return kMaxOpt * kThreads; }

bool grid_supported(int n);
std::vector<int> supported_grids();

struct GridOps {
  ltmp2_status (*orbitals)(const cplx<double>* coef, int nstates, int npw, SphereCols sc, double scale,
                           double* psi, long ld, hipStream_t st);
  ltmp2_status (*overlap)(const double* psi, long ld, int no, int nv, const int* gdesc, int nh,
                          int kmax, double dV, cplx<double>* nd, hipStream_t st);
  ltmp2_status (*chi_rows)(const double* chi, long ld, int nr, const int* gdesc, int nh, int kmax,
                           double dV, cplx<double>* chihat, hipStream_t st);
  ltmp2_status (*chi_cols)(const cplx<double>* chihat, long ld, const int* gdesc, int ng, int nh,
                           const double* v, int kmax, double dV, double* pd,
                           cplx<double>* chi_out, hipStream_t st);
  ltmp2_status (*wstates)(const double* P, int npw, const int* wq, const signed char* wsgn,
                          SphereCols sc, int nitems, double scale, cplx<double>* w, long ld,
                          hipStream_t st);
  ltmp2_status (*pair)(const double* psi, long ld, const cplx<double>* w, int no,
                       const int* pairs, int npairs, int gb, const int* gdesc, int ng,
                       const double* v, int kmax, double dV2, double* xpart, hipStream_t st);
};

const GridOps* grid_ops(int n);

// Convenience wrappers used by the host driver.
#define LTMP2_OPS_OR_FAIL(n)              \
  const GridOps* ops_ = grid_ops(n);      \
  if (!ops_) return LTMP2_EINVAL;

inline ltmp2_status launch_orbitals(int n, const cplx<double>* coef, int nstates, int npw,
                                    SphereCols sc, double scale, double* psi, long ld,
                                    hipStream_t st) {
  LTMP2_OPS_OR_FAIL(n) return ops_->orbitals(coef, nstates, npw, sc, scale, psi, ld, st);
}
inline ltmp2_status launch_overlap(int n, const double* psi, long ld, int no, int nv,
                                   const int* gdesc, int nh, int kmax, double dV,
                                   cplx<double>* nd, hipStream_t st) {
  LTMP2_OPS_OR_FAIL(n) return ops_->overlap(psi, ld, no, nv, gdesc, nh, kmax, dV, nd, st);
}
inline ltmp2_status launch_chi_rows(int n, const double* chi, long ld, int nr, const int* gdesc,
                                    int nh, int kmax, double dV, cplx<double>* chihat,
                                    hipStream_t st) {
  LTMP2_OPS_OR_FAIL(n) return ops_->chi_rows(chi, ld, nr, gdesc, nh, kmax, dV, chihat, st);
}
inline ltmp2_status launch_chi_cols(int n, const cplx<double>* chihat, long ld, const int* gdesc,
                                    int ng, int nh, const double* v, int kmax, double dV,
                                    double* pd, cplx<double>* chi_out, hipStream_t st) {
  LTMP2_OPS_OR_FAIL(n) return ops_->chi_cols(chihat, ld, gdesc, ng, nh, v, kmax, dV, pd, chi_out, st);
}
inline ltmp2_status launch_wstates(int n, const double* P, int npw, const int* wq,
                                   const signed char* wsgn, SphereCols sc, int nitems,
                                   double scale, cplx<double>* w, long ld, hipStream_t st) {
  LTMP2_OPS_OR_FAIL(n) return ops_->wstates(P, npw, wq, wsgn, sc, nitems, scale, w, ld, st);
}
inline ltmp2_status launch_pair(int n, const double* psi, long ld, const cplx<double>* w, int no,
                                const int* pairs, int npairs, int gb, const int* gdesc, int ng,
                                const double* v, int kmax, double dV2, double* xpart,
                                hipStream_t st) {
  LTMP2_OPS_OR_FAIL(n) return ops_->pair(psi, ld, w, no, pairs, npairs, gb, gdesc, ng, v, kmax,
                                         dV2, xpart, st);
}

// Matrix-core contractions (defined in registry.hip, see kernels_gemm.hpp).
__global__ void k_gf_chi(const double* psi, long ld, int no, int nv, const double* fo,
                         const double* fv, double* chi, long ldc);
__global__ void k_gemm_kmajor(const double* A, long lda, const double* B, long ldb, double* C,
                              long ldc, int M, int N, int K, const double* sk,
                              const double* rowscale, int rdiv, int rmod);

// Deterministic single-block reductions of the per-G' partial sums.
//   E_d(tau) = -4 sum_{g in H} pd[g]        (pd includes v(G'); G' and -G')
__global__ void k_reduce_direct(const double* pd, int nh, double* out);
//   E_x(tau) = 2 sum_{g in range} v[g] sum_p xpart[g][p]
__global__ void k_reduce_exchange(const double* xpart, int g0, int gcount, int npairs,
                                  const double* v, double* out);

}  // namespace ltmp2
