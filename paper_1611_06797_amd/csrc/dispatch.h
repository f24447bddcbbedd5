// Launchers of the grid-size-templated transform kernels, one translation
// unit per compiled grid size n (grid_kernels.hip built with -DLTMP2_N=n).
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/ltmp2.h"
#include "kernels_fft.hpp"
#include "modes.h"

namespace ltmp2 {

// Largest auxiliary set a transform kernel can hold in registers.
constexpr int kMaxOpt = 17;
inline int max_outputs() { return kMaxOpt * kThreads; }

bool grid_supported(int n);
std::vector<int> supported_grids();

template <class T>
struct GridOps {
  ltmp2_status (*orbitals)(const cplx<double>* coef, int nstates, int npw, SphereCols sc,
                           double scale, T* psi, long ld, hipStream_t st);
  ltmp2_status (*overlap)(const T* psi, long ld, int no, int nv, const int* gdesc, int nh,
                          int kmax, double dV, cplx<T>* nd, hipStream_t st);
  ltmp2_status (*chi_rows)(const T* chi, long ld, int nr, const int* gdesc, int nh, int kmax,
                           double dV, cplx<T>* chihat, hipStream_t st);
  ltmp2_status (*chi_cols)(const cplx<T>* chihat, long ld, const int* gdesc, int ng, int nh,
                           const double* v, int kmax, double dV, double* pd,
                           cplx<double>* chi_out, ShellBins bins, hipStream_t st);
  ltmp2_status (*wstates)(const T* P, int npw, const int* wq, const signed char* wsgn,
                          SphereCols sc, int nitems, double scale, cplx<T>* w, long ld,
                          hipStream_t st);
  // shell / xbins / nb / g0: optional split by auxiliary cutoff shell (PairCell)
  ltmp2_status (*pair)(const T* psi, long ld, const cplx<T>* w, int no, const int* pairs,
                       int npairs, int gb, const int* gdesc, int ng, const double* v, int kmax,
                       double dV2, double* xpart, const signed char* shell, double* xbins,
                       int nb, int g0, hipStream_t st);
  // persistent multi-cell pair launch (device arrays cells[ncells], prefix[ncells + 1]);
  // all cells share the kept-set instance kfix (pair_kept)
  ltmp2_status (*pair_multi)(const PairCell* cells, const long* prefix, int ncells, int ng_max,
                             int kmax_max, int kfix, int sx, int nblocks, hipStream_t st);
  // Hartree-like direct term of one block of outer G' from h (k_hartree)
  ltmp2_status (*hartree)(const cplx<T>* h, long ld, const int* gdesc, int ng, const double* v,
                          int kmax, double dV, int g0, int gb, double* pdh, hipStream_t st);
  int (*pair_sx_max)(int kmax);
  // kept-set instance of the pair kernels for a cell's kmax (or -1: runtime form)
  int (*pair_kept)(int kmax);
};

template <class T>
const GridOps<T>* grid_ops(int n);

// Matrix-core contractions (instantiated in registry.hip, see kernels_gemm.hpp).
// launch_gf_chi covers the symmetric n x n block (n a multiple of 64) with
// upper-triangular tile pairs.
template <int MODE>
ltmp2_status launch_gf_chi(const void* psi, long ld, int no, int nv, const double* fo,
                           const double* fv, void* chi, long ldc, long n, int accumulate,
                           hipStream_t st);
template <int MODE>
ltmp2_status launch_gemm_kmajor(const void* A, long lda, const void* B, long ldb, void* C,
                                long ldc, int M, int N, int K, const double* sk,
                                const double* rowscale, int rdiv, int rmod, hipStream_t st);

// Split-BF16x3 path (kernels_gemm3.hpp): operand splitting into the
// k-octet-blocked hi / lo layout, the Green's-function tiles, and the
// general product.
ltmp2_status launch_split3(const float* src, long lds, int K, int Kpad, int M, long ldo,
                           const double* sk, int mode, void* hi, void* lo, long o0,
                           hipStream_t st);
ltmp2_status launch_chi3(const void* hi, const void* lo, long ld, int kpo, int kpv, long n,
                         float* chi, long ldc, int accumulate, hipStream_t st);
ltmp2_status launch_mm3(const void* ahi, const void* alo, long lda, long am0, const void* bhi,
                        const void* blo, long ldb, float* C, long ldc, int M, int N, int Kpad,
                        const double* rowscale, int rdiv, int rmod, hipStream_t st);

// h^{(G')}(r) = sum_i psi_i(r) w_i^{(G')}(r) for a block of gb outer vectors
template <class T>
ltmp2_status launch_hsum(const T* psi, long ld, const cplx<T>* w, int no, long nr, int gb,
                         cplx<T>* h, hipStream_t st);

// float -> double copy (diagnostic outputs of FP32 contexts)
__global__ void k_widen(const float* in, double* out, long n);

// Deterministic single-block reductions of the per-G' partial sums.
//   E_d(tau) = -4 sum_{g in H} pd[g]        (pd includes v(G'); G' and -G')
__global__ void k_reduce_direct(const double* pd, int nh, double* out);
//   E_x(tau) = 2 sum_{g in range} v[g] sum_p xpart[g][p]
__global__ void k_reduce_xrows(const double* xpart, int g0, int npairs, const double* v,
                               double* xrow);
__global__ void k_reduce_exchange(const double* xrow, int g0, int gcount, double* out);
// The same three reductions per auxiliary cutoff shell bin (ShellBins):
//   out[b] = -4 sum_g pdb[g][b];  xrowb[g][b] = v[g] sum_p xb[g][p][b];
//   out[b] = 2 sum_{g in range} xrowb[g][b]
__global__ void k_reduce_direct_bins(const double* pdb, int nh, int nb, double* out);
__global__ void k_reduce_xrows_bins(const double* xb, int g0, int npairs, int nb, const double* v,
                                    double* xrowb);
__global__ void k_reduce_exchange_bins(const double* xrowb, int g0, int gcount, int nb,
                                       double* out);

}  // namespace ltmp2
