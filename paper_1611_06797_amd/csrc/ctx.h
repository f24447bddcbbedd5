// Internal state of an LTMP2 context (shared by the C ABI implementation
// files; not part of the public header).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/ltmp2.h"
#include "dispatch.h"

struct ltmp2_ctx {
  bool own_scratch = true;  // false: chi / chihat / P / w belong to a batch
  ltmp2_params prm{};
  std::string err;
  bool failed = false;
  hipStream_t stream = nullptr;

  // sizes
  int n = 0, nr = 0, npw = 0, nst = 0, no = 0, nv = 0, ng = 0, nh = 0, ntau = 0, npairs = 0;
  int ldbpw = 0;  // row stride of d_bpw (n_pw rounded up to a multiple of 4)
  // split-BF16x3 operands (k-octet-blocked hi / lo, see kernels_gemm3.hpp):
  // orbitals scaled by sqrt of the Laplace factors (per tau), overlap
  // densities (once), virtual basis scaled by the virtual factors (per tau)
  int kpo = 0, kpv = 0;  // occupied / virtual counts rounded up to 64
  long ldnd3 = 0, ldb3 = 0;
  void *d_psi3h = nullptr, *d_psi3l = nullptr, *d_nd3h = nullptr, *d_nd3l = nullptr;
  void *d_b3h = nullptr, *d_b3l = nullptr;
  long nrp = 0;  // padded row stride of grid arrays (multiple of 64)
  int kmax_aux = 0, kmax_orb = 0, gblock = 0;
  double omega = 0, dV = 0, mu = 0, xmin = 0, xmax = 0, quad_delta = 0;
  double xmin_force = 0, xmax_force = 0;  // > 0: quadrature range of two spin channels
  double escale = 1.0;  // energies per unit cell: 1 / N for the supercell of an N-point mesh
  int n_kmesh = 1;      // k-point mesh points per axis (1: Gamma only)
  int quad_flags = 0;
  std::string mlp_path;
  std::vector<double> eps, tau, w;
  std::vector<int> aux;  // [ng][3], H first then -H

  // device tables
  ltmp2::SphereCols sc{};
  int* d_cdesc = nullptr;
  int* d_cstart = nullptr;
  int* d_ckx = nullptr;
  int* d_wq = nullptr;
  signed char* d_wsgn = nullptr;
  int* d_gdesc = nullptr;
  int* d_pairs = nullptr;
  double* d_v = nullptr;
  double* d_fo = nullptr;  // [ntau][no]
  double* d_fv = nullptr;  // [ntau][nv]

  // device data, element type double (FP64) or float (FP32, BF16X3)
  size_t esz = sizeof(double);
  void* d_psi = nullptr;       // [nst][nrp]
  void* d_nd = nullptr;        // [nv][nh][no] complex
  void* d_bpw = nullptr;       // [nv][ldbpw] real basis of virtual coefficients
  void* d_chi = nullptr;       // [nrp][nrp]
  void* d_chihat = nullptr;    // [nh][nrp] complex
  double* d_pd = nullptr;      // [nh]
  void* d_P = nullptr;         // [gblock * no * 2][npw]
  void* d_w = nullptr;         // [gblock * no][nrp] complex
  double* d_xpart = nullptr;   // [nh][npairs]
  double* d_xrow = nullptr;    // [nh] v(G') times the row sums of d_xpart
  double* d_scal = nullptr;    // [2 * ntau + 8] device scalars
  // internal cutoff extrapolation: nb nested auxiliary spheres (0 = off)
  int nb = 0;
  double alpha = 1.05;
  std::vector<double> eaux_n;    // [nb] cutoffs eaux / alpha^(n-1)
  signed char* d_shell = nullptr;  // [ng] spheres containing each vector
  double* d_pdb = nullptr;     // [nh][nb] direct-term bins per G'
  double* d_xb = nullptr;      // [nh][npairs][nb] exchange bins per (G', pair)
  double* d_xrowb = nullptr;   // [nh][nb]
  double* d_scalb = nullptr;   // [ntau][2][nb] per-tau bin sums (E_d, E_x)
  bool ext_valid = false;
  std::vector<double> ext_d, ext_x;  // [nb] energies per cutoff (last ltmp2_energy)
  double ext_inf[3] = {0, 0, 0};

  // spin-unrestricted cells: the second spin channel (owned; shares the
  // quadrature and the chi buffer of this context, which holds spin alpha)
  ltmp2_ctx* beta = nullptr;
  std::vector<void*> owned;
  size_t bytes = 0;

  // optional per-stage event timing
  bool timing = false;
  struct Mark {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<Mark> marks;
  std::vector<hipEvent_t> pool;
  double stage_ms[8] = {0};
  long stage_n[8] = {0};
};

namespace ltmp2 {
// Host drivers of one Laplace point (ltmp2.hip); values land in d_scal.
ltmp2_status run_direct(ltmp2_ctx* c, int itau, double* chi_out);
ltmp2_status run_exchange(ltmp2_ctx* c, int itau, int g_first, int g_count);
// Pieces of run_exchange used by batched execution.
ltmp2_status exchange_block_prepare(ltmp2_ctx* c, int itau, int g0, int gb);
ltmp2_status exchange_reduce(ltmp2_ctx* c, int itau, int g_first, int g_count);
ltmp2_status setup_cell(ltmp2_ctx* c, const int32_t* miller, const double* eps,
                        const double* coeff, const double* tau, const double* w);
// Validation of a cell's inputs; *use receives the coefficients to pass on
// (the caller's, or their real form held in `store`).
ltmp2_status validate_inputs(const ltmp2_params* p, const int32_t* miller, const double* eps,
                             const double* coeff, const double* tau, const double* w,
                             std::vector<double>& store, const double** use);
const std::string& setup_error();
void set_setup_error(const std::string& msg);
// Orbitals real up to a phase (or degenerate blocks with a real basis) to
// real form (real_orbitals.cpp); `out` stays empty if nothing changes.
ltmp2_status unfold_kmesh(int n_k, int n_bands, int n_occ, const int32_t* n_pw_k,
                          const int32_t* miller, const double* eps, const double* coeff,
                          std::vector<int32_t>& miller_s, std::vector<double>& eps_s,
                          std::vector<double>& coeff_s, std::string& err);
ltmp2_status real_orbitals(int npw, const int32_t* miller, int nst, const double* eps, int nocc,
                           const double* coeff, std::vector<double>& out, bool* changed,
                           std::string& err);
}  // namespace ltmp2
