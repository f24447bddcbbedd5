// Registry of the compiled grid sizes and the per-tau reduction kernels.
#include <hip/hip_runtime.h>

#include "dispatch.h"
#include "kernels_gemm.hpp"

#ifndef LTMP2_GRID_LIST
#error "LTMP2_GRID_LIST must list the compiled grid sizes as X(n) X(m) ..."
#endif

namespace ltmp2 {

#define X(n)                                \
  extern const GridOps<double> kGridOpsD_##n; \
  extern const GridOps<float> kGridOpsF_##n;
LTMP2_GRID_LIST
#undef X

template <>
const GridOps<double>* grid_ops<double>(int n) {
  switch (n) {
#define X(k) \
  case k:    \
    return &kGridOpsD_##k;
    LTMP2_GRID_LIST
#undef X
    default:
      return nullptr;
  }
}

template <>
const GridOps<float>* grid_ops<float>(int n) {
  switch (n) {
#define X(k) \
  case k:    \
    return &kGridOpsF_##k;
    LTMP2_GRID_LIST
#undef X
    default:
      return nullptr;
  }
}

bool grid_supported(int n) { return grid_ops<double>(n) != nullptr; }

std::vector<int> supported_grids() {
  std::vector<int> g;
#define X(k) g.push_back(k);
  LTMP2_GRID_LIST
#undef X
  return g;
}

template <int MODE>
ltmp2_status launch_gf_chi(const void* psi, long ld, int no, int nv, const double* fo,
                           const double* fv, void* chi, long ldc, long ntiles, hipStream_t st) {
  using T = typename Mma<MODE>::T;
  hipLaunchKernelGGL(k_gf_chi<MODE>, dim3(unsigned(ntiles)), dim3(256), 0, st,
                     static_cast<const T*>(psi), ld, no, nv, fo, fv, static_cast<T*>(chi), ldc);
  return hipGetLastError() == hipSuccess ? LTMP2_OK : LTMP2_EDEVICE;
}

template <int MODE>
ltmp2_status launch_gemm_kmajor(const void* A, long lda, const void* B, long ldb, void* C,
                                long ldc, int M, int N, int K, const double* sk,
                                const double* rowscale, int rdiv, int rmod, hipStream_t st) {
  using T = typename Mma<MODE>::T;
  if (M <= 0 || N <= 0) return LTMP2_OK;
  hipLaunchKernelGGL(k_gemm_kmajor<MODE>, dim3((N + 63) / 64, (M + 63) / 64), dim3(256), 0, st,
                     static_cast<const T*>(A), lda, static_cast<const T*>(B), ldb,
                     static_cast<T*>(C), ldc, M, N, K, sk, rowscale, rdiv, rmod);
  return hipGetLastError() == hipSuccess ? LTMP2_OK : LTMP2_EDEVICE;
}

template ltmp2_status launch_gf_chi<kF64>(const void*, long, int, int, const double*, const double*,
                                          void*, long, long, hipStream_t);
template ltmp2_status launch_gf_chi<kF32>(const void*, long, int, int, const double*, const double*,
                                          void*, long, long, hipStream_t);
template ltmp2_status launch_gf_chi<kBF16x3>(const void*, long, int, int, const double*,
                                             const double*, void*, long, long, hipStream_t);
template ltmp2_status launch_gemm_kmajor<kF64>(const void*, long, const void*, long, void*, long,
                                               int, int, int, const double*, const double*, int,
                                               int, hipStream_t);
template ltmp2_status launch_gemm_kmajor<kF32>(const void*, long, const void*, long, void*, long,
                                               int, int, int, const double*, const double*, int,
                                               int, hipStream_t);

__global__ void k_widen(const float* in, double* out, long n) {
  const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[i];
}

__global__ void k_reduce_direct(const double* pd, int nh, double* out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int g = threadIdx.x; g < nh; g += blockDim.x) s += pd[g];
  s = block_sum(s, red);
  if (threadIdx.x == 0) out[0] = -4.0 * s;
}

__global__ void k_reduce_exchange(const double* xpart, int g0, int gcount, int npairs,
                                  const double* v, double* out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int g = g0 + threadIdx.x; g < g0 + gcount; g += blockDim.x) {
    const double* row = xpart + size_t(g) * npairs;
    double r = 0.0;
    for (int p = 0; p < npairs; ++p) r += row[p];
    s += v[g] * r;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) out[0] = 2.0 * s;
}

}  // namespace ltmp2
