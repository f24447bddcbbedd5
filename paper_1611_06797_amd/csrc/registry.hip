// Registry of the compiled grid sizes and the per-tau reduction kernels.
#include <hip/hip_runtime.h>

#include "dispatch.h"
#include "kernels_gemm3.hpp"
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
                           const double* fv, void* chi, long ldc, long n, int accumulate,
                           hipStream_t st) {
  using T = typename Mma<MODE>::T;
  if (n % 64 != 0) return LTMP2_EINVAL;
  const long t = n / 64;
  hipLaunchKernelGGL(k_gf_chi<MODE>, dim3(unsigned(t * (t + 1) / 2)), dim3(256), 0, st,
                     static_cast<const T*>(psi), ld, no, nv, fo, fv, static_cast<T*>(chi), ldc,
                     accumulate);
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

ltmp2_status launch_split3(const float* src, long lds, int K, int Kpad, int M, long ldo,
                           const double* sk, int mode, void* hi, void* lo, long o0,
                           hipStream_t st) {
  if (Kpad % 64 != 0 || K > Kpad || M > ldo) return LTMP2_EINVAL;
  const long items = long(Kpad / 8) * M;
  if (items == 0) return LTMP2_OK;
  hipLaunchKernelGGL(k_split3, dim3(unsigned((items + 255) / 256)), dim3(256), 0, st, src, lds, K,
                     Kpad, M, ldo, sk, mode, static_cast<__bf16*>(hi), static_cast<__bf16*>(lo),
                     o0);
  return hipGetLastError() == hipSuccess ? LTMP2_OK : LTMP2_EDEVICE;
}

ltmp2_status launch_chi3(const void* hi, const void* lo, long ld, int kpo, int kpv, long n,
                         float* chi, long ldc, int accumulate, hipStream_t st) {
  if (n % 128 != 0 || ld < n || kpo % 64 != 0 || kpv % 64 != 0) return LTMP2_EINVAL;
  const int t = int(n / 128), ts = (t + 7) / 8;
  const long nsuper = long(ts) * (ts + 1) / 2;
  const long blocks = (nsuper + 7) / 8 * 512;
  Op3 op{static_cast<const __bf16*>(hi), static_cast<const __bf16*>(lo), ld};
  hipLaunchKernelGGL(k_chi3, dim3(unsigned(blocks)), dim3(256), 0, st, op, kpo, kpv, t, chi, ldc,
                     accumulate);
  return hipGetLastError() == hipSuccess ? LTMP2_OK : LTMP2_EDEVICE;
}

ltmp2_status launch_mm3(const void* ahi, const void* alo, long lda, long am0, const void* bhi,
                        const void* blo, long ldb, float* C, long ldc, int M, int N, int Kpad,
                        const double* rowscale, int rdiv, int rmod, hipStream_t st) {
  if (M <= 0 || N <= 0) return LTMP2_OK;
  if (Kpad % 64 != 0 || am0 + (M + 127) / 128 * 128 > lda || (N + 127) / 128 * 128 > ldb)
    return LTMP2_EINVAL;
  const long total = long((M + 127) / 128) * ((N + 127) / 128);
  const long blocks = (total + 7) / 8 * 8;
  Op3 a{static_cast<const __bf16*>(ahi), static_cast<const __bf16*>(alo), lda};
  Op3 b{static_cast<const __bf16*>(bhi), static_cast<const __bf16*>(blo), ldb};
  hipLaunchKernelGGL(k_mm3, dim3(unsigned(blocks)), dim3(256), 0, st, a, am0, b, C, ldc, M, N,
                     Kpad, rowscale, rdiv, rmod);
  return hipGetLastError() == hipSuccess ? LTMP2_OK : LTMP2_EDEVICE;
}

template ltmp2_status launch_gf_chi<kF64>(const void*, long, int, int, const double*, const double*,
                                          void*, long, long, int, hipStream_t);
template ltmp2_status launch_gf_chi<kF32>(const void*, long, int, int, const double*, const double*,
                                          void*, long, long, int, hipStream_t);
template ltmp2_status launch_gf_chi<kBF16x3>(const void*, long, int, int, const double*,
                                          const double*, void*, long, long, int, hipStream_t);
template ltmp2_status launch_gemm_kmajor<kF64>(const void*, long, const void*, long, void*, long,
                                               int, int, int, const double*, const double*, int,
                                               int, hipStream_t);
template ltmp2_status launch_gemm_kmajor<kF32>(const void*, long, const void*, long, void*, long,
                                               int, int, int, const double*, const double*, int,
                                               int, hipStream_t);
template ltmp2_status launch_gemm_kmajor<kBF16x3>(const void*, long, const void*, long, void*,
                                                  long, int, int, int, const double*,
                                                  const double*, int, int, hipStream_t);

template <class T>
ltmp2_status launch_hsum(const T* psi, long ld, const cplx<T>* w, int no, long nr, int gb,
                         cplx<T>* h, hipStream_t st) {
  if (gb <= 0) return LTMP2_OK;
  hipLaunchKernelGGL(k_hsum<T>, dim3(unsigned((nr + 255) / 256), unsigned(gb)), dim3(256), 0, st,
                     psi, ld, w, no, nr, h);
  return hipGetLastError() == hipSuccess ? LTMP2_OK : LTMP2_EDEVICE;
}
template ltmp2_status launch_hsum<double>(const double*, long, const cplx<double>*, int, long,
                                          int, cplx<double>*, hipStream_t);
template ltmp2_status launch_hsum<float>(const float*, long, const cplx<float>*, int, long, int,
                                         cplx<float>*, hipStream_t);

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

// one block per G': xrow[g] = v(G') sum_p xpart[g][p] (fixed-order block sum)
__global__ void k_reduce_xrows(const double* xpart, int g0, int npairs, const double* v,
                               double* xrow) {
  __shared__ double red[4];
  const int g = g0 + blockIdx.x;
  const double* row = xpart + size_t(g) * npairs;
  double s = 0.0;
  for (int p = threadIdx.x; p < npairs; p += blockDim.x) s += row[p];
  s = block_sum(s, red);
  if (threadIdx.x == 0) xrow[g] = v[g] * s;
}

__global__ void k_reduce_exchange(const double* xrow, int g0, int gcount, double* out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int g = g0 + threadIdx.x; g < g0 + gcount; g += blockDim.x) s += xrow[g];
  s = block_sum(s, red);
  if (threadIdx.x == 0) out[0] = 2.0 * s;
}

__global__ void k_reduce_direct_bins(const double* pdb, int nh, int nb, double* out) {
  __shared__ double red[4 * kMaxShells];
  double sb[kMaxShells] = {};
  for (int g = threadIdx.x; g < nh; g += blockDim.x)
    for (int b = 0; b < nb; ++b) bin_add(sb, b, pdb[long(g) * nb + b]);
  block_sum_bins(sb, red);
  if (threadIdx.x == 0)
    for (int b = 0; b < nb; ++b) out[b] = -4.0 * sb[b];
}

// one block per G': xrowb[g][b] = v(G') sum_p xb[g][p][b]
__global__ void k_reduce_xrows_bins(const double* xb, int g0, int npairs, int nb, const double* v,
                                    double* xrowb) {
  __shared__ double red[4 * kMaxShells];
  const int g = g0 + blockIdx.x;
  const double* row = xb + size_t(g) * npairs * nb;
  double sb[kMaxShells] = {};
  for (int p = threadIdx.x; p < npairs; p += blockDim.x)
    for (int b = 0; b < nb; ++b) bin_add(sb, b, row[long(p) * nb + b]);
  block_sum_bins(sb, red);
  if (threadIdx.x == 0)
    for (int b = 0; b < nb; ++b) xrowb[long(g) * nb + b] = v[g] * sb[b];
}

__global__ void k_reduce_exchange_bins(const double* xrowb, int g0, int gcount, int nb,
                                       double* out) {
  __shared__ double red[4 * kMaxShells];
  double sb[kMaxShells] = {};
  for (int g = g0 + threadIdx.x; g < g0 + gcount; g += blockDim.x)
    for (int b = 0; b < nb; ++b) bin_add(sb, b, xrowb[long(g) * nb + b]);
  block_sum_bins(sb, red);
  if (threadIdx.x == 0)
    for (int b = 0; b < nb; ++b) out[b] = 2.0 * sb[b];
}

}  // namespace ltmp2
