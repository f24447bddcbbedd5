// Registry of the compiled grid sizes and the per-tau reduction kernels.
#include <hip/hip_runtime.h>

#include "dispatch.h"
#include "kernels_gemm.hpp"

#ifndef LTMP2_GRID_LIST
#error "LTMP2_GRID_LIST must list the compiled grid sizes as X(n) X(m) ..."
#endif

namespace ltmp2 {

#define X(n) extern const GridOps kGridOps_##n;
LTMP2_GRID_LIST
#undef X

const GridOps* grid_ops(int n) {
  switch (n) {
#define X(k) \
  case k:    \
    return &kGridOps_##k;
    LTMP2_GRID_LIST
#undef X
    default:
      return nullptr;
  }
}

bool grid_supported(int n) { return grid_ops(n) != nullptr; }

std::vector<int> supported_grids() {
  std::vector<int> g;
#define X(k) g.push_back(k);
  LTMP2_GRID_LIST
#undef X
  return g;
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
