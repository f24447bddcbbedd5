// Transform kernels instantiated for one grid size n = LTMP2_N.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>

#include "dispatch.h"

#ifndef LTMP2_N
#error "LTMP2_N must be defined"
#endif

namespace ltmp2 {
namespace {

constexpr int N = LTMP2_N;
constexpr size_t kLdsCap = 150 * 1024;
constexpr size_t kLdsHalf = 78 * 1024;
constexpr size_t kLdsQuarter = 39 * 1024;

template <class T>
int choose_sx(int nk, int cap = 10) {
  int sx = slab_tile_at_most(N, cap);
  while (sx > 1 && inv_lds_bytes<T>(N, nk, sx) > kLdsCap) sx = slab_tile_at_most(N, sx - 1);
  return sx;
}

// The same for the forward transforms (z-pass buffer only, see fwd_lds).
template <class T>
int choose_sx_fwd(int nk, int cap = 10) {
  int sx = slab_tile_at_most(N, cap);
  while (sx > 1 && fwd_lds_bytes<T>(N, nk, sx) > kLdsCap) sx = slab_tile_at_most(N, sx - 1);
  return sx;
}

// Dynamic shared memory above the default needs a per-kernel attribute; set
// it once per kernel (never while a stream is being captured into a graph).
bool ensure_lds(const void* kern, size_t lds) {
  static std::mutex mu;
  static std::map<const void*, size_t> done;
  std::lock_guard<std::mutex> lk(mu);
  auto it = done.find(kern);
  if (it != done.end() && it->second >= lds) return true;
  if (hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)) !=
      hipSuccess)
    return false;
  done[kern] = lds;
  return true;
}

template <class K>
ltmp2_status launch_nt(K kern, dim3 grid, int nt, size_t lds, hipStream_t st, auto... args) {
  if (lds > kLdsCap) return LTMP2_EINVAL;
  if (grid.x == 0 || grid.y == 0) return LTMP2_OK;
  if (!ensure_lds(reinterpret_cast<const void*>(kern), lds)) return LTMP2_EDEVICE;
  hipLaunchKernelGGL(kern, grid, dim3(nt), lds, st, args...);
  return hipGetLastError() == hipSuccess ? LTMP2_OK : LTMP2_EDEVICE;
}

template <class K>
ltmp2_status launch(K kern, dim3 grid, size_t lds, hipStream_t st, auto... args) {
  return launch_nt(kern, grid, kThreads, lds, st, args...);
}

// FP32 pair transforms with more than 9 outputs per thread: on grids whose
// auxiliary window allows them (n >= 30) 256-thread workgroups with up to 17
// outputs each, held to two waves per SIMD by their launch bounds, two
// workgroups per CU (36 grid: 118 ns per item against 135 ns for the
// 512-thread joint form below, stand-alone timing); above 17 x 256 outputs
// the 512-thread form with at most 9 each.  (FP64 keeps 256 threads.)
constexpr int kWideNT = 512, kWideOpt = 9;
// The wide form transforms both fields of an item side by side in two slab
// buffers (forward_pruned_joint): on the 36 grid with 12-plane slabs that is
// 864 z lines, 504 y rows and 882 columns per slab group for the 512 threads
// (one field at a time: 432, 252 and 441), with half the barriers; one
// workgroup per CU either way (the registers bind first).  Measured 8 %
// faster than single-field 18-plane slabs, 23 % faster than single-field
// 12-plane slabs.
constexpr int kNarrowNT = 192;

template <template <int> class F>
ltmp2_status by_opt(int nout, auto&&... a) {
  const int need = (nout + kThreads - 1) / kThreads;
  if (need <= 1) return F<1>::go(a...);
  if (need <= 3) return F<3>::go(a...);
  if (need <= 9) return F<9>::go(a...);
  if (need <= 17) return F<17>::go(a...);
  return LTMP2_EINVAL;
}

template <class T>
ltmp2_status orbitals(const cplx<double>* coef, int nstates, int npw, SphereCols sc, double scale,
                      T* psi, long ld, hipStream_t st) {
  const int nk = 2 * sc.kmax + 1, sx = choose_sx<T>(nk);
  return launch(k_orbitals<T, N>, dim3(nstates), inv_lds_bytes<T>(N, nk, sx), st, coef, npw, sc,
                sx, scale, psi, ld);
}

template <class T>
struct OverlapF {
  template <int OPT>
  struct F {
    static ltmp2_status go(const T* psi, long ld, int no, int nv, const int* gdesc, int nh,
                           int kmax, double dV, cplx<T>* nd, hipStream_t st) {
      constexpr int NF = 4;
      const int nk = 2 * kmax + 1, sx = choose_sx_fwd<T>(nk);
      return launch(k_overlap<T, N, NF, OPT>, dim3((no + NF - 1) / NF, nv),
                    fwd_lds_bytes<T>(N, nk, sx), st, psi, ld, no, gdesc, nh, kmax, sx, dV, nd);
    }
  };
};
template <class T>
ltmp2_status overlap(const T* psi, long ld, int no, int nv, const int* gdesc, int nh, int kmax,
                     double dV, cplx<T>* nd, hipStream_t st) {
  return by_opt<OverlapF<T>::template F>(nh, psi, ld, no, nv, gdesc, nh, kmax, dV, nd, st);
}

template <class T>
struct ChiRowsF {
  template <int OPT>
  struct F {
    static ltmp2_status go(const T* chi, long ld, int nr, const int* gdesc, int nh, int kmax,
                           double dV, cplx<T>* chihat, hipStream_t st) {
      constexpr int NF = 2;
      const int nk = 2 * kmax + 1, sx = choose_sx_fwd<T>(nk);
      return launch(k_chi_rows<T, N, NF, OPT>, dim3((nr + NF - 1) / NF),
                    fwd_lds_bytes<T>(N, nk, sx), st, chi, ld, nr, gdesc, nh, kmax, sx, dV,
                    chihat);
    }
  };
};
template <class T>
ltmp2_status chi_rows(const T* chi, long ld, int nr, const int* gdesc, int nh, int kmax, double dV,
                      cplx<T>* chihat, hipStream_t st) {
  return by_opt<ChiRowsF<T>::template F>(nh, chi, ld, nr, gdesc, nh, kmax, dV, chihat, st);
}

template <class T>
struct ChiColsF {
  template <int OPT>
  struct F {
    static ltmp2_status go(const cplx<T>* chihat, long ld, const int* gdesc, int ng, int nh,
                           const double* v, int kmax, double dV, double* pd,
                           cplx<double>* chi_out, ShellBins bins, hipStream_t st) {
      const int nk = 2 * kmax + 1, sx = choose_sx_fwd<T>(nk);
      return launch(k_chi_cols<T, N, OPT>, dim3(nh), fwd_lds_bytes<T>(N, nk, sx), st, chihat, ld,
                    gdesc, ng, nh, v, kmax, sx, dV, pd, chi_out, bins);
    }
  };
};
template <class T>
ltmp2_status chi_cols(const cplx<T>* chihat, long ld, const int* gdesc, int ng, int nh,
                      const double* v, int kmax, double dV, double* pd, cplx<double>* chi_out,
                      ShellBins bins, hipStream_t st) {
  return by_opt<ChiColsF<T>::template F>(ng, chihat, ld, gdesc, ng, nh, v, kmax, dV, pd, chi_out,
                                         bins, st);
}

template <class T>
struct HartreeF {
  template <int OPT>
  struct F {
    static ltmp2_status go(const cplx<T>* h, long ld, const int* gdesc, int ng, const double* v,
                           int kmax, double dV, int g0, int gb, double* pdh, hipStream_t st) {
      const int nk = 2 * kmax + 1, sx = choose_sx_fwd<T>(nk);
      return launch(k_hartree<T, N, OPT>, dim3(gb), fwd_lds_bytes<T>(N, nk, sx), st, h, ld, gdesc,
                    ng, v, kmax, sx, dV, g0, pdh);
    }
  };
};
template <class T>
ltmp2_status hartree(const cplx<T>* h, long ld, const int* gdesc, int ng, const double* v,
                     int kmax, double dV, int g0, int gb, double* pdh, hipStream_t st) {
  return by_opt<HartreeF<T>::template F>(ng, h, ld, gdesc, ng, v, kmax, dV, g0, gb, pdh, st);
}

template <class T>
ltmp2_status wstates(const T* P, int npw, const int* wq, const signed char* wsgn, SphereCols sc,
                     int nitems, double scale, cplx<T>* w, long ld, hipStream_t st) {
  // the largest slab tile that lets four workgroups share a CU, unless two
  // workgroups per CU would allow more than twice that tile
  const int nk = 2 * sc.kmax + 1;
  auto tile = [nk](size_t cap) {
    int sx = slab_tile_at_most(N, 10);
    while (sx > 1 && inv_lds_bytes<T>(N, nk, sx) > cap) sx = slab_tile_at_most(N, sx - 1);
    return sx;
  };
  const int s4 = tile(kLdsQuarter), s2 = tile(kLdsHalf);
  const int sx = 2 * s4 >= s2 ? s4 : s2;
  const size_t lds = inv_lds_bytes<T>(N, nk, sx);
  // orbital spheres at the alias-free window and one below run kernels
  // compiled for that kmax (no per-element branches in the y and z stages)
  constexpr int ko = korb_win(N);
  if (sc.kmax == ko)
    return launch(k_wstates<T, N, ko>, dim3(nitems), lds, st, P, npw, wq, wsgn, sc, sx, scale, w,
                  ld);
  if constexpr (ko > 1)
    if (sc.kmax == ko - 1)
      return launch(k_wstates<T, N, ko - 1>, dim3(nitems), lds, st, P, npw, wq, wsgn, sc, sx,
                    scale, w, ld);
  return launch(k_wstates<T, N>, dim3(nitems), lds, st, P, npw, wq, wsgn, sc, sx, scale, w, ld);
}

// Kept-set instance of the pair kernels for a cell: kwin(N), kwin(N) - 1 or
// the runtime form (-1).
inline int pair_kfix(int kmax) {
  return (kmax == kwin(N) || (kwin(N) > 1 && kmax == kwin(N) - 1)) ? kmax : -1;
}

// Launches that split by cutoff shell run an instance with that epilogue
// compiled in; the others run one without it (fewer live registers; in FP32
// single-buffer forms its z lines are read through buffer resources).
template <class T, int NT, int OPT, int KM, bool JOINT, int MINW>
ltmp2_status pair_go(const PairCell& pc, int sx, hipStream_t st) {
  const long total = long(pc.npairs) * pc.gb;
  const int nk = 2 * pc.kmax + 1;
  const dim3 grid(unsigned((total + 7) / 8 * 8));
  const size_t lds = JOINT ? fwd2_lds_bytes<T>(N, nk, sx) : fwd_lds_bytes<T>(N, nk, sx);
  if (pc.shell)
    return launch_nt(k_pair<T, N, OPT, NT, KM, JOINT, true, MINW>, grid, NT, lds, st, pc, sx);
  return launch_nt(k_pair<T, N, OPT, NT, KM, JOINT, false, MINW>, grid, NT, lds, st, pc, sx);
}

template <class T, int NT, int OPT, bool JOINT = false, int MINW = 1>
ltmp2_status pair_km(const PairCell& pc, int sx, hipStream_t st) {
  constexpr int kw = kwin(N);
  const int kf = pair_kfix(pc.kmax);
  if (kf == kw) return pair_go<T, NT, OPT, kw, JOINT, MINW>(pc, sx, st);
  if constexpr (kw > 1)
    if (kf == kw - 1) return pair_go<T, NT, OPT, kw - 1, JOINT, MINW>(pc, sx, st);
  return pair_go<T, NT, OPT, -1, JOINT, MINW>(pc, sx, st);
}

// Largest slab tile d <= cap whose single slab buffer fits `limit` bytes.
template <class T>
int choose_sx_fwd_within(int nk, int cap, size_t limit) {
  int sx = slab_tile_at_most(N, cap);
  while (sx > 1 && fwd_lds_bytes<T>(N, nk, sx) > limit) sx = slab_tile_at_most(N, sx - 1);
  return sx;
}

// Largest slab tile d <= cap whose two slab buffers (both fields of a pair
// item side by side) fit the shared memory.
template <class T>
int choose_sx_joint(int nk, int cap) {
  int sx = slab_tile_at_most(N, cap);
  while (sx > 1 && fwd2_lds_bytes<T>(N, nk, sx) > kLdsCap) sx = slab_tile_at_most(N, sx - 1);
  return sx;
}

template <class T>
struct PairF {
  template <int OPT>
  struct F {
    static ltmp2_status go(const PairCell& pc, int sx, hipStream_t st) {
      if constexpr (sizeof(T) == sizeof(float) && OPT > 9) {
        return LTMP2_EINVAL;  // FP32 takes the 512-thread form above 9 outputs
      } else {
        return pair_km<T, kThreads, OPT>(pc, sx, st);
      }
    }
  };
};
template <class T>
ltmp2_status pair(const T* psi, long ld, const cplx<T>* w, int no, const int* pairs, int npairs,
                  int gb, const int* gdesc, int ng, const double* v, int kmax, double dV2,
                  double* xpart, const signed char* shell, double* xbins, int nb, int g0,
                  hipStream_t st) {
  PairCell pc{psi, w, pairs, gdesc, v, xpart, ld, no, npairs, gb, ng, kmax, dV2};
  pc.shell = shell;
  pc.xbins = xbins;
  pc.nb = nb;
  pc.g0 = g0;
  if constexpr (sizeof(T) == sizeof(float)) {
    if (ng > 9 * kThreads) {
      // up to 17 outputs per thread: 256 threads with two waves per SIMD
      // held by the launch bounds (244 registers, no spills on the 36 grid)
      // and 12-plane slabs within half the shared memory, so two workgroups
      // share a CU and overlap each other's barriers
      // (compiled for the two fixed kept sets only: the runtime-kmax form
      // spills at 256 registers and takes the 512-thread path instead)
      if constexpr (kwin(N) >= 9) {
        constexpr int kw = kwin(N);
        const int kf = pair_kfix(kmax);
        const int sx = choose_sx_fwd_within<T>(2 * kmax + 1, 12, kLdsHalf);
        if (ng <= 17 * kThreads && kf == kw)
          return pair_go<T, kThreads, 17, kw, false, 2>(pc, sx, st);
        if (ng <= 17 * kThreads && kf == kw - 1)
          return pair_go<T, kThreads, 17, kw - 1, false, 2>(pc, sx, st);
      }
      if (ng > kWideOpt * kWideNT) return LTMP2_EINVAL;
      return pair_km<T, kWideNT, kWideOpt, true>(pc, choose_sx_joint<T>(2 * kmax + 1, 12), st);
    }
  }
  return by_opt<PairF<T>::template F>(ng, pc, choose_sx_fwd<T>(2 * kmax + 1), st);
}

template <class T, int NT, int OPT, int KM, int MINW = 1>
ltmp2_status pair_multi_go(const PairCell* cells, const long* prefix, int ncells, int kmax_max,
                           int sx, int nblocks, hipStream_t st) {
  return launch_nt(k_pair_multi<T, N, OPT, NT, KM, MINW>, dim3(unsigned(nblocks)), NT,
                   fwd_lds_bytes<T>(N, 2 * kmax_max + 1, sx), st, cells, prefix, ncells, sx);
}

template <class T, int NT, int OPT>
ltmp2_status pair_multi_km(int kfix, const PairCell* cells, const long* prefix, int ncells,
                           int kmax_max, int sx, int nblocks, hipStream_t st) {
  constexpr int kw = kwin(N);
  if (kfix >= 0 && kfix != kmax_max) return LTMP2_EINVAL;
  if (kfix == kw) return pair_multi_go<T, NT, OPT, kw>(cells, prefix, ncells, kmax_max, sx, nblocks, st);
  if constexpr (kw > 1)
    if (kfix == kw - 1)
      return pair_multi_go<T, NT, OPT, kw - 1>(cells, prefix, ncells, kmax_max, sx, nblocks, st);
  if (kfix >= 0) return LTMP2_EINVAL;
  return pair_multi_go<T, NT, OPT, -1>(cells, prefix, ncells, kmax_max, sx, nblocks, st);
}

template <class T>
struct PairMultiF {
  template <int OPT>
  struct F {
    static ltmp2_status go(int kfix, const PairCell* cells, const long* prefix, int ncells,
                           int kmax_max, int sx, int nblocks, hipStream_t st) {
      if (sx < 1 || N % sx != 0 || sx > 10) return LTMP2_EINVAL;
      if constexpr (sizeof(T) == sizeof(float) && OPT > 9) {
        return LTMP2_EINVAL;
      } else {
        return pair_multi_km<T, kThreads, OPT>(kfix, cells, prefix, ncells, kmax_max, sx, nblocks,
                                               st);
      }
    }
  };
};
// Several cells of one grid size in one persistent launch; kfix is the kept
// set all of them share (kwin(N) or kwin(N) - 1, see pair_kfix) or -1.
template <class T>
ltmp2_status pair_multi(const PairCell* cells, const long* prefix, int ncells, int ng_max,
                        int kmax_max, int kfix, int sx, int nblocks, hipStream_t st) {
  if constexpr (sizeof(T) == sizeof(float)) {
    if (ng_max > 9 * kThreads) {
      if (sx < 1 || N % sx != 0 || sx > 12) return LTMP2_EINVAL;
      // the single-cell wide form: 256 threads, up to 17 outputs, two
      // workgroups per CU when the slab fits half the shared memory
      if constexpr (kwin(N) >= 9) {
        constexpr int kw = kwin(N);
        if (ng_max <= 17 * kThreads && fwd_lds_bytes<T>(N, 2 * kmax_max + 1, sx) <= kLdsHalf) {
          if (kfix == kw)
            return pair_multi_go<T, kThreads, 17, kw, 2>(cells, prefix, ncells, kmax_max, sx,
                                                         nblocks, st);
          if (kfix == kw - 1)
            return pair_multi_go<T, kThreads, 17, kw - 1, 2>(cells, prefix, ncells, kmax_max,
                                                             sx, nblocks, st);
        }
      }
      if (ng_max > kWideOpt * kWideNT) return LTMP2_EINVAL;
      return pair_multi_km<T, kWideNT, kWideOpt>(kfix, cells, prefix, ncells, kmax_max, sx,
                                                  nblocks, st);
    }
    // a slab group of 129..192 z lines: 192-thread workgroups, one line each
    if (sx >= 1 && sx <= 10 && N % sx == 0 && sx * N > 128 && sx * N <= kNarrowNT &&
        ng_max <= 9 * kNarrowNT) {
      if (ng_max <= 3 * kNarrowNT)
        return pair_multi_km<T, kNarrowNT, 3>(kfix, cells, prefix, ncells, kmax_max, sx, nblocks,
                                              st);
      return pair_multi_km<T, kNarrowNT, 9>(kfix, cells, prefix, ncells, kmax_max, sx, nblocks,
                                            st);
    }
  }
  return by_opt<PairMultiF<T>::template F>(ng_max, kfix, cells, prefix, ncells, kmax_max, sx,
                                           nblocks, st);
}

// Kept-set instance (kwin(N), kwin(N) - 1 or -1) the pair kernels use for kmax.
int pair_kept_instance(int kmax) { return pair_kfix(kmax); }

// Largest slab group of the pair transform that fits the shared memory.
template <class T>
int pair_sx_max(int kmax) {
  return choose_sx_fwd<T>(2 * kmax + 1);
}

// Explicit instantiation in both compilation passes, so the device pass
// instantiates every kernel the host launchers reference.
#define LTMP2_INST(T)                                                                          \
  template ltmp2_status orbitals<T>(const cplx<double>*, int, int, SphereCols, double, T*, long, \
                                    hipStream_t);                                              \
  template ltmp2_status overlap<T>(const T*, long, int, int, const int*, int, int, double,     \
                                   cplx<T>*, hipStream_t);                                     \
  template ltmp2_status chi_rows<T>(const T*, long, int, const int*, int, int, double, cplx<T>*, \
                                    hipStream_t);                                              \
  template ltmp2_status chi_cols<T>(const cplx<T>*, long, const int*, int, int, const double*, \
                                    int, double, double*, cplx<double>*, ShellBins,            \
                                    hipStream_t);                                              \
  template ltmp2_status wstates<T>(const T*, int, const int*, const signed char*, SphereCols,   \
                                   int, double, cplx<T>*, long, hipStream_t);                  \
  template ltmp2_status pair<T>(const T*, long, const cplx<T>*, int, const int*, int, int,     \
                                const int*, int, const double*, int, double, double*,          \
                                const signed char*, double*, int, int, hipStream_t);           \
  template ltmp2_status pair_multi<T>(const PairCell*, const long*, int, int, int, int, int,   \
                                      int, hipStream_t);                                       \
  template int pair_sx_max<T>(int);                                                            \
  template ltmp2_status hartree<T>(const cplx<T>*, long, const int*, int, const double*, int,   \
                                   double, int, int, double*, hipStream_t);
LTMP2_INST(double)
LTMP2_INST(float)

}  // namespace

#define LTMP2_CAT2(a, b) a##b
#define LTMP2_CAT(a, b) LTMP2_CAT2(a, b)
#if !defined(__HIP_DEVICE_COMPILE__)
extern const GridOps<double> LTMP2_CAT(kGridOpsD_, LTMP2_N);
extern const GridOps<float> LTMP2_CAT(kGridOpsF_, LTMP2_N);
const GridOps<double> LTMP2_CAT(kGridOpsD_, LTMP2_N) = {
    orbitals<double>, overlap<double>, chi_rows<double>, chi_cols<double>, wstates<double>,
    pair<double>, pair_multi<double>, hartree<double>, pair_sx_max<double>, pair_kept_instance};
const GridOps<float> LTMP2_CAT(kGridOpsF_, LTMP2_N) = {
    orbitals<float>, overlap<float>, chi_rows<float>, chi_cols<float>, wstates<float>,
    pair<float>, pair_multi<float>, hartree<float>, pair_sx_max<float>, pair_kept_instance};
#endif

}  // namespace ltmp2
