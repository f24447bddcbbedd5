// Transform kernels of the LTMP2 path (templated on precision T and grid n).
#pragma once
#include "transforms.hpp"

namespace ltmp2 {

struct SphereCols {
  int ncol;
  int kmax;
  const int* cdesc;   // [ncol]
  const int* cstart;  // [ncol + 1]
  const int* ckx;     // [n_pw]
};

// ---------------------------------------------------------------------------
// Orbitals on the grid: psi_p(r) = Omega^-1/2 sum_G c_p(G) e^{iG.r}, real for
// time-reversal-invariant coefficients (Gamma point).
//   coef: [n_items][n_pw] complex, entries in column order of the sphere
//   psi:  [n_items][ld] real
template <class T, int N>
__global__ __launch_bounds__(kThreads) void k_orbitals(const cplx<double>* __restrict__ coef, int npw,
                                                       SphereCols sc, int sx, double scale,
                                                       T* __restrict__ psi, long ld) {
  extern __shared__ __align__(16) char smem[];
  const int nk = 2 * sc.kmax + 1;
  SlabLds<T> L = inv_lds<T>(smem, N, nk, sx);
  fill_twiddles<T, 1, N>(L.tw);
  const long p = blockIdx.x;
  const cplx<double>* c = coef + p * npw;
  T* out = psi + p * ld;
  auto cf = [&](int, int e) { return cplx<T>{T(c[e].x), T(c[e].y)}; };
  auto st = [&](int, int x, int y, int z, cplx<T> v) { out[(x * N + z) * N + y] = T(scale) * v.x; };
  inverse_sphere<T, N, 1>(cf, st, 1, sc.kmax, sx, sc.ncol, sc.cdesc, sc.cstart, sc.ckx, L);
}

// ---------------------------------------------------------------------------
// Overlap densities (step (i)): n_aj(G) = dV sum_r psi_a(r) psi_j(r) e^{-iG.r}
// for G in the half set H.  Block (jblock, a); NF occupied j per block.
//   nd: [n_vir][n_h][n_occ] complex
template <class T, int N, int NF, int OPT>
__global__ __launch_bounds__(kThreads) void k_overlap(const T* __restrict__ psi, long ld, int nocc,
                                                      const int* __restrict__ gdesc_all, int nh,
                                                      int kmax, int sx, double dV,
                                                      cplx<T>* __restrict__ nd) {
  extern __shared__ __align__(16) char smem[];
  const int nk = 2 * kmax + 1;
  SlabLds<T> L = fwd_lds<T>(smem, N, nk, sx);
  fill_twiddles<T, -1, N>(L.tw);
  const int j0 = blockIdx.x * NF;
  const int a = blockIdx.y;
  const int nf = min(NF, nocc - j0);
  const T* pa = psi + long(nocc + a) * ld;
  const T* pj = psi + long(j0) * ld;
  int gd[OPT];
  cplx<T> acc[NF][OPT];
#pragma unroll
  for (int t = 0; t < OPT; ++t) {
    const int o = threadIdx.x + t * kThreads;
    gd[t] = (o < nh) ? gdesc_all[o] : 0;
#pragma unroll
    for (int f = 0; f < NF; ++f) acc[f][t] = {T(0), T(0)};
  }
  __syncthreads();
  auto ld_ = [&](int f, int x, int y, int z) {
    const long r = (x * N + z) * N + y;
    return cplx<T>{pa[r] * pj[f * ld + r], T(0)};
  };
  forward_pruned<T, -1, N, NF, OPT>(ld_, nf, kmax, sx, gd, nh, acc, L);
#pragma unroll
  for (int t = 0; t < OPT; ++t) {
    const int o = threadIdx.x + t * kThreads;
    if (o < nh) {
#pragma unroll
      for (int f = 0; f < NF; ++f)
        if (f < nf)
          nd[(long(a) * nh + o) * nocc + j0 + f] = {T(dV) * acc[f][t].x, T(dV) * acc[f][t].y};
    }
  }
}

// ---------------------------------------------------------------------------
// First pass of the double transform of chi (rows): for NF rows r,
//   chihat(r, G') = dV sum_r' chi(r, r') e^{+iG'.r'},  G' in H.
//   chi: [n_r][ld] real;  chihat: [n_h][ld] complex (column-major in r)
template <class T, int N, int NF, int OPT>
__global__ __launch_bounds__(kThreads) void k_chi_rows(const T* __restrict__ chi, long ld, int nr,
                                                       const int* __restrict__ gdesc_all, int nh,
                                                       int kmax, int sx, double dV,
                                                       cplx<T>* __restrict__ chihat) {
  extern __shared__ __align__(16) char smem[];
  const int nk = 2 * kmax + 1;
  SlabLds<T> L = fwd_lds<T>(smem, N, nk, sx);
  fill_twiddles<T, 1, N>(L.tw);
  const int r0 = blockIdx.x * NF;
  const int nf = min(NF, nr - r0);
  const T* row = chi + long(r0) * ld;
  int gd[OPT];
  cplx<T> acc[NF][OPT];
#pragma unroll
  for (int t = 0; t < OPT; ++t) {
    const int o = threadIdx.x + t * kThreads;
    gd[t] = (o < nh) ? gdesc_all[o] : 0;
#pragma unroll
    for (int f = 0; f < NF; ++f) acc[f][t] = {T(0), T(0)};
  }
  __syncthreads();
  auto ld_ = [&](int f, int x, int y, int z) {
    return cplx<T>{row[f * ld + (x * N + z) * N + y], T(0)};
  };
  forward_pruned<T, 1, N, NF, OPT>(ld_, nf, kmax, sx, gd, nh, acc, L);
#pragma unroll
  for (int t = 0; t < OPT; ++t) {
    const int o = threadIdx.x + t * kThreads;
    if (o < nh) {
#pragma unroll
      for (int f = 0; f < NF; ++f)
        if (f < nf) chihat[long(o) * ld + r0 + f] = {T(dV) * acc[f][t].x, T(dV) * acc[f][t].y};
    }
  }
}

// ---------------------------------------------------------------------------
// Second pass (columns) and the Coulomb trace: for G' = H[g],
//   chi(G, G') = dV sum_r e^{-iG.r} chihat(r, G'),  G in the full set,
//   pd[g] = v(G') sum_G v(G) |chi(G, G')|^2.
// Optionally stores chi(G, G') for G' in H and, by chi(-G, -G') =
// conj chi(G, G') (real chi(r, r')), for G' in -H:  out[G][G'] (ng x ng),
// and the same sum split by auxiliary cutoff shell (bins.out [n_h][nb]).
template <class T, int N, int OPT>
__global__ __launch_bounds__(kThreads) void k_chi_cols(const cplx<T>* __restrict__ chihat, long ld,
                                                       const int* __restrict__ gdesc_all, int ng,
                                                       int nh, const double* __restrict__ v,
                                                       int kmax, int sx, double dV,
                                                       double* __restrict__ pd,
                                                       cplx<double>* __restrict__ chi_out,
                                                       ShellBins bins) {
  extern __shared__ __align__(16) char smem[];
  __shared__ double red[kThreads / 64];
  __shared__ double redb[kThreads / 64 * kMaxShells];
  const int nk = 2 * kmax + 1;
  SlabLds<T> L = fwd_lds<T>(smem, N, nk, sx);
  fill_twiddles<T, -1, N>(L.tw);
  const int g = blockIdx.x;
  const cplx<T>* col = chihat + long(g) * ld;
  int gd[OPT];
  cplx<T> acc[1][OPT];
#pragma unroll
  for (int t = 0; t < OPT; ++t) {
    const int o = threadIdx.x + t * kThreads;
    gd[t] = (o < ng) ? gdesc_all[o] : 0;
    acc[0][t] = {T(0), T(0)};
  }
  __syncthreads();
  auto ld_ = [&](int, int x, int y, int z) { return col[(x * N + z) * N + y]; };
  forward_pruned<T, -1, N, 1, OPT>(ld_, 1, kmax, sx, gd, ng, acc, L);
  double s = 0.0;
  double sb[kMaxShells] = {};
  const int sg = bins.shell ? bins.shell[g] : 0;
#pragma unroll
  for (int t = 0; t < OPT; ++t) {
    const int o = threadIdx.x + t * kThreads;
    if (o < ng) {
      const double re = dV * double(acc[0][t].x), im = dV * double(acc[0][t].y);
      const double term = v[o] * (re * re + im * im);
      s += term;
      if (bins.shell) bin_add(sb, min(int(bins.shell[o]), sg) - 1, term);
      if (chi_out) {
        const int on = (o < nh) ? o + nh : o - nh;
        chi_out[long(o) * ng + g] = {re, im};
        chi_out[long(on) * ng + g + nh] = {re, -im};
      }
    }
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) pd[g] = v[g] * s;
  if (bins.shell) {
    block_sum_bins(sb, redb);
    if (threadIdx.x == 0)
      for (int b = 0; b < bins.nb; ++b) bins.out[long(g) * bins.nb + b] = v[g] * sb[b];
  }
}

// ---------------------------------------------------------------------------
// Hartree-like route to the direct term (Implementation section, step
// (iv.a)), a cross-check of the chi route that shares none of its kernels:
//   h^{(G')}(r)  = sum_i psi_i(r) w_i^{(G')}(r)
//   X^{(G')}(G)  = dV sum_r e^{-iG.r} h^{(G')}(r)      (= chi(G, -G'))
//   pdh[g0 + gl] = v(G') sum_G v(G) |X^{(G')}(G)|^2,   E_d(tau) = -4 sum_{H} pdh.
// k_hsum: grid (ceil(n_r / 256), gb); h [gb][ld] complex.
template <class T>
__global__ __launch_bounds__(256) void k_hsum(const T* __restrict__ psi, long ld,
                                              const cplx<T>* __restrict__ w, int no, long nr,
                                              cplx<T>* __restrict__ h) {
  const long r = long(blockIdx.x) * 256 + threadIdx.x;
  const long gl = blockIdx.y;
  if (r >= nr) return;
  cplx<T> s = {T(0), T(0)};
  for (int i = 0; i < no; ++i) {
    const T a = psi[long(i) * ld + r];
    const cplx<T> b = w[(gl * no + i) * ld + r];
    s.x += a * b.x;
    s.y += a * b.y;
  }
  h[gl * ld + r] = s;
}

// one block per outer vector gl of the block
template <class T, int N, int OPT>
__global__ __launch_bounds__(kThreads) void k_hartree(const cplx<T>* __restrict__ h, long ld,
                                                      const int* __restrict__ gdesc_all, int ng,
                                                      const double* __restrict__ v, int kmax,
                                                      int sx, double dV, int g0,
                                                      double* __restrict__ pdh) {
  extern __shared__ __align__(16) char smem[];
  __shared__ double red[kThreads / 64];
  const int nk = 2 * kmax + 1;
  SlabLds<T> L = fwd_lds<T>(smem, N, nk, sx);
  fill_twiddles<T, -1, N>(L.tw);
  const int gl = blockIdx.x;
  const cplx<T>* col = h + long(gl) * ld;
  int gd[OPT];
  cplx<T> acc[1][OPT];
#pragma unroll
  for (int t = 0; t < OPT; ++t) {
    const int o = threadIdx.x + t * kThreads;
    gd[t] = (o < ng) ? gdesc_all[o] : 0;
    acc[0][t] = {T(0), T(0)};
  }
  __syncthreads();
  auto ld_ = [&](int, int x, int y, int z) { return col[(x * N + z) * N + y]; };
  forward_pruned<T, -1, N, 1, OPT>(ld_, 1, kmax, sx, gd, ng, acc, L);
  double s = 0.0;
#pragma unroll
  for (int t = 0; t < OPT; ++t) {
    const int o = threadIdx.x + t * kThreads;
    if (o < ng) {
      const double re = dV * double(acc[0][t].x), im = dV * double(acc[0][t].y);
      s += v[o] * (re * re + im * im);
    }
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) pdh[g0 + gl] = v[g0 + gl] * s;
}

// ---------------------------------------------------------------------------
// Transformed states on the grid (step (iii)):
//   w_j^{(G')}(r) = Omega^-1/2 sum_G W_j(G) e^{iG.r},
// with W_j(G) rebuilt from the real-basis product P = C Psi_v:
//   P[(g, j, 0)][q] = sum_a Re C_ja B[a][q],  P[(g, j, 1)][q] = sum_a Im C_ja B[a][q],
// where B[a][q] holds Re c_a(0), Re c_a(G_k), Im c_a(G_k) for the half sphere.
// W_j(G) is gathered from P where the x stage needs it.
// Entry e of the sphere (column order) uses wq[e] = q_re | (q_im + 1) << 16
// and the sign s = +1 for G_k, -1 for -G_k (c_a(-G) = conj c_a(G)):
//   W(G) = (P_re[q_re] - s P_im[q_im]) + i (P_im[q_re] + s P_re[q_im]).
template <class T, int N, int KO = -1>
__global__ __launch_bounds__(kThreads) void k_wstates(const T* __restrict__ P, int npw,
                                                      const int* __restrict__ wq,
                                                      const signed char* __restrict__ wsgn,
                                                      SphereCols sc, int sx, double scale,
                                                      cplx<T>* __restrict__ w, long ld) {
  extern __shared__ __align__(16) char smem[];
  const int nk = 2 * (KO >= 0 ? KO : sc.kmax) + 1;
  SlabLds<T> L = inv_lds<T>(smem, N, nk, sx);
  fill_twiddles<T, 1, N>(L.tw);
  const long item = blockIdx.x;
  const T* pre = P + (2 * item) * long(npw);
  const T* pim = pre + npw;
  cplx<T>* out = w + item * ld;
  // W_j(G) of sphere entry e, gathered from the real basis (each entry is
  // used once per slab group)
  auto cf = [&](int, int e) {
    const int q = wq[e];
    const int qr = q & 0xffff, qi = (q >> 16) - 1;
    const T s = T(wsgn[e]);
    T re = pre[qr], im = pim[qr];
    if (qi >= 0) {
      re -= s * pim[qi];
      im += s * pre[qi];
    }
    return cplx<T>{re, im};
  };
  auto st = [&](int, int x, int y, int z, cplx<T> v) {
    out[(x * N + z) * N + y] = {T(scale) * v.x, T(scale) * v.y};
  };
  inverse_sphere<T, N, 1, KO>(cf, st, 1, sc.kmax, sx, sc.ncol, sc.cdesc, sc.cstart, sc.ckx, L);
}

// ---------------------------------------------------------------------------
// Fock-like contraction (step (iv.b)) for one G' and one occupied pair i <= j:
//   A_ij(G) = dV sum_r psi_i(r) w_j(r) e^{-iG.r},  G in the full set,
//   xpart = sum_G v(G) [A_ij conj(A_ji) + A_ji conj(A_ij)]   (i < j)
//         = sum_G v(G) |A_ii|^2                               (i = j).
// Summed over pairs this is S_x(G') = sum_G v(G) sum_ij A_ij(G) A^{(-G')}_ji(-G),
// using A^{(-G')}_ji(-G) = conj A^{(G')}_ji(G) for real orbitals.

// The pair item's rows are the same for every lane of the workgroup; taking
// a row's address from the first lane tells the compiler so, and lets it
// address the z line as scalar base + 32-bit lane offset + the step along z
// folded into the load instruction, with no per-load 64-bit arithmetic.
template <class V>
using global_row = const __attribute__((address_space(1))) V*;
template <class V>
__device__ inline global_row<V> uniform_row(const V* p) {
  const unsigned long long u = reinterpret_cast<unsigned long long>(p);
  const unsigned lo = __builtin_amdgcn_readfirstlane(unsigned(u));
  const unsigned hi = __builtin_amdgcn_readfirstlane(unsigned(u >> 32));
  return reinterpret_cast<global_row<V>>((static_cast<unsigned long long>(hi) << 32) | lo);
}

// The same rows through buffer resources: the base in scalar registers, a
// 32-bit lane offset, the step along z in the instruction, no address
// arithmetic at all.  Word 3 holds the gfx9-family default format;
// num_records bounds every access to the row (reads past it return zero).
// Used for FP32 where the compiler keeps a whole z line of these loads in
// flight (the forms without the per-shell epilogue or a second slab
// buffer); with more live registers it spaces them out, and the global
// loads above then do better.
template <class V>
__device__ inline __amdgpu_buffer_rsrc_t row_rsrc(const V* p, unsigned n) {
  const unsigned long long u = reinterpret_cast<unsigned long long>(p);
  const unsigned lo = __builtin_amdgcn_readfirstlane(unsigned(u));
  const unsigned hi = __builtin_amdgcn_readfirstlane(unsigned(u >> 32));
  void* q = reinterpret_cast<void*>((static_cast<unsigned long long>(hi) << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(q, short(0), int(n * sizeof(V)), 0x00020000);
}
template <class V>
__device__ inline V row_load(__amdgpu_buffer_rsrc_t rs, unsigned off);
template <>
__device__ inline float row_load<float>(__amdgpu_buffer_rsrc_t rs, unsigned off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0));
}
template <>
__device__ inline cplx<float> row_load<cplx<float>>(__amdgpu_buffer_rsrc_t rs, unsigned off) {
  return __builtin_bit_cast(cplx<float>, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
}

// Everything one cell contributes to a pair launch.
struct PairCell {
  const void* psi;     // [nocc..][ld] orbitals (T)
  const void* w;       // [gb][nocc][ld] transformed states (cplx<T>)
  const int* pairs;    // [npairs] i | j << 16
  const int* gdesc;    // [ng]
  const double* v;     // [ng]
  double* xpart;       // [gb][npairs] partial sums of this block
  long ld;
  int nocc, npairs, gb, ng, kmax;
  double dV2;
  // optional split by auxiliary cutoff shell (ShellBins): shell [ng], the
  // block's first outer vector g0 (shell of G' = shell[g0 + gl]) and
  // xbins [gb][npairs][nb] (nullptr: no split)
  const signed char* shell = nullptr;
  double* xbins = nullptr;
  int nb = 0, g0 = 0;
};

// KM >= 0: the cell's kept set is kmax = KM, known at compile time (see kwin);
// KM = -1: runtime kmax.  JOINT: both fields side by side in two slab
// buffers (forward_pruned_joint; shared memory fwd2_lds_bytes).  BINS: the
// per-shell split of the cutoff extrapolation is compiled in (taken when
// pc.shell is set); the batched launches, which never split, leave it out.
template <class T, int N, int OPT, int NT = kThreads, int KM = -1, bool JOINT = false,
          bool BINS = true>
__device__ inline void pair_item(const PairCell& pc, int gl, int p, int sx, void* smem,
                                 double* red) {
  const int nk = 2 * (KM >= 0 ? KM : pc.kmax) + 1;
  SlabLds<T> L = JOINT ? fwd2_lds<T>(smem, N, nk, sx) : fwd_lds<T>(smem, N, nk, sx);
  fill_twiddles<T, -1, N>(L.tw);
  const int i = pc.pairs[p] & 0xffff, j = pc.pairs[p] >> 16;
  const T* psi = static_cast<const T*>(pc.psi);
  const cplx<T>* w = static_cast<const cplx<T>*>(pc.w);
  const T* pi = psi + long(i) * pc.ld;
  const T* pj = psi + long(j) * pc.ld;
  const cplx<T>* wi = w + (long(gl) * pc.nocc + i) * pc.ld;
  const cplx<T>* wj = w + (long(gl) * pc.nocc + j) * pc.ld;
  constexpr unsigned nr = unsigned(N) * N * N;
  // FP32: buffer loads where the whole line stays in flight, else scalar-base
  // global loads; FP64 (twice the registers per value) keeps plain 64-bit
  // addresses, which the compiler schedules best there
  constexpr bool kFp32 = sizeof(T) == sizeof(float);
  constexpr bool kBuffer = kFp32 && !JOINT && !BINS;
  int gd[OPT];
  cplx<T> acc[2][OPT];
#pragma unroll
  for (int t = 0; t < OPT; ++t) {
    const int o = threadIdx.x + t * NT;
    gd[t] = (o < pc.ng) ? pc.gdesc[o] : 0;
    acc[0][t] = {T(0), T(0)};
    acc[1][t] = {T(0), T(0)};
  }
  __syncthreads();
  const auto gpi = uniform_row(pi), gpj = uniform_row(pj);
  const auto gwi = uniform_row(wi), gwj = uniform_row(wj);
  const auto bpi = row_rsrc(pi, nr), bpj = row_rsrc(pj, nr);
  const auto bwi = row_rsrc(wi, nr), bwj = row_rsrc(wj, nr);
  // grid index r = (x N + z) N + y: the lane's line start r0, then z N
  auto ld_ = [&](int f, int x, int y, int z) {
    const unsigned r0 = unsigned(x * N * N + y);
    if constexpr (kBuffer) {
      const unsigned r = r0 + unsigned(z * N);
      const T a = row_load<T>(f == 0 ? bpi : bpj, r * unsigned(sizeof(T)));
      const cplx<T> b = row_load<cplx<T>>(f == 0 ? bwj : bwi, r * unsigned(sizeof(cplx<T>)));
      return cplx<T>{a * b.x, a * b.y};
    } else if constexpr (kFp32) {
      const T a = ((f == 0) ? gpi : gpj)[size_t(r0) + z * N];
      const auto& b = ((f == 0) ? gwj : gwi)[size_t(r0) + z * N];
      return cplx<T>{a * b.x, a * b.y};
    } else {
      const long r = (x * N + z) * N + y;
      const T a = (f == 0) ? pi[r] : pj[r];
      const cplx<T> b = (f == 0) ? wj[r] : wi[r];
      return cplx<T>{a * b.x, a * b.y};
    }
  };
  if constexpr (JOINT)
    forward_pruned_joint<T, -1, N, OPT, NT, KM>(ld_, (i == j) ? 1 : 2, pc.kmax, sx, gd, pc.ng, acc,
                                                L);
  else
    forward_pruned<T, -1, N, 2, OPT, NT, KM>(ld_, (i == j) ? 1 : 2, pc.kmax, sx, gd, pc.ng, acc,
                                             L);
  double s = 0.0;
  double sb[kMaxShells] = {};
  const bool split = BINS && pc.shell;
  const int sg = split ? pc.shell[pc.g0 + gl] : 0;
#pragma unroll
  for (int t = 0; t < OPT; ++t) {
    const int o = threadIdx.x + t * NT;
    if (o < pc.ng) {
      const double ar = acc[0][t].x, ai = acc[0][t].y;
      double term;
      if (i == j) {
        term = pc.v[o] * (ar * ar + ai * ai);
      } else {
        const double br = acc[1][t].x, bi = acc[1][t].y;
        term = 2.0 * pc.v[o] * (ar * br + ai * bi);
      }
      s += term;
      if constexpr (BINS)
        if (split) bin_add(sb, min(int(pc.shell[o]), sg) - 1, term);
    }
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) pc.xpart[long(gl) * pc.npairs + p] = pc.dV2 * s;
  if constexpr (BINS) {
    if (split) {
      __shared__ double redb[NT / 64 * kMaxShells];
      block_sum_bins(sb, redb);
      if (threadIdx.x == 0)
        for (int b = 0; b < pc.nb; ++b)
          pc.xbins[(long(gl) * pc.npairs + p) * pc.nb + b] = pc.dV2 * sb[b];
    }
  }
}

// One cell: workgroups are dispatched round-robin over the 8 XCDs; each XCD
// gets a contiguous range of the (G', pair) list, whose pairs come in 8 x 8
// blocks of (i, j), so the workgroups resident on one XCD share a handful of
// psi_i and w_j^{(G')} in that XCD's L2.
template <class T, int N, int OPT, int NT = kThreads, int KM = -1, bool JOINT = false,
          bool BINS = true, int MINW = 1>
__global__ __launch_bounds__(NT, MINW) void k_pair(PairCell pc, int sx) {
  extern __shared__ __align__(16) char smem[];
  __shared__ double red[NT / 64];
  const long total = long(pc.npairs) * pc.gb;
  const long per_xcd = (total + 7) / 8;
  const long t = long(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (t >= total) return;
  const int gl = int(t / pc.npairs);
  pair_item<T, N, OPT, NT, KM, JOINT, BINS>(pc, gl, int(t - long(gl) * pc.npairs), sx, smem,
                                            red);
}

// Several cells of the same grid in one persistent launch: the work list is
// the concatenation of every cell's (G', pair) items (prefix[c] = first item
// of cell c); each XCD owns a contiguous range and its workgroups stride
// through it, so every workgroup exits after a bounded number of items.
template <class T, int N, int OPT, int NT = kThreads, int KM = -1, int MINW = 1>
__global__ __launch_bounds__(NT, MINW) void k_pair_multi(const PairCell* __restrict__ cells,
                                                         const long* __restrict__ prefix,
                                                         int ncells, int sx) {
  extern __shared__ __align__(16) char smem[];
  __shared__ double red[NT / 64];
  const long total = prefix[ncells];
  const long per_xcd = (total + 7) / 8;
  const long stride = gridDim.x / 8;
  for (long q = blockIdx.x / 8; q < per_xcd; q += stride) {
    const long t = long(blockIdx.x % 8) * per_xcd + q;
    if (t >= total) break;
    int lo = 0, hi = ncells - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (prefix[mid] <= t) lo = mid; else hi = mid - 1;
    }
    const PairCell pc = cells[lo];
    const long u = t - prefix[lo];
    const int gl = int(u / pc.npairs);
    pair_item<T, N, OPT, NT, KM, false, false>(pc, gl, int(u - long(gl) * pc.npairs), sx, smem,
                                               red);
    __syncthreads();
  }
}

}  // namespace ltmp2
