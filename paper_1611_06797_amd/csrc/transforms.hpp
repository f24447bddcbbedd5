// Slab-streamed 3-D transforms between the real-space grid and a pruned set
// of reciprocal vectors (a sphere), built on the register FFTs of fft.hpp.
//
// Real-space fields are stored with flat index r = (x * n + z) * n + y, so
// that threads owning consecutive y read consecutive addresses while each
// walks its own z-line.
//
// Forward (grid -> G list):  out(G) = sum_r f(r) exp(S i G.r)
//   per slab group of SX x-planes:  FFT along z (keep |kz| <= kmax), FFT
//   along y (keep |ky| <= kmax), then a direct DFT along x accumulated into
//   the outputs each thread owns.  The x-DFT only touches the kept G, so the
//   transform never forms the full n^3 spectrum.
// Inverse (G list -> grid):  f(r) = sum_G c(G) exp(+i G.r)
//   per slab group: direct DFT along x from the sphere's (ky, kz) columns,
//   FFT along y, FFT along z, write the slab.
#pragma once
#include <utility>

#include "fft.hpp"

namespace ltmp2 {

constexpr int kThreads = 256;

// Packed descriptor of one kept reciprocal vector:
//   bits 0-7   kx mod n
//   bits 8-15  ky + kmax
//   bits 16-23 kz + kmax
__host__ __device__ inline int pack_g(int kxm, int kyi, int kzi) {
  return kxm | (kyi << 8) | (kzi << 16);
}

// Row length of the z-pass buffer: even grids get one pad element against
// shared-memory bank conflicts, odd ones need none.
__host__ __device__ constexpr int slab_row(int n) { return n + (n % 2 == 0 ? 1 : 0); }

template <class T>
struct SlabLds {
  cplx<T>* t1;  // [SX][nk][slab_row(n)]
  cplx<T>* tw;  // [n]
  int* cmap;    // inverse transforms: [nk][nk] packed sphere column of each (kz, ky) slot
};

// Both transform directions keep a slab group in one buffer,
// t1 [SX][nk][slab_row(n)], followed by the twiddles.  Forward: the z pass
// fills rows (xs, kz), the y pass writes its kept outputs back into the
// start of the row it read.  Inverse: the x stage fills the start of each
// row (kept ky), the y stage expands the row in place to all n values of y.
template <class T>
__host__ __device__ inline size_t fwd_lds_bytes(int n, int nk, int sx) {
  return sizeof(cplx<T>) * (size_t(sx) * nk * slab_row(n) + n);
}

template <class T>
__device__ inline SlabLds<T> fwd_lds(void* base, int n, int nk, int sx) {
  SlabLds<T> s;
  s.t1 = reinterpret_cast<cplx<T>*>(base);
  s.tw = s.t1 + size_t(sx) * nk * slab_row(n);
  s.cmap = nullptr;
  return s;
}

// The inverse layout adds the slot-to-column map after the twiddles: per
// (kz, ky) slot, the column's first entry | its length << 16 | (kx of its
// first entry mod n) << 22, or 0 outside the sphere (entries < 2^16, column
// lengths and n < 64).
template <class T>
__host__ __device__ inline size_t inv_lds_bytes(int n, int nk, int sx) {
  return fwd_lds_bytes<T>(n, nk, sx) + sizeof(int) * size_t(nk) * nk;
}

template <class T>
__device__ inline SlabLds<T> inv_lds(void* base, int n, int nk, int sx) {
  SlabLds<T> s = fwd_lds<T>(base, n, nk, sx);
  s.cmap = reinterpret_cast<int*>(s.tw + n);
  return s;
}

// exp(S 2 pi i e / N), e = 0..N-1, as a compile-time table in constant memory.
template <class T, int S, int N, class Seq = std::make_integer_sequence<int, N>>
struct TwiddleTable;
template <class T, int S, int N, int... E>
struct TwiddleTable<T, S, N, std::integer_sequence<int, E...>> {
  static constexpr cplx<T> v[N] = {twiddle<T, S>(E, N)...};
};

// exp(S 2 pi i e / N) for e = 0..N-1 into shared memory
template <class T, int S, int N>
__device__ inline void fill_twiddles(cplx<T>* tw) {
  for (int e = threadIdx.x; e < N; e += blockDim.x) tw[e] = TwiddleTable<T, S, N>::v[e];
}

// Compile-time pruning window of a grid: the largest kept set an alias-free
// transform grid can have (N >= 2 k_orb + k_aux + 1 >= 3 k_aux + 1).  Pair
// transforms with kept set kmax = kwin(N) or kwin(N) - 1 run kernels compiled
// for that kmax, so which FFT outputs are stored needs no per-element branch.
__host__ __device__ constexpr int kwin(int n) { return (n - 1) / 3; }

// The same for the orbital sphere of the inverse transforms: with the
// auxiliary window kwin(N), an alias-free grid allows k_orb <= korb_win(N).
__host__ __device__ constexpr int korb_win(int n) { return (n - 1 - kwin(n)) / 2; }

// Largest slab tile d <= cap that divides n (tiles are 1..6, 8, 9, 10, 12).
__host__ __device__ constexpr int slab_tile_at_most(int n, int cap) {
  for (int d = cap < 12 ? cap : 12; d > 1; --d)
    if (d != 7 && d != 11 && n % d == 0) return d;
  return 1;
}

// In-place length-D transforms of the nc columns of a [D][nc] LDS array.
template <class T, int S, int D, int NT = kThreads>
__device__ inline void column_fft(cplx<T>* a, int nc) {
  for (int c = threadIdx.x; c < nc; c += NT) {
    cplx<T> v[D];
#pragma unroll
    for (int k = 0; k < D; ++k) v[k] = a[k * nc + c];
    Fft<T, S, D>::run(v);
#pragma unroll
    for (int k = 0; k < D; ++k) a[k * nc + c] = v[k];
  }
}

// Slab tiles: divisors d <= 12 of the grid size (d = 1 is a no-op).
template <class T, int S, int N, int NT = kThreads>
__device__ inline void column_fft_tile(cplx<T>* a, int d, int nc) {
  if constexpr (N % 12 == 0) if (d == 12) return column_fft<T, S, 12, NT>(a, nc);
  if constexpr (N % 10 == 0) if (d == 10) return column_fft<T, S, 10, NT>(a, nc);
  if constexpr (N % 9 == 0) if (d == 9) return column_fft<T, S, 9, NT>(a, nc);
  if constexpr (N % 8 == 0) if (d == 8) return column_fft<T, S, 8, NT>(a, nc);
  if constexpr (N % 6 == 0) if (d == 6) return column_fft<T, S, 6, NT>(a, nc);
  if constexpr (N % 5 == 0) if (d == 5) return column_fft<T, S, 5, NT>(a, nc);
  if constexpr (N % 4 == 0) if (d == 4) return column_fft<T, S, 4, NT>(a, nc);
  if constexpr (N % 3 == 0) if (d == 3) return column_fft<T, S, 3, NT>(a, nc);
  if constexpr (N % 2 == 0) if (d == 2) return column_fft<T, S, 2, NT>(a, nc);
}

// Length-D transforms across the planes of the forward layout: column
// (kzi, kyi) of plane xs sits at a[xs * pstride + kzi * R + kyi].
template <class T, int S, int D, int NT>
__device__ inline void column_fft_rows(cplx<T>* a, int nk, int R, int pstride) {
  // c / nk by a multiply-high: exact for c < nk^2 <= 2^12 (the error of the
  // rounded-up reciprocal stays below 2^32 / c)
  const unsigned inv = 0xffffffffu / unsigned(nk) + 1u;
  for (int c = threadIdx.x; c < nk * nk; c += NT) {
    const int kzi = int(__umulhi(unsigned(c), inv)), kyi = c - kzi * nk;
    cplx<T>* b = a + kzi * R + kyi;
    cplx<T> v[D];
#pragma unroll
    for (int k = 0; k < D; ++k) v[k] = b[k * pstride];
    Fft<T, S, D>::run(v);
#pragma unroll
    for (int k = 0; k < D; ++k) b[k * pstride] = v[k];
  }
}

template <class T, int S, int N, int NT = kThreads>
__device__ inline void column_fft_rows_tile(cplx<T>* a, int d, int nk, int R, int pstride) {
  if constexpr (N % 12 == 0) if (d == 12) return column_fft_rows<T, S, 12, NT>(a, nk, R, pstride);
  if constexpr (N % 10 == 0) if (d == 10) return column_fft_rows<T, S, 10, NT>(a, nk, R, pstride);
  if constexpr (N % 9 == 0) if (d == 9) return column_fft_rows<T, S, 9, NT>(a, nk, R, pstride);
  if constexpr (N % 8 == 0) if (d == 8) return column_fft_rows<T, S, 8, NT>(a, nk, R, pstride);
  if constexpr (N % 6 == 0) if (d == 6) return column_fft_rows<T, S, 6, NT>(a, nk, R, pstride);
  if constexpr (N % 5 == 0) if (d == 5) return column_fft_rows<T, S, 5, NT>(a, nk, R, pstride);
  if constexpr (N % 4 == 0) if (d == 4) return column_fft_rows<T, S, 4, NT>(a, nk, R, pstride);
  if constexpr (N % 3 == 0) if (d == 3) return column_fft_rows<T, S, 3, NT>(a, nk, R, pstride);
  if constexpr (N % 2 == 0) if (d == 2) return column_fft_rows<T, S, 2, NT>(a, nk, R, pstride);
}

// Forward pruned transform of NF fields.  Load(f, x, y, z) returns the
// field value; acc[f][t] accumulates output o = threadIdx.x + t * NT
// (o < nout; NT threads per workgroup) whose packed descriptor is gdesc[t]
// (pre-loaded by the caller).
//
// The x transform is split as N = M * sx (sx divides N): slab group x2
// holds the planes x = x2 + M xs, xs < sx.  After the z and y passes of the
// group, a length-sx FFT across its planes gives, for every kept (ky, kz),
// Y_x2(q) = sum_xs f(x2 + M xs) w_sx^{q xs}; output kx then needs only
// w_N^{kx x2} Y_x2(kx mod sx), one product per group instead of sx.
// KM >= 0 fixes kmax = KM at compile time (see kwin).  L is the forward
// layout (fwd_lds).
template <class T, int S, int N, int NF, int OPT, int NT = kThreads, int KM = -1, class Load>
__device__ __forceinline__ void forward_pruned(const Load& ld, int nf_active, int kmax_rt, int sx,
                                               const int (&gdesc)[OPT], int nout,
                                               cplx<T> (&acc)[NF][OPT], const SlabLds<T>& L) {
  constexpr int R = slab_row(N);
  const int kmax = KM >= 0 ? KM : kmax_rt;
  const int nk = 2 * kmax + 1, M = N / sx, pstride = nk * R;
  const int tid = threadIdx.x;
  // per output: offset of its (residue plane, kz, ky) entry (low 24 bits) and kx
  int ox[OPT];
#pragma unroll
  for (int t = 0; t < OPT; ++t) {
    const int kxm = gdesc[t] & 0xff, kyi = (gdesc[t] >> 8) & 0xff, kzi = gdesc[t] >> 16;
    ox[t] = ((kxm % sx) * pstride + kzi * R + kyi) | (kxm << 24);
  }
  for (int x2 = 0; x2 < M; ++x2) {
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      if (f >= nf_active) break;
      // z pass: line (xs, y) -> rows (xs, kz)
      for (int l = tid; l < sx * N; l += NT) {
        const int xs = l / N, y = l - xs * N, x = x2 + M * xs;
        cplx<T> v[N];
#pragma unroll
        for (int z = 0; z < N; ++z) v[z] = ld(f, x, y, z);
        Fft<T, S, N>::run(v);
#pragma unroll
        for (int z = 0; z < N; ++z) {
          const int kz = (z <= N / 2) ? z : z - N;
          if (kz >= -kmax && kz <= kmax) L.t1[(xs * nk + kz + kmax) * R + y] = v[z];
        }
      }
      __syncthreads();
      // y pass: row (xs, kz) in place; the kept ky land at the row's start
      for (int l = tid; l < sx * nk; l += NT) {
        cplx<T>* row = L.t1 + l * R;
        cplx<T> v[N];
#pragma unroll
        for (int y = 0; y < N; ++y) v[y] = row[y];
        Fft<T, S, N>::run(v);
#pragma unroll
        for (int y = 0; y < N; ++y) {
          const int ky = (y <= N / 2) ? y : y - N;
          if (ky >= -kmax && ky <= kmax) row[ky + kmax] = v[y];
        }
      }
      __syncthreads();
      // x: length-sx FFT across the group's planes, then one product per output
      column_fft_rows_tile<T, S, N, NT>(L.t1, sx, nk, R, pstride);
      if (sx > 1) __syncthreads();
#pragma unroll
      for (int t = 0; t < OPT; ++t) {
        const int o = tid + t * NT;
        if (o < nout)
          acc[f][t] = cfma(L.tw[((ox[t] >> 24) * x2) % N], L.t1[ox[t] & 0xffffff], acc[f][t]);
      }
      __syncthreads();  // the next z pass overwrites the rows
    }
  }
}

// Both fields of forward_pruned (NF = 2) side by side: two slab buffers
// (fwd2_lds), so every pass works on the lines, rows and columns of both
// fields at once.  For a slab of sx planes the z pass has 2 sx N lines, the
// y pass 2 sx nk rows and the x stage 2 nk^2 columns, which fill a wide
// workgroup better than one field at a time, with half the barriers.  Same
// arithmetic, same order per field, as forward_pruned.
template <class T>
__host__ __device__ inline size_t fwd2_lds_bytes(int n, int nk, int sx) {
  return sizeof(cplx<T>) * (2 * size_t(sx) * nk * slab_row(n) + n);
}

template <class T>
__device__ inline SlabLds<T> fwd2_lds(void* base, int n, int nk, int sx) {
  SlabLds<T> s;
  s.t1 = reinterpret_cast<cplx<T>*>(base);
  s.tw = s.t1 + 2 * size_t(sx) * nk * slab_row(n);
  s.cmap = nullptr;
  return s;
}

template <class T, int S, int D, int NT>
__device__ inline void column_fft_rows2(cplx<T>* a, int nf, int nk, int R, int pstride,
                                        int fstride) {
  const int nc = nk * nk;
  const unsigned inv = 0xffffffffu / unsigned(nk) + 1u;
  for (int c = threadIdx.x; c < nf * nc; c += NT) {
    const int f = c >= nc ? 1 : 0, cc = c - f * nc;
    const int kzi = int(__umulhi(unsigned(cc), inv)), kyi = cc - kzi * nk;
    cplx<T>* b = a + f * fstride + kzi * R + kyi;
    cplx<T> v[D];
#pragma unroll
    for (int k = 0; k < D; ++k) v[k] = b[k * pstride];
    Fft<T, S, D>::run(v);
#pragma unroll
    for (int k = 0; k < D; ++k) b[k * pstride] = v[k];
  }
}

template <class T, int S, int N, int NT>
__device__ inline void column_fft_rows2_tile(cplx<T>* a, int d, int nf, int nk, int R,
                                             int pstride, int fstride) {
  if constexpr (N % 12 == 0) if (d == 12) return column_fft_rows2<T, S, 12, NT>(a, nf, nk, R, pstride, fstride);
  if constexpr (N % 10 == 0) if (d == 10) return column_fft_rows2<T, S, 10, NT>(a, nf, nk, R, pstride, fstride);
  if constexpr (N % 9 == 0) if (d == 9) return column_fft_rows2<T, S, 9, NT>(a, nf, nk, R, pstride, fstride);
  if constexpr (N % 8 == 0) if (d == 8) return column_fft_rows2<T, S, 8, NT>(a, nf, nk, R, pstride, fstride);
  if constexpr (N % 6 == 0) if (d == 6) return column_fft_rows2<T, S, 6, NT>(a, nf, nk, R, pstride, fstride);
  if constexpr (N % 5 == 0) if (d == 5) return column_fft_rows2<T, S, 5, NT>(a, nf, nk, R, pstride, fstride);
  if constexpr (N % 4 == 0) if (d == 4) return column_fft_rows2<T, S, 4, NT>(a, nf, nk, R, pstride, fstride);
  if constexpr (N % 3 == 0) if (d == 3) return column_fft_rows2<T, S, 3, NT>(a, nf, nk, R, pstride, fstride);
  if constexpr (N % 2 == 0) if (d == 2) return column_fft_rows2<T, S, 2, NT>(a, nf, nk, R, pstride, fstride);
}

template <class T, int S, int N, int OPT, int NT = kThreads, int KM = -1, class Load>
__device__ __forceinline__ void forward_pruned_joint(const Load& ld, int nf_active, int kmax_rt,
                                                     int sx, const int (&gdesc)[OPT], int nout,
                                                     cplx<T> (&acc)[2][OPT],
                                                     const SlabLds<T>& L) {
  constexpr int R = slab_row(N);
  const int kmax = KM >= 0 ? KM : kmax_rt;
  const int nk = 2 * kmax + 1, M = N / sx, pstride = nk * R, fstride = sx * pstride;
  const int tid = threadIdx.x;
  const int nl = sx * N, nr = sx * nk;
  int ox[OPT];
#pragma unroll
  for (int t = 0; t < OPT; ++t) {
    const int kxm = gdesc[t] & 0xff, kyi = (gdesc[t] >> 8) & 0xff, kzi = gdesc[t] >> 16;
    ox[t] = ((kxm % sx) * pstride + kzi * R + kyi) | (kxm << 24);
  }
  for (int x2 = 0; x2 < M; ++x2) {
    // z pass: line (f, xs, y) -> rows (f, xs, kz)
    for (int l = tid; l < nf_active * nl; l += NT) {
      const int f = l >= nl ? 1 : 0, lf = l - f * nl;
      const int xs = lf / N, y = lf - xs * N, x = x2 + M * xs;
      cplx<T> v[N];
#pragma unroll
      for (int z = 0; z < N; ++z) v[z] = ld(f, x, y, z);
      Fft<T, S, N>::run(v);
      cplx<T>* out = L.t1 + f * fstride + xs * pstride + y;
#pragma unroll
      for (int z = 0; z < N; ++z) {
        const int kz = (z <= N / 2) ? z : z - N;
        if (kz >= -kmax && kz <= kmax) out[(kz + kmax) * R] = v[z];
      }
    }
    __syncthreads();
    // y pass: row (f, xs, kz) in place; the kept ky land at the row's start
    for (int l = tid; l < nf_active * nr; l += NT) {
      const int f = l >= nr ? 1 : 0;
      cplx<T>* row = L.t1 + f * fstride + (l - f * nr) * R;
      cplx<T> v[N];
#pragma unroll
      for (int y = 0; y < N; ++y) v[y] = row[y];
      Fft<T, S, N>::run(v);
#pragma unroll
      for (int y = 0; y < N; ++y) {
        const int ky = (y <= N / 2) ? y : y - N;
        if (ky >= -kmax && ky <= kmax) row[ky + kmax] = v[y];
      }
    }
    __syncthreads();
    column_fft_rows2_tile<T, S, N, NT>(L.t1, sx, nf_active, nk, R, pstride, fstride);
    if (sx > 1) __syncthreads();
#pragma unroll
    for (int t = 0; t < OPT; ++t) {
      const int o = tid + t * NT;
      if (o < nout) {
        const cplx<T> tw = L.tw[((ox[t] >> 24) * x2) % N];
        acc[0][t] = cfma(tw, L.t1[ox[t] & 0xffffff], acc[0][t]);
        if (nf_active > 1) acc[1][t] = cfma(tw, L.t1[fstride + (ox[t] & 0xffffff)], acc[1][t]);
      }
    }
    __syncthreads();  // the next z pass overwrites the rows
  }
}

// Inverse transform of NF coefficient vectors given on a sphere whose
// entries are grouped in (ky, kz) columns: column c covers entries
// [cstart[c], cstart[c+1]) with packed (ky + kmax) | (kz + kmax) << 8 in
// cdesc[c] and consecutive, ascending kx values ckx[e].  Coef(f, e) returns
// entry e of item f; Store(f, x, y, z, v) receives the synthesised grid
// value.  L is the inverse layout (inv_lds) with its twiddles filled; the
// first barrier inside orders them before their use.  Requires fewer than
// 2^16 entries, and column lengths and N below 64.
//
// The x transform uses the same split as the forward one (sx divides N,
// group x2 = planes x2 + M xs): per (ky, kz) slot and residue q < sx,
// Z(q) = sum_{kx = q mod sx} c(kx) w_N^{kx x2} (zero for slots outside the
// sphere), then a length-sx FFT over q gives the group's planes.
// KO >= 0 fixes kmax = KO at compile time (see korb_win).
template <class T, int N, int NF, int KO = -1, class Coef, class Store>
__device__ inline void inverse_sphere(const Coef& cf, const Store& st, int nf_active,
                                      int kmax_rt, int sx, int ncol, const int* cdesc,
                                      const int* cstart, const int* ckx, const SlabLds<T>& L) {
  constexpr int R = slab_row(N);
  const int kmax = KO >= 0 ? KO : kmax_rt;
  const int nk = 2 * kmax + 1, nc = nk * nk, M = N / sx;
  const int tid = threadIdx.x;
  for (int s = tid; s < nc; s += kThreads) L.cmap[s] = 0;
  __syncthreads();
  for (int c = tid; c < ncol; c += kThreads) {
    const int d = cdesc[c], e0 = cstart[c];
    int kxm = ckx[e0] % N;
    if (kxm < 0) kxm += N;
    L.cmap[(d >> 8) * nk + (d & 0xff)] = e0 | ((cstart[c + 1] - e0) << 16) | (kxm << 22);
  }
  __syncthreads();
  for (int x2 = 0; x2 < M; ++x2) {
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      if (f >= nf_active) break;
      // x stage: residue sums for every slot s = kzi * nk + kyi
      for (int l = tid; l < sx * nc; l += kThreads) {
        const int q = l / nc, sl = l - q * nc;
        const int m = L.cmap[sl];
        cplx<T> s = {T(0), T(0)};
        if (m != 0) {
          const int e0 = m & 0xffff, e1 = e0 + ((m >> 16) & 63);
          int kxm = (m >> 22) & 63;
          const int skip = (q - kxm % sx + sx) % sx;
          kxm += skip;
          for (int e = e0 + skip; e < e1; e += sx) {
            s = cfma(cf(f, e), L.tw[(kxm * x2) % N], s);
            kxm += sx;
          }
        }
        const int kzi = sl / nk;
        L.t1[(q * nk + kzi) * R + (sl - kzi * nk)] = s;
      }
      __syncthreads();
      column_fft_rows_tile<T, 1, N>(L.t1, sx, nk, R, nk * R);
      if (sx > 1) __syncthreads();
      // y stage: line (xs, kz), expanded in place from nk to N values
      for (int l = tid; l < sx * nk; l += kThreads) {
        cplx<T>* row = L.t1 + l * R;
        cplx<T> v[N];
#pragma unroll
        for (int y = 0; y < N; ++y) {
          const int ky = (y <= N / 2) ? y : y - N;
          v[y] = (ky >= -kmax && ky <= kmax) ? row[ky + kmax] : cplx<T>{T(0), T(0)};
        }
        Fft<T, 1, N>::run(v);
#pragma unroll
        for (int y = 0; y < N; ++y) row[y] = v[y];
      }
      __syncthreads();
      // z stage: line (xs, y)
      for (int l = tid; l < sx * N; l += kThreads) {
        const int xs = l / N, y = l - xs * N, x = x2 + M * xs;
        cplx<T> v[N];
#pragma unroll
        for (int z = 0; z < N; ++z) {
          const int kz = (z <= N / 2) ? z : z - N;
          v[z] = (kz >= -kmax && kz <= kmax) ? L.t1[(xs * nk + kz + kmax) * R + y]
                                             : cplx<T>{T(0), T(0)};
        }
        Fft<T, 1, N>::run(v);
#pragma unroll
        for (int z = 0; z < N; ++z) st(f, x, y, z, v[z]);
      }
      __syncthreads();  // the next x stage overwrites the rows
    }
  }
}

// Block-wide sum of a double (deterministic order), result valid in thread 0.
__device__ inline double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += red[k];
  __syncthreads();
  return s;
}

// ---- partial sums by auxiliary cutoff shell ---------------------------------
// Internal cutoff extrapolation: nested auxiliary spheres E_aux / alpha^(n-1),
// n = 1..nb; shell[k] = the number of those spheres that contain auxiliary
// vector k (1..nb).  A (G, G') term of a Coulomb-weighted sum belongs to the
// energy of sphere n iff both vectors lie in it, so it is binned at
// min(shell(G), shell(G')) - 1 and the energy of sphere n is the sum of bins
// n-1 .. nb-1.
constexpr int kMaxShells = 8;

struct ShellBins {
  const signed char* shell = nullptr;  // [n_g] (nullptr: no binning)
  int nb = 0;                          // 1..kMaxShells
  double* out = nullptr;               // [rows][nb] per-row bin sums
};

// Adds x into bin b (0 <= b < kMaxShells) without indexing a register array.
__device__ __forceinline__ void bin_add(double (&sb)[kMaxShells], int b, double x) {
#pragma unroll
  for (int k = 0; k < kMaxShells; ++k) sb[k] += (k == b) ? x : 0.0;
}

// Block-wide sums of the kMaxShells bins (deterministic order), valid in
// thread 0; red holds (blockDim.x / 64) * kMaxShells doubles.
__device__ inline void block_sum_bins(double (&sb)[kMaxShells], double* red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kMaxShells; ++k) {
    double v = sb[k];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) red[w * kMaxShells + k] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < kMaxShells; ++k) {
      double s = 0.0;
      for (int q = 0; q < (int)(blockDim.x >> 6); ++q) s += red[q * kMaxShells + k];
      sb[k] = s;
    }
  }
  __syncthreads();
}

}  // namespace ltmp2
