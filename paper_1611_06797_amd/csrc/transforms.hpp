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

template <class T>
struct SlabLds {
  cplx<T>* t1;  // [SX][nk][n + 1]
  cplx<T>* t2;  // [SX][nk][nk]
  cplx<T>* tw;  // [n]
};

template <class T>
__host__ __device__ inline size_t slab_lds_bytes(int n, int nk, int sx) {
  return sizeof(cplx<T>) * (size_t(sx) * nk * (n + 1) + size_t(sx) * nk * nk + n);
}

template <class T>
__device__ inline SlabLds<T> slab_lds(void* base, int n, int nk, int sx) {
  SlabLds<T> s;
  s.t1 = reinterpret_cast<cplx<T>*>(base);
  s.t2 = s.t1 + size_t(sx) * nk * (n + 1);
  s.tw = s.t2 + size_t(sx) * nk * nk;
  return s;
}

// exp(S 2 pi i e / n) for e = 0..n-1 into shared memory
template <class T, int S>
__device__ inline void fill_twiddles(cplx<T>* tw, int n) {
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    cs v = unit_root(e, n);
    tw[e] = {T(v.c), T(S * v.s)};
  }
}

// Forward pruned transform of NF fields.  Load(f, x, y, z) returns the
// field value; acc[f][t] accumulates output o = threadIdx.x + t * kThreads
// (o < nout) whose packed descriptor is gdesc[t] (pre-loaded by the caller).
template <class T, int S, int N, int NF, int OPT, class Load>
__device__ inline void forward_pruned(const Load& ld, int nf_active, int kmax, int sx,
                                      const int (&gdesc)[OPT], int nout,
                                      cplx<T> (&acc)[NF][OPT], const SlabLds<T>& L) {
  const int nk = 2 * kmax + 1;
  const int tid = threadIdx.x;
  for (int x0 = 0; x0 < N; x0 += sx) {
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      if (f >= nf_active) break;
      // z pass: line (xs, y)
      for (int l = tid; l < sx * N; l += kThreads) {
        const int xs = l / N, y = l - xs * N, x = x0 + xs;
        if (x >= N) continue;
        cplx<T> v[N];
#pragma unroll
        for (int z = 0; z < N; ++z) v[z] = ld(f, x, y, z);
        Fft<T, S, N>::run(v);
#pragma unroll
        for (int z = 0; z < N; ++z) {
          const int kz = (z <= N / 2) ? z : z - N;
          if (kz >= -kmax && kz <= kmax) L.t1[(xs * nk + kz + kmax) * (N + 1) + y] = v[z];
        }
      }
      __syncthreads();
      // y pass: line (xs, kz)
      for (int l = tid; l < sx * nk; l += kThreads) {
        const int xs = l / nk, kzi = l - xs * nk;
        if (x0 + xs >= N) continue;
        cplx<T> v[N];
        const cplx<T>* src = L.t1 + (xs * nk + kzi) * (N + 1);
#pragma unroll
        for (int y = 0; y < N; ++y) v[y] = src[y];
        Fft<T, S, N>::run(v);
#pragma unroll
        for (int y = 0; y < N; ++y) {
          const int ky = (y <= N / 2) ? y : y - N;
          if (ky >= -kmax && ky <= kmax) L.t2[(xs * nk + ky + kmax) * nk + kzi] = v[y];
        }
      }
      __syncthreads();
      // x direct DFT into the owned outputs
#pragma unroll
      for (int t = 0; t < OPT; ++t) {
        const int o = tid + t * kThreads;
        if (o < nout) {
          const int kxm = gdesc[t] & 0xff, kyi = (gdesc[t] >> 8) & 0xff, kzi = gdesc[t] >> 16;
          cplx<T> a = acc[f][t];
          for (int xs = 0; xs < sx && x0 + xs < N; ++xs) {
            const int e = (kxm * (x0 + xs)) % N;
            a = cfma(L.tw[e], L.t2[(xs * nk + kyi) * nk + kzi], a);
          }
          acc[f][t] = a;
        }
      }
      __syncthreads();
    }
  }
}

// Inverse transform of NF coefficient vectors given on a sphere whose
// entries are grouped in (ky, kz) columns: column c covers entries
// [cstart[c], cstart[c+1]) with packed (ky + kmax) | (kz + kmax) << 8 in
// cdesc[c] and kx values ckx[e].  Coef(f, e) returns entry e of item f;
// Store(f, x, y, z, v) receives the synthesised grid value.  t2 must be
// zeroed once by the caller (entries outside the columns stay zero).
template <class T, int N, int NF, class Coef, class Store>
__device__ inline void inverse_sphere(const Coef& cf, const Store& st, int nf_active, int kmax,
                                      int sx, int ncol, const int* cdesc, const int* cstart,
                                      const int* ckx, const SlabLds<T>& L) {
  const int nk = 2 * kmax + 1;
  const int tid = threadIdx.x;
  for (int x0 = 0; x0 < N; x0 += sx) {
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      if (f >= nf_active) break;
      // x stage: column sums for each slab
      for (int l = tid; l < sx * ncol; l += kThreads) {
        const int xs = l / ncol, c = l - xs * ncol, x = x0 + xs;
        if (x >= N) continue;
        cplx<T> s = {T(0), T(0)};
        const int e1 = cstart[c + 1];
        for (int e = cstart[c]; e < e1; ++e) {
          int kxm = ckx[e] % N;
          if (kxm < 0) kxm += N;
          s = cfma(cf(f, e), L.tw[(kxm * x) % N], s);
        }
        const int d = cdesc[c];
        L.t2[(xs * nk + (d & 0xff)) * nk + (d >> 8)] = s;
      }
      __syncthreads();
      // y stage: line (xs, kz)
      for (int l = tid; l < sx * nk; l += kThreads) {
        const int xs = l / nk, kzi = l - xs * nk;
        if (x0 + xs >= N) continue;
        cplx<T> v[N];
#pragma unroll
        for (int y = 0; y < N; ++y) {
          const int ky = (y <= N / 2) ? y : y - N;
          v[y] = (ky >= -kmax && ky <= kmax) ? L.t2[(xs * nk + ky + kmax) * nk + kzi]
                                             : cplx<T>{T(0), T(0)};
        }
        Fft<T, 1, N>::run(v);
        cplx<T>* dst = L.t1 + (xs * nk + kzi) * (N + 1);
#pragma unroll
        for (int y = 0; y < N; ++y) dst[y] = v[y];
      }
      __syncthreads();
      // z stage: line (xs, y)
      for (int l = tid; l < sx * N; l += kThreads) {
        const int xs = l / N, y = l - xs * N, x = x0 + xs;
        if (x >= N) continue;
        cplx<T> v[N];
#pragma unroll
        for (int z = 0; z < N; ++z) {
          const int kz = (z <= N / 2) ? z : z - N;
          v[z] = (kz >= -kmax && kz <= kmax) ? L.t1[(xs * nk + kz + kmax) * (N + 1) + y]
                                             : cplx<T>{T(0), T(0)};
        }
        Fft<T, 1, N>::run(v);
#pragma unroll
        for (int z = 0; z < N; ++z) st(f, x, y, z, v[z]);
      }
      __syncthreads();
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

}  // namespace ltmp2
