// Dense contractions of the LTMP2 path on CDNA matrix cores.
//
//   k_gf_chi:  chi(r, r') = G_occ(r, r') * G_vir(r, r') for one 64 x 64 tile
//              (added to chi when accumulating the spin channels)
//              pair (tile and its transpose; chi is symmetric for real
//              orbitals), with
//                G_occ = sum_i psi_i(r) exp((e_i - mu) tau) psi_i(r')
//                G_vir = sum_a psi_a(r) exp(-(e_a - mu) tau) psi_a(r')
//              both accumulated in the same kernel and multiplied in the
//              epilogue (G_vir(r', r) = G_vir(r, r') needs no transpose).
//   k_gemm_kmajor: C[m][n] = rs(m) sum_k A[k][m] s_k B[k][n], used for the
//              transformed-state product W = C Psi_v and for exporting
//              Green's-function rows.
//
// Arithmetic modes (template MODE):
//   kF64    v_mfma_f64_16x16x4f64, FP64 operands and accumulation
//   kF32    v_mfma_f32_16x16x4f32, FP32 operands and accumulation
//   kBF16x3 v_mfma_f32_16x16x32_bf16 on split operands x = hi + lo
//           (hi = bf16(x), lo = bf16(x - hi)), hi*hi + hi*lo + lo*hi with FP32
//           accumulation (Henry, Tang, Heinecke, ARITH 2019)
// Operand lanes: lane l supplies A[l % 16][k] and B[k][l % 16] for the
// k-slice (l / 16) of the instruction (one value for K = 4, eight consecutive
// values for K = 32).  Accumulator element v of lane l is
// D[(l / 16) + 4 v][l % 16] for the FP64 instruction and
// D[LTMP2_F32_ROW(l, v)][l % 16] for the FP32-accumulating ones (measured on
// gfx950 with single-instruction probes).
#pragma once
#include <hip/hip_runtime.h>

#include "modes.h"

#ifndef LTMP2_F32_ROW
#define LTMP2_F32_ROW(l, v) (4 * ((l) >> 4) + (v))
#endif

namespace ltmp2 {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

template <int MODE>
struct Mma;

template <>
struct Mma<kF64> {
  using T = double;
  using Acc = d4v;
  static constexpr int BK = 16;
  static __device__ __forceinline__ int row(int l, int v) { return (l >> 4) + 4 * v; }
  static __device__ __forceinline__ Acc zero() { return Acc{0, 0, 0, 0}; }
};
template <>
struct Mma<kF32> {
  using T = float;
  using Acc = f4v;
  static constexpr int BK = 16;
  static __device__ __forceinline__ int row(int l, int v) { return LTMP2_F32_ROW(l, v); }
  static __device__ __forceinline__ Acc zero() { return Acc{0, 0, 0, 0}; }
};
template <>
struct Mma<kBF16x3> {
  using T = float;
  using Acc = f4v;
  static constexpr int BK = 32;
  static __device__ __forceinline__ int row(int l, int v) { return LTMP2_F32_ROW(l, v); }
  static __device__ __forceinline__ Acc zero() { return Acc{0, 0, 0, 0}; }
};

constexpr int GB_M = 64, GB_N = 64, GB_PAD = 4;

// One K-slice step on the LDS tiles As[BK][64 + PAD], Bs[BK][64 + PAD].
template <int MODE>
__device__ __forceinline__ void mma_step(const typename Mma<MODE>::T (*As)[GB_M + GB_PAD],
                                         const typename Mma<MODE>::T (*Bs)[GB_N + GB_PAD],
                                         int lane, int wr, int wc,
                                         typename Mma<MODE>::Acc (&acc)[2][2]) {
  if constexpr (MODE == kBF16x3) {
    const int kb = 8 * (lane >> 4);
    bf8v ah[2], al[2], bh[2], bl[2];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        const float a = As[kb + t][wr * 32 + p * 16 + (lane & 15)];
        const float b = Bs[kb + t][wc * 32 + p * 16 + (lane & 15)];
        const __bf16 a1 = (__bf16)a, b1 = (__bf16)b;
        ah[p][t] = a1;
        al[p][t] = (__bf16)(a - (float)a1);
        bh[p][t] = b1;
        bl[p][t] = (__bf16)(b - (float)b1);
      }
    }
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        acc[p][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[p], bh[q], acc[p][q], 0, 0, 0);
        acc[p][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[p], bl[q], acc[p][q], 0, 0, 0);
        acc[p][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[p], bh[q], acc[p][q], 0, 0, 0);
      }
  } else {
#pragma unroll
    for (int ks = 0; ks < Mma<MODE>::BK / 4; ++ks) {
      const int k = ks * 4 + (lane >> 4);
      const auto a0 = As[k][wr * 32 + (lane & 15)];
      const auto a1 = As[k][wr * 32 + 16 + (lane & 15)];
      const auto b0 = Bs[k][wc * 32 + (lane & 15)];
      const auto b1 = Bs[k][wc * 32 + 16 + (lane & 15)];
      if constexpr (MODE == kF64) {
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
      } else {
        acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
      }
    }
  }
}

// One K-phase of a 64 x 64 tile: acc += sum_k A[k][m0 + .] s_k B[k][n0 + .]
// for k in [0, K) of the row-major operands (row k of A starts at a + k lda).
template <int MODE, class S>
__device__ inline void mfma_tile_phase(const typename Mma<MODE>::T* __restrict__ a, long lda,
                                       int mvalid, const typename Mma<MODE>::T* __restrict__ b,
                                       long ldb, int nvalid, int K, const S* __restrict__ sk,
                                       typename Mma<MODE>::T (*As)[GB_M + GB_PAD],
                                       typename Mma<MODE>::T (*Bs)[GB_N + GB_PAD],
                                       typename Mma<MODE>::Acc (&acc)[2][2]) {
  using T = typename Mma<MODE>::T;
  constexpr int BK = Mma<MODE>::BK;
  constexpr int PER = BK * GB_M / 256;        // elements per thread per tile
  constexpr int TPR = GB_M / PER;             // threads per tile row
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int kr = tid / TPR, cc = (tid % TPR) * PER;
  for (int k0 = 0; k0 < K; k0 += BK) {
    const int kk = k0 + kr;
    T av[PER], bv[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) av[u] = bv[u] = T(0);
    if (kk < K) {
      const T s = sk ? T(sk[kk]) : T(1);
      const T* ar = a + long(kk) * lda;
      const T* br = b + long(kk) * ldb;
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        if (cc + u < mvalid) av[u] = s * ar[cc + u];
        if (cc + u < nvalid) bv[u] = br[cc + u];
      }
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      As[kr][cc + u] = av[u];
      Bs[kr][cc + u] = bv[u];
    }
    __syncthreads();
    mma_step<MODE>(As, Bs, lane, wr, wc, acc);
    __syncthreads();
  }
}

// Upper-triangular tile index t -> (bi <= bj).
__device__ inline void tri_tile(long t, int& bi, int& bj) {
  int j = int((sqrt(8.0 * double(t) + 1.0) - 1.0) * 0.5);
  while (long(j) * (j + 1) / 2 > t) --j;
  while (long(j + 1) * (j + 2) / 2 <= t) ++j;
  bj = j;
  bi = int(t - long(j) * (j + 1) / 2);
}

// psi: [n_states][ld] real orbitals on the grid (occupied rows first).
// fo[i] = exp((e_i - mu) tau), fv[a] = exp(-(e_a - mu) tau).
// chi: [n_rp][ldc]; tiles cover n_rp = 64 * ntile rows and columns.
template <int MODE>
__global__ __launch_bounds__(256) void k_gf_chi(const typename Mma<MODE>::T* __restrict__ psi,
                                               long ld, int no, int nv,
                                               const double* __restrict__ fo,
                                               const double* __restrict__ fv,
                                               typename Mma<MODE>::T* __restrict__ chi, long ldc,
                                               int accumulate) {
  using T = typename Mma<MODE>::T;
  using Acc = typename Mma<MODE>::Acc;
  constexpr int BK = Mma<MODE>::BK;
  __shared__ T As[BK][GB_M + GB_PAD];
  __shared__ T Bs[BK][GB_N + GB_PAD];
  __shared__ T Cs[GB_M][GB_N + 1];
  int bi, bj;
  tri_tile(blockIdx.x, bi, bj);
  const long m0 = long(bi) * GB_M, n0 = long(bj) * GB_N;
  Acc ao[2][2], av[2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      ao[p][q] = Mma<MODE>::zero();
      av[p][q] = Mma<MODE>::zero();
    }
  mfma_tile_phase<MODE>(psi + m0, ld, GB_M, psi + n0, ld, GB_N, no, fo, As, Bs, ao);
  mfma_tile_phase<MODE>(psi + long(no) * ld + m0, ld, GB_M, psi + long(no) * ld + n0, ld, GB_N, nv,
                        fv, As, Bs, av);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        Cs[wr * 32 + p * 16 + Mma<MODE>::row(lane, v)][wc * 32 + q * 16 + (lane & 15)] =
            ao[p][q][v] * av[p][q][v];
  __syncthreads();
  for (int e = tid; e < GB_M * GB_N; e += 256) {
    const int r = e >> 6, c = e & 63;
    T* d = &chi[(m0 + r) * ldc + n0 + c];
    *d = accumulate ? *d + Cs[r][c] : Cs[r][c];
    if (bi != bj) {
      T* dt = &chi[(n0 + r) * ldc + m0 + c];
      *dt = accumulate ? *dt + Cs[c][r] : Cs[c][r];
    }
  }
}

// C[m][n] = rs(m) sum_k A[k][m] s_k B[k][n] for m < M, n < N;
// rs(m) = rowscale[(m / rdiv) % rmod] (or 1 if rowscale is null).
// Grid: (ceil(N / 64), ceil(M / 64)).
template <int MODE>
__global__ __launch_bounds__(256) void k_gemm_kmajor(const typename Mma<MODE>::T* __restrict__ A,
                                                    long lda,
                                                    const typename Mma<MODE>::T* __restrict__ B,
                                                    long ldb, typename Mma<MODE>::T* __restrict__ C,
                                                    long ldc, int M, int N, int K,
                                                    const double* __restrict__ sk,
                                                    const double* __restrict__ rowscale, int rdiv,
                                                    int rmod) {
  using T = typename Mma<MODE>::T;
  using Acc = typename Mma<MODE>::Acc;
  constexpr int BK = Mma<MODE>::BK;
  __shared__ T As[BK][GB_M + GB_PAD];
  __shared__ T Bs[BK][GB_N + GB_PAD];
  const long m0 = long(blockIdx.y) * GB_M, n0 = long(blockIdx.x) * GB_N;
  Acc acc[2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[p][q] = Mma<MODE>::zero();
  mfma_tile_phase<MODE>(A + m0, lda, int(min(long(GB_M), M - m0)), B + n0, ldb,
                        int(min(long(GB_N), N - n0)), K, sk, As, Bs, acc);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const long m = m0 + wr * 32 + p * 16 + Mma<MODE>::row(lane, v);
        const long n = n0 + wc * 32 + q * 16 + (lane & 15);
        if (m < M && n < N) {
          const T s = rowscale ? T(rowscale[(m / rdiv) % rmod]) : T(1);
          C[m * ldc + n] = s * acc[p][q][v];
        }
      }
}

}  // namespace ltmp2
