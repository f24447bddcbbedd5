// Dense contractions of the LTMP2 path on CDNA matrix cores (FP64 MFMA).
//
//   k_gf_chi:  chi(r, r') = G_occ(r, r') * G_vir(r, r') for one 64 x 64 tile
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
// MFMA v_mfma_f64_16x16x4f64: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; accumulator element v of lane l is D[(l / 16) + 4 v][l % 16]
// (checked on gfx950 with a single-instruction probe).
#pragma once
#include <hip/hip_runtime.h>

namespace ltmp2 {

typedef double d4v __attribute__((ext_vector_type(4)));

constexpr int GB_M = 64, GB_N = 64, GB_K = 16, GB_PAD = 4;

// One K-phase of a 64 x 64 tile: acc += sum_k A[k][m0 + .] s_k B[k][n0 + .]
// for k in [0, K) of the row-major operands (row k of A starts at a + k lda).
__device__ inline void mfma_tile_phase(const double* __restrict__ a, long lda, int mvalid,
                                       const double* __restrict__ b, long ldb, int nvalid, int K,
                                       const double* __restrict__ sk, double (*As)[GB_M + GB_PAD],
                                       double (*Bs)[GB_N + GB_PAD], d4v (&acc)[2][2]) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int kr = tid >> 4, c4 = (tid & 15) * 4;
  for (int k0 = 0; k0 < K; k0 += GB_K) {
    const int kk = k0 + kr;
    double av[4] = {0, 0, 0, 0}, bv[4] = {0, 0, 0, 0};
    if (kk < K) {
      const double s = sk ? sk[kk] : 1.0;
      const double* ar = a + long(kk) * lda;
      const double* br = b + long(kk) * ldb;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (c4 + u < mvalid) av[u] = s * ar[c4 + u];
        if (c4 + u < nvalid) bv[u] = br[c4 + u];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      As[kr][c4 + u] = av[u];
      Bs[kr][c4 + u] = bv[u];
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < GB_K / 4; ++ks) {
      const int k = ks * 4 + (lane >> 4);
      const double a0 = As[k][wr * 32 + (lane & 15)];
      const double a1 = As[k][wr * 32 + 16 + (lane & 15)];
      const double b0 = Bs[k][wc * 32 + (lane & 15)];
      const double b1 = Bs[k][wc * 32 + 16 + (lane & 15)];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
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
__global__ __launch_bounds__(256) void k_gf_chi(const double* __restrict__ psi, long ld, int no,
                                               int nv, const double* __restrict__ fo,
                                               const double* __restrict__ fv,
                                               double* __restrict__ chi, long ldc) {
  __shared__ double As[GB_K][GB_M + GB_PAD];
  __shared__ double Bs[GB_K][GB_N + GB_PAD];
  __shared__ double Cs[GB_M][GB_N + 1];
  int bi, bj;
  tri_tile(blockIdx.x, bi, bj);
  const long m0 = long(bi) * GB_M, n0 = long(bj) * GB_N;
  d4v ao[2][2], av[2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      ao[p][q] = d4v{0, 0, 0, 0};
      av[p][q] = d4v{0, 0, 0, 0};
    }
  mfma_tile_phase(psi + m0, ld, GB_M, psi + n0, ld, GB_N, no, fo, As, Bs, ao);
  mfma_tile_phase(psi + long(no) * ld + m0, ld, GB_M, psi + long(no) * ld + n0, ld, GB_N, nv, fv,
                  As, Bs, av);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        Cs[wr * 32 + p * 16 + (lane >> 4) + 4 * v][wc * 32 + q * 16 + (lane & 15)] =
            ao[p][q][v] * av[p][q][v];
  __syncthreads();
  for (int e = tid; e < GB_M * GB_N; e += 256) {
    const int r = e >> 6, c = e & 63;
    chi[(m0 + r) * ldc + n0 + c] = Cs[r][c];
    if (bi != bj) chi[(n0 + r) * ldc + m0 + c] = Cs[c][r];
  }
}

// C[m][n] = rs(m) sum_k A[k][m] s_k B[k][n] for m < M, n < N;
// rs(m) = rowscale[(m / rdiv) % rmod] (or 1 if rowscale is null).
// Grid: (ceil(N / 64), ceil(M / 64)).
__global__ __launch_bounds__(256) void k_gemm_kmajor(const double* __restrict__ A, long lda,
                                                    const double* __restrict__ B, long ldb,
                                                    double* __restrict__ C, long ldc, int M, int N,
                                                    int K, const double* __restrict__ sk,
                                                    const double* __restrict__ rowscale, int rdiv,
                                                    int rmod) {
  __shared__ double As[GB_K][GB_M + GB_PAD];
  __shared__ double Bs[GB_K][GB_N + GB_PAD];
  const long m0 = long(blockIdx.y) * GB_M, n0 = long(blockIdx.x) * GB_N;
  d4v acc[2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[p][q] = d4v{0, 0, 0, 0};
  mfma_tile_phase(A + m0, lda, int(min(long(GB_M), M - m0)), B + n0, ldb,
                  int(min(long(GB_N), N - n0)), K, sk, As, Bs, acc);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const long m = m0 + wr * 32 + p * 16 + (lane >> 4) + 4 * v;
        const long n = n0 + wc * 32 + q * 16 + (lane & 15);
        if (m < M && n < N) {
          const double s = rowscale ? rowscale[(m / rdiv) % rmod] : 1.0;
          C[m * ldc + n] = s * acc[p][q][v];
        }
      }
}

}  // namespace ltmp2
