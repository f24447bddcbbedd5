// Split-BF16x3 contractions on 128 x 128 tiles (v_mfma_f32_16x16x32_bf16).
//
// Operands are split once, by k_split3, into hi = bf16(x) and lo = bf16(x - hi)
// and stored k-octet-blocked: element (k, m) of an operand lives at
// [k / 8][m][k % 8], so that sixteen bytes hold the eight consecutive k one
// MFMA lane needs.  A tile product is hi*hi + hi*lo + lo*hi accumulated in
// FP32 (the lo*lo term is below the FP32 rounding of the sum; Henry, Tang,
// Heinecke, ARITH 2019).
//
// Per K-slice of 32 the workgroup stages the four split operand tiles in
// shared memory ([128][32 + 8] bf16 each, k-contiguous per row) with 16-byte
// loads and stores, in two alternating buffers: while the matrix cores work
// on one slice, the next is fetched into registers and stored into the other
// buffer (one barrier per slice).  Four waves each own a 64 x 64 quarter of the tile
// (4 x 4 blocks of 16 x 16); accumulator element v of lane l of a block is
// D[4 (l / 16) + v][l % 16].  Tiles are assigned so that the workgroups
// resident on one XCD (dispatch is round-robin over the 8 XCDs) share their
// operand strips in that XCD's L2.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace ltmp2 {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr int T3 = 128, T3_K = 32, T3_KP = 40;

struct Split3Tile {
  __bf16 ah[T3][T3_KP], al[T3][T3_KP], bh[T3][T3_KP], bl[T3][T3_KP];
};

// One split operand: rows m of k-octet o at hi/lo + (o * ld + m) * 8.
struct Op3 {
  const __bf16* hi;
  const __bf16* lo;
  long ld;
};

// dst[(o0 + k / 8) * ldo + m][k % 8] = split(s_k src[k][m]) for k < Kpad,
// m < M, with s_k = sqrt(sk[k]) (mode 2), sk[k] (mode 1) or 1 (mode 0), and
// zero for k >= K.  One thread per (octet, m).
__global__ __launch_bounds__(256) void k_split3(const float* __restrict__ src, long lds, int K,
                                               int Kpad, int M, long ldo,
                                               const double* __restrict__ sk, int mode,
                                               __bf16* __restrict__ hi, __bf16* __restrict__ lo,
                                               long o0) {
  const long t = long(blockIdx.x) * 256 + threadIdx.x;
  if (t >= long(Kpad / 8) * M) return;
  const int oc = int(t / M), m = int(t - long(oc) * M);
  bf16x8 vh, vl;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int k = 8 * oc + u;
    float x = 0.f;
    if (k < K) {
      const double s = mode == 2 ? sqrt(sk[k]) : mode == 1 ? sk[k] : 1.0;
      x = float(s * double(src[long(k) * lds + m]));
    }
    const __bf16 b = (__bf16)x;
    vh[u] = b;
    vl[u] = (__bf16)(x - (float)b);
  }
  const long d = ((o0 + oc) * ldo + m) * 8;
  *reinterpret_cast<bf16x8*>(hi + d) = vh;
  *reinterpret_cast<bf16x8*>(lo + d) = vl;
}

// Thread t fetches k-octet oct + (t / 64), rows m0 + (t % 64) and
// m0 + 64 + (t % 64), hi and lo (4 x 16 bytes).
__device__ __forceinline__ void m3_fetch(const Op3& a, long m0, long oct, u32x4 (&r)[4]) {
  const int o = threadIdx.x >> 6, mm = threadIdx.x & 63;
  const long base = ((oct + o) * a.ld + m0 + mm) * 8;
  r[0] = *reinterpret_cast<const u32x4*>(a.hi + base);
  r[1] = *reinterpret_cast<const u32x4*>(a.hi + base + 64 * 8);
  r[2] = *reinterpret_cast<const u32x4*>(a.lo + base);
  r[3] = *reinterpret_cast<const u32x4*>(a.lo + base + 64 * 8);
}

__device__ __forceinline__ void m3_store(__bf16 (*hi)[T3_KP], __bf16 (*lo)[T3_KP],
                                         const u32x4 (&r)[4]) {
  const int o = threadIdx.x >> 6, mm = threadIdx.x & 63;
  const int kc = 8 * o;
  *reinterpret_cast<u32x4*>(&hi[mm][kc]) = r[0];
  *reinterpret_cast<u32x4*>(&hi[mm + 64][kc]) = r[1];
  *reinterpret_cast<u32x4*>(&lo[mm][kc]) = r[2];
  *reinterpret_cast<u32x4*>(&lo[mm + 64][kc]) = r[3];
}

__device__ __forceinline__ void m3_mma(const Split3Tile& s, f32x4 (&acc)[4][4]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r0 = (wave >> 1) * 64 + (lane & 15), c0 = (wave & 1) * 64 + (lane & 15);
#pragma unroll
  for (int kh = 0; kh < T3_K / 32; ++kh) {
    const int kk = 32 * kh + 8 * (lane >> 4);
    bf16x8 bh[4], bl[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      bh[q] = *reinterpret_cast<const bf16x8*>(&s.bh[c0 + 16 * q][kk]);
      bl[q] = *reinterpret_cast<const bf16x8*>(&s.bl[c0 + 16 * q][kk]);
    }
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const bf16x8 ah = *reinterpret_cast<const bf16x8*>(&s.ah[r0 + 16 * p][kk]);
      const bf16x8 al = *reinterpret_cast<const bf16x8*>(&s.al[r0 + 16 * p][kk]);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        acc[p][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[q], acc[p][q], 0, 0, 0);
        acc[p][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[q], acc[p][q], 0, 0, 0);
        acc[p][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[q], acc[p][q], 0, 0, 0);
      }
    }
  }
}

// acc += sum over k-octets [oa, oa + Kpad / 8) of A and [ob, ...) of B on the
// tile rows m0 .. m0 + 127 of A and n0 .. n0 + 127 of B (Kpad a multiple of
// 32).  Ends with a barrier, so the buffers may be refilled at once.
__device__ __forceinline__ void m3_phase(const Op3& A, long m0, long oa, const Op3& B, long n0,
                                         long ob, int Kpad, Split3Tile (&s)[2],
                                         f32x4 (&acc)[4][4]) {
  constexpr int OCT = T3_K / 8;
  const int nks = Kpad / T3_K;
  if (nks <= 0) return;
  u32x4 ra[4], rb[4];
  m3_fetch(A, m0, oa, ra);
  m3_fetch(B, n0, ob, rb);
  m3_store(s[0].ah, s[0].al, ra);
  m3_store(s[0].bh, s[0].bl, rb);
  __syncthreads();
  for (int ks = 0; ks < nks; ++ks) {
    const bool more = ks + 1 < nks;
    if (more) {
      m3_fetch(A, m0, oa + OCT * (ks + 1), ra);
      m3_fetch(B, n0, ob + OCT * (ks + 1), rb);
    }
    m3_mma(s[ks & 1], acc);
    if (more) {
      // buffer (ks + 1) & 1 was last read in slice ks - 1, before the barrier
      Split3Tile& d = s[(ks + 1) & 1];
      m3_store(d.ah, d.al, ra);
      m3_store(d.bh, d.bl, rb);
    }
    __syncthreads();
  }
}

__device__ __forceinline__ void m3_zero(f32x4 (&acc)[4][4]) {
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[p][q] = f32x4{0.f, 0.f, 0.f, 0.f};
}

// chi(r, r') = G_occ(r, r') G_vir(r, r') (added to chi when accumulating the
// spin channels) from the split, sqrt-scaled orbitals
// (occupied k-octets [0, kpo / 8), virtual ones [kpo / 8, (kpo + kpv) / 8)):
// G_occ = sum_i (sqrt(f_i) psi_i)(r) (sqrt(f_i) psi_i)(r'), likewise G_vir.
// Tiles are the upper-triangular pairs of an n x n block (t = n / 128 per
// side) grouped in 8 x 8 super-tiles; the 64 workgroups of one super-tile run
// on one XCD.  Off-diagonal tiles are also written transposed.
__global__ __launch_bounds__(256, 2) void k_chi3(Op3 psi, int kpo, int kpv, int t,
                                                float* __restrict__ chi, long ldc,
                                                int accumulate) {
  __shared__ Split3Tile s[2];
  const int ts = (t + 7) / 8;
  const long nsuper = long(ts) * (ts + 1) / 2;
  const long b = blockIdx.x;
  const long sidx = (b / 512) * 8 + (b % 8);
  const int u = int((b / 8) % 64);
  if (sidx >= nsuper) return;
  int I, J;
  {
    int j = int((sqrt(8.0 * double(sidx) + 1.0) - 1.0) * 0.5);
    while (long(j) * (j + 1) / 2 > sidx) --j;
    while (long(j + 1) * (j + 2) / 2 <= sidx) ++j;
    J = j;
    I = int(sidx - long(j) * (j + 1) / 2);
  }
  const int bi = 8 * I + u / 8, bj = 8 * J + u % 8;
  if (bi > bj || bj >= t) return;
  const long m0 = long(bi) * T3, n0 = long(bj) * T3;
  f32x4 ao[4][4], av[4][4];
  m3_zero(ao);
  m3_zero(av);
  m3_phase(psi, m0, 0, psi, n0, 0, kpo, s, ao);
  m3_phase(psi, m0, kpo / 8, psi, n0, kpo / 8, kpv, s, av);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rb = (wave >> 1) * 64 + 4 * (lane >> 4), cb = (wave & 1) * 64 + (lane & 15);
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const f32x4 x = ao[p][q] * av[p][q];
      const long m = m0 + rb + 16 * p, n = n0 + cb + 16 * q;
#pragma unroll
      for (int v = 0; v < 4; ++v)
        chi[(m + v) * ldc + n] = accumulate ? chi[(m + v) * ldc + n] + x[v] : x[v];
      if (bi != bj) {
        f32x4* dt = reinterpret_cast<f32x4*>(&chi[n * ldc + m]);
        *dt = accumulate ? *dt + x : x;
      }
    }
}

// C[m][n] = rs(m) sum_k A(k, am0 + m) B(k, n) for m < M, n < N over Kpad / 8
// octets; rs(m) = rowscale[(m / rdiv) % rmod] or 1.  A rows must be readable
// up to am0 + (M rounded up to 128) and B rows up to N rounded up to 128.
// XCD x takes the contiguous range [x P, (x + 1) P) of the row-major tiles.
__global__ __launch_bounds__(256, 2) void k_mm3(Op3 A, long am0, Op3 B, float* __restrict__ C,
                                               long ldc, int M, int N, int Kpad,
                                               const double* __restrict__ rowscale, int rdiv,
                                               int rmod) {
  __shared__ Split3Tile s[2];
  const int tn = (N + T3 - 1) / T3;
  const long total = long((M + T3 - 1) / T3) * tn;
  const long per = (total + 7) / 8;
  const long tile = long(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (tile >= total) return;
  const long m0 = (tile / tn) * T3, n0 = (tile % tn) * T3;
  f32x4 acc[4][4];
  m3_zero(acc);
  m3_phase(A, am0 + m0, 0, B, n0, 0, Kpad, s, acc);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rb = (wave >> 1) * 64 + 4 * (lane >> 4), cb = (wave & 1) * 64 + (lane & 15);
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const long m = m0 + rb + 16 * p + v;
      if (m >= M) continue;
      const float rs = rowscale ? float(rowscale[(m / rdiv) % rmod]) : 1.f;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const long n = n0 + cb + 16 * q;
        if (n < N) C[m * ldc + n] = rs * acc[p][q][v];
      }
    }
}

}  // namespace ltmp2
