// Register-resident mixed-radix FFTs for the short lines of a cubic grid
// (n = 2^a 3^b 5^c <= 64), used by every transform of the LTMP2 path: the
// orbital and transformed-state syntheses (inverse), the overlap densities
// and the Fock-like pair products (forward), and both passes of the double
// Fourier transform of chi.
//
// One thread owns one line of N complex values in registers.  Lengths with
// coprime factors use the prime-factor algorithm (no twiddles between the
// factors); prime powers a decimation-in-time recursion N = R * M with R the
// leading radix.  All loops are unrolled at compile time, and twiddles are
// compile-time constants (own constexpr sine/cosine: octant reduction plus
// Taylor series, exact zeros and symmetric values at the multiples of pi/4).
#pragma once
#include <hip/hip_runtime.h>

#define LT_HD __host__ __device__ __forceinline__

namespace ltmp2 {

template <class T>
struct cplx {
  T x, y;
};

template <class T>
LT_HD cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <class T>
LT_HD cplx<T> cadd(cplx<T> a, cplx<T> b) {
  return {a.x + b.x, a.y + b.y};
}
template <class T>
LT_HD cplx<T> csub(cplx<T> a, cplx<T> b) {
  return {a.x - b.x, a.y - b.y};
}
// a * w for a twiddle w known at compile time after unrolling: the quarter
// turns (+-1, +-i) fold into sign changes and swaps.
template <class T>
LT_HD cplx<T> cmul_tw(cplx<T> a, cplx<T> w) {
  if (w.y == T(0) && w.x == T(1)) return a;
  if (w.y == T(0) && w.x == T(-1)) return {-a.x, -a.y};
  if (w.x == T(0) && w.y == T(1)) return {-a.y, a.x};
  if (w.x == T(0) && w.y == T(-1)) return {a.y, -a.x};
  return cmul(a, w);
}
template <class T>
LT_HD cplx<T> cfma(cplx<T> a, cplx<T> b, cplx<T> acc) {
  return {acc.x + a.x * b.x - a.y * b.y, acc.y + a.x * b.y + a.y * b.x};
}

// ---- compile-time trigonometry ---------------------------------------------
constexpr double kHalfPi = 1.57079632679489661923132169163975144;

constexpr double taylor_sin(double x) {
  double x2 = x * x, term = x, s = x;
  for (int k = 1; k <= 13; ++k) {
    term *= -x2 / double((2 * k) * (2 * k + 1));
    s += term;
  }
  return s;
}
constexpr double taylor_cos(double x) {
  double x2 = x * x, term = 1.0, s = 1.0;
  for (int k = 1; k <= 13; ++k) {
    term *= -x2 / double((2 * k - 1) * (2 * k));
    s += term;
  }
  return s;
}

struct cs {
  double c = 0.0, s = 0.0;
};

// cos and sin of 2 pi e / n, with exact reduction to |angle| <= pi / 4.
constexpr cs unit_root(long e, long n) {
  e %= n;
  if (e < 0) e += n;
  long q4 = 4 * e;                 // angle in quarter turns: q4 / n
  long quad = q4 / n;              // 0..3
  long rem = q4 - quad * n;        // angle within quadrant = (pi/2) rem / n
  double c = 0.0, s = 0.0;
  if (2 * rem <= n) {
    double a = kHalfPi * double(rem) / double(n);
    c = (rem == 0) ? 1.0 : taylor_cos(a);
    s = (rem == 0) ? 0.0 : taylor_sin(a);
  } else {
    double a = kHalfPi * double(n - rem) / double(n);
    c = taylor_sin(a);
    s = taylor_cos(a);
  }
  switch (quad) {
    case 0: return {c, s};
    case 1: return {-s, c};
    case 2: return {-c, -s};
    default: return {s, -c};
  }
}

// exp(S * 2 pi i e / n), S = -1 (forward) or +1 (inverse)
template <class T, int S>
LT_HD constexpr cplx<T> twiddle(long e, long n) {
  cs v = unit_root(e, n);
  return {T(v.c), T(S * v.s)};
}

constexpr int lead_radix(int n) {
  return (n % 4 == 0 && n != 8) ? 4 : (n % 2 == 0) ? 2 : (n % 3 == 0) ? 3 : (n % 5 == 0) ? 5 : n;
}

// Coprime split n = n1 * n2 for the prime-factor algorithm: n1 is the largest
// power of 2 dividing n, else the power of 3; 0 if n is a prime power.
constexpr int pfa_first(int n) {
  int p2 = 1;
  while (n % (2 * p2) == 0) p2 *= 2;
  if (p2 > 1 && p2 < n) return p2;
  int p3 = 1;
  while (n % (3 * p3) == 0) p3 *= 3;
  if (p3 > 1 && p3 < n) return p3;
  return 0;
}
// inverse of a modulo m (a, m coprime), by search (compile time only)
constexpr int inv_mod(int a, int m) {
  for (int t = 1; t < m; ++t)
    if ((a * t) % m == 1) return t;
  return m == 1 ? 0 : -1;
}

// ---- small DFT kernels ------------------------------------------------------
template <class T, int S, int R>
struct Dft;

template <class T, int S>
struct Dft<T, S, 1> {
  static LT_HD void run(cplx<T>*) {}
};

template <class T, int S>
struct Dft<T, S, 2> {
  static LT_HD void run(cplx<T>* a) {
    cplx<T> t = a[0];
    a[0] = cadd(t, a[1]);
    a[1] = csub(t, a[1]);
  }
};

template <class T, int S>
struct Dft<T, S, 3> {
  static LT_HD void run(cplx<T>* a) {
    constexpr T c = T(-0.5);
    constexpr T s = T(S * 0.866025403784438646763723170752936183);
    cplx<T> t1 = cadd(a[1], a[2]);
    cplx<T> t2 = csub(a[1], a[2]);
    cplx<T> m = {a[0].x + c * t1.x, a[0].y + c * t1.y};
    a[0] = cadd(a[0], t1);
    // m +- i s t2, each component one fused multiply-add
    a[1] = {m.x - s * t2.y, m.y + s * t2.x};
    a[2] = {m.x + s * t2.y, m.y - s * t2.x};
  }
};

template <class T, int S>
struct Dft<T, S, 4> {
  static LT_HD void run(cplx<T>* a) {
    cplx<T> t0 = cadd(a[0], a[2]);
    cplx<T> t1 = csub(a[0], a[2]);
    cplx<T> t2 = cadd(a[1], a[3]);
    cplx<T> t3 = csub(a[1], a[3]);
    cplx<T> it3 = {T(-S) * t3.y, T(S) * t3.x};  // S i t3
    a[0] = cadd(t0, t2);
    a[2] = csub(t0, t2);
    a[1] = cadd(t1, it3);
    a[3] = csub(t1, it3);
  }
};

template <class T, int S>
struct Dft<T, S, 5> {
  static LT_HD void run(cplx<T>* a) {
    constexpr cs w1 = unit_root(1, 5);
    constexpr cs w2 = unit_root(2, 5);
    constexpr T c1 = T(w1.c), c2 = T(w2.c);
    constexpr T s1 = T(S * w1.s), s2 = T(S * w2.s);
    cplx<T> b1 = cadd(a[1], a[4]), d1 = csub(a[1], a[4]);
    cplx<T> b2 = cadd(a[2], a[3]), d2 = csub(a[2], a[3]);
    cplx<T> m1 = {a[0].x + c1 * b1.x + c2 * b2.x, a[0].y + c1 * b1.y + c2 * b2.y};
    cplx<T> m2 = {a[0].x + c2 * b1.x + c1 * b2.x, a[0].y + c2 * b1.y + c1 * b2.y};
    // i (s1 d1 + s2 d2) and i (s2 d1 - s1 d2)
    cplx<T> r1 = {-(s1 * d1.y + s2 * d2.y), s1 * d1.x + s2 * d2.x};
    cplx<T> r2 = {-(s2 * d1.y - s1 * d2.y), s2 * d1.x - s1 * d2.x};
    a[0] = {a[0].x + b1.x + b2.x, a[0].y + b1.y + b2.y};
    a[1] = cadd(m1, r1);
    a[4] = csub(m1, r1);
    a[2] = cadd(m2, r2);
    a[3] = csub(m2, r2);
  }
};

// ---- recursive transforms ---------------------------------------------------
// Sizes with coprime factors n = n1 n2 use the prime-factor algorithm (Good
// 1958, Thomas 1963): input index (n2 i1 + n1 i2) mod n, output index
// (n2 <n2^-1>_{n1} k1 + n1 <n1^-1>_{n2} k2) mod n, and the n-point DFT becomes
// n2 DFTs of length n1 followed by n1 DFTs of length n2 with no twiddle
// factors in between.  Prime powers use decimation in time:
// X[k' + M q] = sum_r W_R^{r q} (W_N^{r k'} Y_r[k']),  Y_r = FFT_M(x[m R + r]).
template <class T, int S, int N>
struct Fft {
  static LT_HD void run(cplx<T>* x) {
    constexpr int R = lead_radix(N);
    constexpr int N1 = pfa_first(N);
    if constexpr (N1 > 0) {
      constexpr int N2 = N / N1;
      constexpr int T1 = inv_mod(N2 % N1, N1), T2 = inv_mod(N1 % N2, N2);
      cplx<T> y[N1][N2];
#pragma unroll
      for (int i2 = 0; i2 < N2; ++i2) {
        cplx<T> t[N1];
#pragma unroll
        for (int i1 = 0; i1 < N1; ++i1) t[i1] = x[(N2 * i1 + N1 * i2) % N];
        Fft<T, S, N1>::run(t);
#pragma unroll
        for (int k1 = 0; k1 < N1; ++k1) y[k1][i2] = t[k1];
      }
#pragma unroll
      for (int k1 = 0; k1 < N1; ++k1) {
        Fft<T, S, N2>::run(y[k1]);
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) x[(N2 * T1 * k1 + N1 * T2 * k2) % N] = y[k1][k2];
      }
    } else if constexpr (R == N) {
      Dft<T, S, N>::run(x);
    } else {
      constexpr int M = N / R;
      cplx<T> y[R][M];
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int m = 0; m < M; ++m) y[r][m] = x[m * R + r];
#pragma unroll
      for (int r = 0; r < R; ++r) Fft<T, S, M>::run(y[r]);
#pragma unroll
      for (int k = 0; k < M; ++k) {
        cplx<T> t[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (r * k == 0) {
            t[r] = y[r][k];
          } else {
            t[r] = cmul_tw(y[r][k], twiddle<T, S>(long(r) * k, N));
          }
        }
        Dft<T, S, R>::run(t);
#pragma unroll
        for (int q = 0; q < R; ++q) x[k + M * q] = t[q];
      }
    }
  }
};

template <class T, int S>
struct Fft<T, S, 1> {
  static LT_HD void run(cplx<T>*) {}
};

}  // namespace ltmp2
