// Register-resident complex FFT codelets for gfx950.
//
// A length-N transform lives in a thread's registers as cx<T> x[N] and is
// evaluated by a compile-time mixed-radix Cooley-Tukey recursion (radix 2, 3
// and 4 butterflies) with every index and every twiddle a compile-time
// constant, so the whole transform unrolls into straight-line VALU code with
// literal coefficients.  Twiddles are evaluated in FP64 at compile time
// (exact octant reduction, then a Taylor series on |x| <= pi/4) and rounded
// once to T.
//
// Convention: fft<N, SIGN>(x) computes X_k = sum_n x_n exp(SIGN 2 pi i k n / N)
// in natural order, without scaling.
#pragma once

#include <hip/hip_runtime.h>

#define BZK_HD __host__ __device__ __forceinline__

namespace bzk {

template <typename T>
struct cx {
  T x, y;
};

constexpr double kPi = 3.14159265358979323846264338327950288;

// sin and cos of |x| <= pi/4 by Taylor series (terms below 1e-20).
constexpr double taylor_sin(double x) {
  double x2 = x * x, t = x, s = x;
  for (int i = 1; i < 12; ++i) {
    t *= -x2 / double((2 * i) * (2 * i + 1));
    s += t;
  }
  return s;
}
constexpr double taylor_cos(double x) {
  double x2 = x * x, t = 1.0, s = 1.0;
  for (int i = 1; i < 12; ++i) {
    t *= -x2 / double((2 * i - 1) * (2 * i));
    s += t;
  }
  return s;
}

// cos and sin of 2 pi num/den, reduced exactly with integer arithmetic to an
// angle in [0, pi/4].
struct SinCos {
  double c, s;
};
constexpr SinCos sincos_frac(long num, long den) {
  num %= den;
  if (num < 0) num += den;
  // 8 num / den = octant + frac, angle = 2 pi num/den = (pi/4) (octant + frac)
  long o8 = 8 * num;
  long oct = o8 / den;
  long rem = o8 - oct * den;  // frac = rem / den in [0,1)
  double c = 0, s = 0;
  // within the octant use the angle (pi/4) frac or (pi/4) (1 - frac)
  bool mirror = (oct % 2) == 1;
  double a = mirror ? (kPi / 4.0) * double(den - rem) / double(den)
                    : (kPi / 4.0) * double(rem) / double(den);
  double ca = taylor_cos(a), sa = taylor_sin(a);
  // base angle b = oct*pi/4 (+ a) or (oct+1)*pi/4 (- a)
  switch (oct) {
    case 0: c = ca; s = sa; break;            // a
    case 1: c = sa; s = ca; break;            // pi/2 - a
    case 2: c = -sa; s = ca; break;           // pi/2 + a
    case 3: c = -ca; s = sa; break;           // pi - a
    case 4: c = -ca; s = -sa; break;          // pi + a
    case 5: c = -sa; s = -ca; break;          // 3pi/2 - a
    case 6: c = sa; s = -ca; break;           // 3pi/2 + a
    default: c = ca; s = -sa; break;          // 2pi - a
  }
  return SinCos{c, s};
}

template <int N>
struct TwTable {
  double c[N], s[N];
  constexpr TwTable() : c(), s() {
    for (int k = 0; k < N; ++k) {
      SinCos v = sincos_frac(k, N);
      c[k] = v.c;
      s[k] = v.s;
    }
  }
};
template <int N>
inline constexpr TwTable<N> kTw{};

template <typename T>
BZK_HD cx<T> cadd(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
BZK_HD cx<T> csub(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
// multiply by SIGN * i
template <int SIGN, typename T>
BZK_HD cx<T> mul_si(cx<T> a) {
  if constexpr (SIGN > 0) return {-a.y, a.x};
  else return {a.y, -a.x};
}

// a * exp(SIGN 2 pi i k / N) for a compile-time-constant k after unrolling
template <int N, int SIGN, typename T>
BZK_HD cx<T> twiddle(cx<T> a, int k) {
  k %= N;
  if (k == 0) return a;
  if (4 * k == N) return mul_si<SIGN>(a);
  if (2 * k == N) return {-a.x, -a.y};
  if (4 * k == 3 * N) return mul_si<-SIGN>(a);
  const T c = T(kTw<N>.c[k]);
  const T s = T(SIGN * kTw<N>.s[k]);
  return {a.x * c - a.y * s, a.x * s + a.y * c};
}

template <int N, int SIGN, typename T>
BZK_HD void fft(cx<T> (&x)[N]);

template <int SIGN, typename T>
BZK_HD void dft2(cx<T> (&x)[2]) {
  cx<T> a = x[0], b = x[1];
  x[0] = cadd(a, b);
  x[1] = csub(a, b);
}

template <int SIGN, typename T>
BZK_HD void dft3(cx<T> (&x)[3]) {
  // X1,2 = a - (b+c)/2 +- SIGN i (sqrt(3)/2) (b - c)
  const T h = T(0.86602540378443864676372317075293618);
  cx<T> a = x[0], b = x[1], c = x[2];
  cx<T> t = cadd(b, c);
  cx<T> d = csub(b, c);
  cx<T> m = {a.x - T(0.5) * t.x, a.y - T(0.5) * t.y};
  cx<T> r = mul_si<SIGN>(cx<T>{h * d.x, h * d.y});
  x[0] = cadd(a, t);
  x[1] = cadd(m, r);
  x[2] = csub(m, r);
}

template <int SIGN, typename T>
BZK_HD void dft4(cx<T> (&x)[4]) {
  cx<T> s02 = cadd(x[0], x[2]), d02 = csub(x[0], x[2]);
  cx<T> s13 = cadd(x[1], x[3]), d13 = mul_si<SIGN>(csub(x[1], x[3]));
  x[0] = cadd(s02, s13);
  x[2] = csub(s02, s13);
  x[1] = cadd(d02, d13);
  x[3] = csub(d02, d13);
}

// N = N1 * N2: input index n = n1 + N1 n2, output index k = k2 + N2 k1.
template <int N1, int N2, int SIGN, typename T>
BZK_HD void fft_ct(cx<T> (&x)[N1 * N2]) {
  constexpr int N = N1 * N2;
  cx<T> a[N1][N2];
#pragma unroll
  for (int n1 = 0; n1 < N1; ++n1) {
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) a[n1][n2] = x[n1 + N1 * n2];
    fft<N2, SIGN>(a[n1]);
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) a[n1][k2] = twiddle<N, SIGN>(a[n1][k2], n1 * k2);
  }
#pragma unroll
  for (int k2 = 0; k2 < N2; ++k2) {
    cx<T> b[N1];
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) b[n1] = a[n1][k2];
    fft<N1, SIGN>(b);
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) x[k2 + N2 * k1] = b[k1];
  }
}

template <int N, int SIGN, typename T>
BZK_HD void fft(cx<T> (&x)[N]) {
  if constexpr (N == 1) {
  } else if constexpr (N == 2) {
    dft2<SIGN>(x);
  } else if constexpr (N == 3) {
    dft3<SIGN>(x);
  } else if constexpr (N == 4) {
    dft4<SIGN>(x);
  } else if constexpr (N % 3 == 0) {
    fft_ct<3, N / 3, SIGN>(x);
  } else if constexpr (N == 8) {
    fft_ct<2, 4, SIGN>(x);
  } else if constexpr (N % 4 == 0) {
    fft_ct<4, N / 4, SIGN>(x);
  } else {
    static_assert(N % 2 == 0, "fft: N must factor into 2, 3 and 4");
    fft_ct<2, N / 2, SIGN>(x);
  }
}

// The r-th input the transform's first stage consumes: fft_ct<N1, N2> first
// transforms the N1 subsequences x[n1 + N1 n2] (n1 = 0, 1, ...), so reading
// inputs in this order lets the first sub-transform start before the last
// input arrives.
template <int N>
constexpr int first_stage_order(int r) {
  if constexpr (N % 3 == 0 && N > 3) {
    return (r % (N / 3)) * 3 + r / (N / 3);
  } else if constexpr (N == 8) {
    return (r % 4) * 2 + r / 4;
  } else if constexpr (N % 4 == 0 && N > 4) {
    return (r % (N / 4)) * 4 + r / (N / 4);
  } else {
    return r;
  }
}

}  // namespace bzk
