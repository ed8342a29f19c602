// Register-resident complex FFT codelets for gfx950.
//
// A length-N transform lives in a thread's registers as cx<T> x[N] and is
// evaluated by a compile-time mixed-radix Cooley-Tukey recursion (radix 2, 3
// and 4 butterflies) with every index and every twiddle a compile-time
// constant, so the whole transform unrolls into straight-line VALU code with
// literal coefficients.  Twiddles are evaluated in FP64 at compile time
// (exact octant reduction, then a Taylor series on |x| <= pi/4), applied in
// scaled form (see ScaledTw: two FMAs per twiddle, the scale folded into the
// butterfly's own FMAs) and rounded once to T.  FP32 arithmetic instructions
// per transform: 52 (N = 8), 144 (16), 274 (24), 376 (32), 678 (48).
//
// Convention: fft<N, SIGN>(x) computes X_k = sum_n x_n exp(SIGN 2 pi i k n / N)
// in natural order, without scaling.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

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
  // X1,2 = a - (b+c)/2 +- SIGN i (sqrt(3)/2) (b - c); the last products fold into FMAs
  constexpr T h = T(SIGN * 0.86602540378443864676372317075293618);
  cx<T> a = x[0], b = x[1], c = x[2];
  cx<T> t = cadd(b, c);
  cx<T> d = csub(b, c);
  cx<T> m = {a.x - T(0.5) * t.x, a.y - T(0.5) * t.y};
  x[0] = cadd(a, t);
  x[1] = {m.x - h * d.y, m.y + h * d.x};
  x[2] = {m.x + h * d.y, m.y - h * d.x};
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

// Twiddle factors in scaled form: w = exp(SIGN 2 pi i k / N) = c (1 + i t) when
// |cos| >= |sin| (t = tan, c = cos), else c (u + i) (u = cot, c = sin), so that
// w b = c y with y = b + i t b (or u b + i b) costing two FMAs.  The factor c
// is not applied to y: the butterfly that consumes the twiddled value
// multiplies it in with FMAs (X = a + c y), which saves the separate complex
// multiplication (the FMA factorisation of Linzer and Feig, IBM J. Res. Dev.
// 1993).  Kinds: 0 = trivial (y = +-b or +-i b, c = 1), 1 = tangent, 2 =
// cotangent; at odd multiples of pi/4 t and u are exactly +-1 (y = b -+ i b...).
struct ScaledTw {
  int kind;  // 0 trivial, 1 tangent, 2 cotangent
  int rot;   // trivial kind: y = b * i^rot (SIGN folded in)
  double t;  // tan or cot
  double c;  // cos or sin (scale applied by the consumer)
};
constexpr double cabs_d(double v) { return v < 0 ? -v : v; }
template <int N, int SIGN>
constexpr ScaledTw scaled_tw(int k) {
  k %= N;
  if (k < 0) k += N;
  if (k == 0) return ScaledTw{0, 0, 0.0, 1.0};
  if (4 * k == N) return ScaledTw{0, SIGN > 0 ? 1 : 3, 0.0, 1.0};
  if (2 * k == N) return ScaledTw{0, 2, 0.0, 1.0};
  if (4 * k == 3 * N) return ScaledTw{0, SIGN > 0 ? 3 : 1, 0.0, 1.0};
  const double c = kTw<N>.c[k], s = SIGN * kTw<N>.s[k];
  const bool diag = (8 * k) % N == 0;  // odd multiple of pi/4: |c| = |s|
  if (cabs_d(c) >= cabs_d(s) || diag) {
    const double t = diag ? (s / c > 0 ? 1.0 : -1.0) : s / c;
    return ScaledTw{1, 0, t, c};
  }
  return ScaledTw{2, 0, c / s, s};
}
template <int N, int SIGN>
struct ScaledTable {
  ScaledTw v[N];
  constexpr ScaledTable() : v() {
    for (int k = 0; k < N; ++k) v[k] = scaled_tw<N, SIGN>(k);
  }
};
template <int N, int SIGN>
inline constexpr ScaledTable<N, SIGN> kScTw{};

// y of the scaled form for twiddle index K (compile time)
template <int N, int SIGN, int K, typename T>
BZK_HD cx<T> scaled_y(cx<T> b) {
  constexpr ScaledTw w = kScTw<N, SIGN>.v[((K % N) + N) % N];
  if constexpr (w.kind == 0) {
    if constexpr (w.rot == 0) return b;
    else if constexpr (w.rot == 1) return {-b.y, b.x};
    else if constexpr (w.rot == 2) return {-b.x, -b.y};
    else return {b.y, -b.x};
  } else if constexpr (w.kind == 1) {
    constexpr T t = T(w.t);
    return {b.x - t * b.y, b.y + t * b.x};
  } else {
    constexpr T u = T(w.t);
    return {u * b.x - b.y, u * b.y + b.x};
  }
}
template <int N, int SIGN, int K>
constexpr double scaled_c() { return kScTw<N, SIGN>.v[((K % N) + N) % N].c; }

// Radix-N1 butterfly of fft_ct over b[n1] = (sub-transform n1 at output k2),
// with the twiddles exp(SIGN 2 pi i n1 k2 / N) applied in scaled form.
template <int N1, int N, int SIGN, int K2, typename T>
BZK_HD void twiddled_dft(cx<T> (&b)[N1]) {
  if constexpr (K2 == 0) {
    fft<N1, SIGN>(b);
  } else if constexpr (N1 == 2) {
    const cx<T> y1 = scaled_y<N, SIGN, K2>(b[1]);
    constexpr T c1 = T(scaled_c<N, SIGN, K2>());
    const cx<T> a = b[0];
    b[0] = {a.x + c1 * y1.x, a.y + c1 * y1.y};
    b[1] = {a.x - c1 * y1.x, a.y - c1 * y1.y};
  } else if constexpr (N1 == 3) {
    // b' = c1 y1, c' = c2 y2 = c1 r y2: b' + c' = c1 (y1 + r y2), b' - c' = c1 (y1 - r y2)
    const cx<T> y1 = scaled_y<N, SIGN, K2>(b[1]);
    const cx<T> y2 = scaled_y<N, SIGN, 2 * K2>(b[2]);
    constexpr double c1d = scaled_c<N, SIGN, K2>(), c2d = scaled_c<N, SIGN, 2 * K2>();
    constexpr T r = T(c2d / c1d);
    constexpr T c1 = T(c1d), hc = T(0.5 * c1d);
    constexpr T g = T(SIGN * 0.86602540378443864676372317075293618 * c1d);
    const cx<T> sm = {y1.x + r * y2.x, y1.y + r * y2.y};
    const cx<T> df = {y1.x - r * y2.x, y1.y - r * y2.y};
    const cx<T> a = b[0];
    const cx<T> m = {a.x - hc * sm.x, a.y - hc * sm.y};
    b[0] = {a.x + c1 * sm.x, a.y + c1 * sm.y};
    b[1] = {m.x - g * df.y, m.y + g * df.x};
    b[2] = {m.x + g * df.y, m.y - g * df.x};
  } else {
    static_assert(N1 == 4, "twiddled butterflies of radix 2, 3 and 4");
    // A, B = x0 +- c2 y2; c1 y1 +- c3 y3 = c1 (y1 +- r y3), r = c3 / c1
    const cx<T> y1 = scaled_y<N, SIGN, K2>(b[1]);
    const cx<T> y2 = scaled_y<N, SIGN, 2 * K2>(b[2]);
    const cx<T> y3 = scaled_y<N, SIGN, 3 * K2>(b[3]);
    constexpr double c1d = scaled_c<N, SIGN, K2>();
    constexpr T c1 = T(c1d), c2 = T(scaled_c<N, SIGN, 2 * K2>());
    constexpr T r = T(scaled_c<N, SIGN, 3 * K2>() / c1d);
    constexpr T sc1 = T(SIGN * c1d);
    const cx<T> a = b[0];
    const cx<T> A = {a.x + c2 * y2.x, a.y + c2 * y2.y};
    const cx<T> B = {a.x - c2 * y2.x, a.y - c2 * y2.y};
    const cx<T> zp = {y1.x + r * y3.x, y1.y + r * y3.y};
    const cx<T> zm = {y1.x - r * y3.x, y1.y - r * y3.y};
    b[0] = {A.x + c1 * zp.x, A.y + c1 * zp.y};
    b[2] = {A.x - c1 * zp.x, A.y - c1 * zp.y};
    // SIGN i c1 zm = sc1 (-zm.y, zm.x)
    b[1] = {B.x - sc1 * zm.y, B.y + sc1 * zm.x};
    b[3] = {B.x + sc1 * zm.y, B.y - sc1 * zm.x};
  }
}

template <int I, int E, typename F>
BZK_HD void static_for(F&& f) {
  if constexpr (I < E) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, E>(f);
  }
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
  }
  static_for<0, N2>([&](auto kc) {
    constexpr int k2 = decltype(kc)::value;
    cx<T> b[N1];
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) b[n1] = a[n1][k2];
    twiddled_dft<N1, N, SIGN, k2>(b);
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) x[k2 + N2 * k1] = b[k1];
  });
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
