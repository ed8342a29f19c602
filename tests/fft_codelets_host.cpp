// Host check of the register FFT codelets (paper_2505_03360_amd/csrc/fft.hpp):
// every length the library instantiates, both signs, float and double, against
// a direct DFT summed in long double.  Prints one line per case:
//   N SIGN type max_rel_l2
#include <cmath>
#include <cstdio>
#include <random>

#include "fft.hpp"

using bzk::cx;

template <int N, int SIGN, typename T>
double worst(int trials) {
  std::mt19937_64 g(1000u * N + (SIGN > 0 ? 1 : 2) + sizeof(T));
  std::normal_distribution<double> nd;
  const long double pi = 3.14159265358979323846264338327950288L;
  double w = 0.0;
  for (int r = 0; r < trials; ++r) {
    cx<T> x[N];
    long double re[N], im[N];
    for (int i = 0; i < N; ++i) {
      x[i] = {T(nd(g)), T(nd(g))};
      re[i] = x[i].x;
      im[i] = x[i].y;
    }
    bzk::fft<N, SIGN>(x);
    long double num = 0, den = 0;
    for (int k = 0; k < N; ++k) {
      long double sx = 0, sy = 0;
      for (int n = 0; n < N; ++n) {
        const long double a = SIGN * 2.0L * pi * (long double)((long long)k * n % N) / N;
        sx += re[n] * cosl(a) - im[n] * sinl(a);
        sy += re[n] * sinl(a) + im[n] * cosl(a);
      }
      num += (x[k].x - sx) * (x[k].x - sx) + (x[k].y - sy) * (x[k].y - sy);
      den += sx * sx + sy * sy;
    }
    w = std::fmax(w, std::sqrt(double(num / den)));
  }
  return w;
}

template <int N>
void run() {
  printf("%d 1 f %.6e\n", N, worst<N, 1, float>(50));
  printf("%d -1 f %.6e\n", N, worst<N, -1, float>(50));
  printf("%d 1 d %.6e\n", N, worst<N, 1, double>(50));
  printf("%d -1 d %.6e\n", N, worst<N, -1, double>(50));
}

int main() {
  run<2>(); run<3>(); run<4>(); run<6>(); run<8>(); run<12>(); run<16>();
  run<24>(); run<32>(); run<48>(); run<64>(); run<96>();
  return 0;
}
