// Spherical-design direction rule for the angular quadrature of the fast
// method (Sec. 4.4.1, 3D case: the half-sphere integral of the kernel's
// Fourier factors, approximated by a sum over directions).
//
// The integrand is even in the direction e, so a half-sphere rule {e_p} with
// equal weights 2 pi / m, extended antipodally, integrates every polynomial of
// degree <= t exactly (an antipodal spherical t-design) iff
//   sum_p Y_lm(e_p) = 0   for every real harmonic of even degree 2 <= l <= t - 1.
// The generator starts from the golden spiral and solves these equations (fewer
// equations than unknowns) by damped minimum-norm Gauss-Newton steps in the
// tangent planes of the points, with a fixed damping schedule, so that the
// result is a deterministic function of m.
#include <algorithm>
#include <cmath>
#include <vector>

#include "bz_internal.hpp"

namespace bz {
namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;

// Real orthonormal harmonics of the even degrees 2..L at unit vector e and
// their gradients in R^3.  Y = c Q_l^m(z) Re/Im (x + i y)^m with
// Q_l^m = P_l^m / (1 - z^2)^(m/2) (a polynomial in z), by the recurrence
// Q_m^m = (2m-1)!!, Q_{m+1}^m = (2m+1) z Q_m^m,
// (l - m) Q_l^m = (2l - 1) z Q_{l-1}^m - (l + m - 1) Q_{l-2}^m.
// Rows are ordered by l, then m, then (cos, sin) part; `row` receives the
// value and grad[3 * row ..] the gradient.
void harmonics(const double* e, int L, double* val, double* grad) {
  const double x = e[0], y = e[1], z = e[2];
  // (x + i y)^m and m (x + i y)^(m - 1) for m = 0..L
  std::vector<double> pr(L + 1), pi(L + 1), dr(L + 1), di(L + 1);
  pr[0] = 1.0;
  pi[0] = 0.0;
  dr[0] = di[0] = 0.0;
  for (int m = 1; m <= L; ++m) {
    dr[m] = m * pr[m - 1];
    di[m] = m * pi[m - 1];
    pr[m] = pr[m - 1] * x - pi[m - 1] * y;
    pi[m] = pr[m - 1] * y + pi[m - 1] * x;
  }
  // Q_l^m and dQ/dz for every (l, m), l <= L
  std::vector<double> Q((L + 1) * (L + 1)), D((L + 1) * (L + 1));
  for (int m = 0; m <= L; ++m) {
    double qmm = 1.0;
    for (int k = 1; k < 2 * m; k += 2) qmm *= k;
    double qa = qmm, da = 0.0;
    Q[m * (L + 1) + m] = qa;
    D[m * (L + 1) + m] = da;
    if (m == L) continue;
    double qb = (2 * m + 1) * z * qmm, db = (2 * m + 1) * qmm;
    Q[(m + 1) * (L + 1) + m] = qb;
    D[(m + 1) * (L + 1) + m] = db;
    for (int l = m + 2; l <= L; ++l) {
      const double qn = ((2 * l - 1) * z * qb - (l + m - 1) * qa) / (l - m);
      const double dn = ((2 * l - 1) * (qb + z * db) - (l + m - 1) * da) / (l - m);
      qa = qb;
      da = db;
      qb = qn;
      db = dn;
      Q[l * (L + 1) + m] = qb;
      D[l * (L + 1) + m] = db;
    }
  }
  int row = 0;
  for (int l = 2; l <= L; l += 2) {
    for (int m = 0; m <= l; ++m) {
      double ratio = 1.0;  // (l - m)! / (l + m)!
      for (int k = l - m + 1; k <= l + m; ++k) ratio /= k;
      double c = std::sqrt((2 * l + 1) / (4.0 * kPi) * ratio);
      if (m > 0) c *= std::sqrt(2.0);
      const double q = Q[l * (L + 1) + m], dq = D[l * (L + 1) + m];
      // cos part: W = Re w^m, dW/dx = Re(m w^(m-1)), dW/dy = Re(i m w^(m-1)) = -Im(m w^(m-1))
      val[row] = c * q * pr[m];
      grad[3 * row] = c * q * dr[m];
      grad[3 * row + 1] = -c * q * di[m];
      grad[3 * row + 2] = c * dq * pr[m];
      ++row;
      if (m > 0) {  // sin part: W = Im w^m, dW/dx = Im(m w^(m-1)), dW/dy = Re(m w^(m-1))
        val[row] = c * q * pi[m];
        grad[3 * row] = c * q * di[m];
        grad[3 * row + 1] = c * q * dr[m];
        grad[3 * row + 2] = c * dq * pi[m];
        ++row;
      }
    }
  }
}

int rows_for(int L) { return L * (L + 3) / 2; }

// Solve (A + mu I) x = b in place (A symmetric positive semi-definite, n x n,
// row-major) by Cholesky.  Returns false if a pivot is not positive.
bool chol_solve(std::vector<double>& A, int n, double mu, std::vector<double>& b) {
  for (int i = 0; i < n; ++i) A[size_t(i) * n + i] += mu;
  for (int j = 0; j < n; ++j) {
    double s = A[size_t(j) * n + j];
    for (int k = 0; k < j; ++k) s -= A[size_t(j) * n + k] * A[size_t(j) * n + k];
    if (!(s > 0.0)) return false;
    const double djj = std::sqrt(s);
    A[size_t(j) * n + j] = djj;
    for (int i = j + 1; i < n; ++i) {
      double t = A[size_t(i) * n + j];
      for (int k = 0; k < j; ++k) t -= A[size_t(i) * n + k] * A[size_t(j) * n + k];
      A[size_t(i) * n + j] = t / djj;
    }
  }
  for (int i = 0; i < n; ++i) {
    double t = b[i];
    for (int k = 0; k < i; ++k) t -= A[size_t(i) * n + k] * b[k];
    b[i] = t / A[size_t(i) * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double t = b[i];
    for (int k = i + 1; k < n; ++k) t -= A[size_t(k) * n + i] * b[k];
    b[i] = t / A[size_t(i) * n + i];
  }
  return true;
}

void tangent_frame(const double* e, double* t1, double* t2) {
  const double a[3] = {std::fabs(e[2]) < 0.9 ? 0.0 : 1.0, 0.0, std::fabs(e[2]) < 0.9 ? 1.0 : 0.0};
  t1[0] = e[1] * a[2] - e[2] * a[1];
  t1[1] = e[2] * a[0] - e[0] * a[2];
  t1[2] = e[0] * a[1] - e[1] * a[0];
  const double n = std::sqrt(t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2]);
  for (int k = 0; k < 3; ++k) t1[k] /= n;
  t2[0] = e[1] * t1[2] - e[2] * t1[1];
  t2[1] = e[2] * t1[0] - e[0] * t1[2];
  t2[2] = e[0] * t1[1] - e[1] * t1[0];
}

}  // namespace

int design_terms(int m) {
  int L = 0;
  while ((L + 2) * (L + 5) / 2 <= 2 * m - 3) L += 2;
  return L;
}

// Equal-weight design rule of m half-sphere directions; *t receives the
// degree reached (L + 1 for the largest L the iteration solves, 1 if none).
void rule_design(int m, std::vector<double>& d, std::vector<double>& w, int* t) {
  constexpr int kIters = 40;
  std::vector<double> e(3 * size_t(m));
  for (int L = design_terms(m); L >= 2; L -= 2) {
    rule_spiral(m, e, w);
    const int R = rows_for(L);
    std::vector<double> val(R), grad(3 * size_t(R)), r(R), J(size_t(R) * 2 * m), A(size_t(R) * R), tf(6 * size_t(m));
    bool ok = false;
    for (int k = 0; k < kIters; ++k) {
      std::fill(r.begin(), r.end(), 0.0);
      for (int p = 0; p < m; ++p) {
        const double* ep = &e[3 * size_t(p)];
        double* t1 = &tf[6 * size_t(p)];
        double* t2 = t1 + 3;
        tangent_frame(ep, t1, t2);
        harmonics(ep, L, val.data(), grad.data());
        for (int i = 0; i < R; ++i) {
          r[i] += val[i];
          const double* g = &grad[3 * size_t(i)];
          J[size_t(i) * 2 * m + 2 * p] = g[0] * t1[0] + g[1] * t1[1] + g[2] * t1[2];
          J[size_t(i) * 2 * m + 2 * p + 1] = g[0] * t2[0] + g[1] * t2[1] + g[2] * t2[2];
        }
      }
      double rn = 0.0;
      for (double x : r) rn += x * x;
      if (std::sqrt(rn) <= 1e-13 * std::sqrt(double(R))) {
        ok = true;
        break;
      }
      // d = -J^T (J J^T + mu I)^-1 r
      for (int i = 0; i < R; ++i)
        for (int j = 0; j <= i; ++j) {
          double s = 0.0;
          const double* ji = &J[size_t(i) * 2 * m];
          const double* jj = &J[size_t(j) * 2 * m];
          for (int c = 0; c < 2 * m; ++c) s += ji[c] * jj[c];
          A[size_t(i) * R + j] = A[size_t(j) * R + i] = s;
        }
      std::vector<double> y = r;
      if (!chol_solve(A, R, 1e-2 * std::pow(0.3, k), y)) break;
      for (int p = 0; p < m; ++p) {
        double d1 = 0.0, d2 = 0.0;
        for (int i = 0; i < R; ++i) {
          d1 -= J[size_t(i) * 2 * m + 2 * p] * y[i];
          d2 -= J[size_t(i) * 2 * m + 2 * p + 1] * y[i];
        }
        double* ep = &e[3 * size_t(p)];
        const double* t1 = &tf[6 * size_t(p)];
        const double* t2 = t1 + 3;
        double nn = 0.0;
        for (int c = 0; c < 3; ++c) {
          ep[c] += d1 * t1[c] + d2 * t2[c];
          nn += ep[c] * ep[c];
        }
        nn = std::sqrt(nn);
        for (int c = 0; c < 3; ++c) ep[c] /= nn;
      }
    }
    if (ok) {
      for (int p = 0; p < m; ++p)
        if (e[3 * size_t(p) + 2] < 0.0)
          for (int c = 0; c < 3; ++c) e[3 * size_t(p) + c] = -e[3 * size_t(p) + c];
      d = e;
      w.assign(m, 2.0 * kPi / m);
      *t = L + 1;
      return;
    }
  }
  rule_spiral(m, d, w);
  *t = 1;
}

// Antipodal design degree of any half-sphere rule: the largest odd t with
// sum_{p,q} w_p w_q P_l(e_p . e_q) / (sum w)^2 <= 1e-12 for every even
// 2 <= l <= t - 1 (addition theorem), checked up to l = 80.
int rule_degree(const std::vector<double>& d, const std::vector<double>& w) {
  const int m = int(w.size());
  double sw = 0.0;
  for (double x : w) sw += x;
  constexpr int kLmax = 80;
  std::vector<double> acc(kLmax + 1, 0.0);
  for (int p = 0; p < m; ++p)
    for (int q = 0; q < m; ++q) {
      double c = d[3 * size_t(p)] * d[3 * size_t(q)] + d[3 * size_t(p) + 1] * d[3 * size_t(q) + 1] +
                 d[3 * size_t(p) + 2] * d[3 * size_t(q) + 2];
      c = std::max(-1.0, std::min(1.0, c));
      const double ww = w[p] * w[q];
      double p0 = 1.0, p1 = c;
      for (int l = 2; l <= kLmax; ++l) {
        const double p2 = ((2 * l - 1) * c * p1 - (l - 1) * p0) / l;
        p0 = p1;
        p1 = p2;
        if ((l & 1) == 0) acc[l] += ww * p2;
      }
    }
  int t = 1;
  for (int l = 2; l <= kLmax; l += 2) {
    if (acc[l] / (sw * sw) > 1e-12) break;
    t = l + 1;
  }
  return t;
}

}  // namespace bz
