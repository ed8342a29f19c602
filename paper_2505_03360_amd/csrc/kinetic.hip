// Per-cell reductions over the velocity grid on gfx950, FP64: macroscopic
// fields and the L1 distance of the kinetic-to-fluid criterion (Sec. 2 and
// 3.3), and the parameters of the penalised IMEX update of the Boltzmann layer
// (Sec. 4.4, eq. (4.24)).
//
// One workgroup of 1024 threads per cell (16 waves per CU keep enough loads in
// flight for these HBM-bound sums).  Each thread accumulates a strided subset
// of the nodes, then the partial sums are combined across the wave
// (butterfly) and across the sixteen waves in a fixed order, so the result of
// a cell does not depend on the batch it is in.
#include "bz_internal.hpp"
#include "kinetic.hpp"

#include <cmath>

namespace {

constexpr int kThreads = 1024;
constexpr int kWaves = kThreads / 64;

__device__ __forceinline__ int live_cells(int ncells, const int32_t* ncells_dev) {
  int c = ncells;
  if (ncells_dev) {
    const int d = *ncells_dev;
    c = d < c ? d : c;
    if (c < 0) c = 0;
  }
  return c;
}

// Sum K per-thread values over the workgroup; every thread gets the totals.
// red holds K * (kWaves + 1) doubles: the per-wave partials, then the totals.
// Thread k sums the partials of value k over the waves in order (a fixed
// order), so that no thread holds more than K partials at once.
template <int K>
__device__ __forceinline__ void block_sum(double (&m)[K], double* red) {
  static_assert(K <= kThreads, "one thread per value");
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m[k] += __shfl_xor(m[k], o);
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) red[k * kWaves + wv] = m[k];
  __syncthreads();
  if (t < K) {
    double x = red[t * kWaves];
    for (int w = 1; w < kWaves; ++w) x += red[t * kWaves + w];
    red[K * kWaves + t] = x;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) m[k] = red[K * kWaves + k];
  __syncthreads();
}

struct MomArgs {
  int ncells;
  const int32_t* ncells_dev;
  const void* f;
  int f_fp32;
  const int32_t* idx;
  int scatter;
  double dv;
  double *rho, *u1, *u2, *u3, *T, *l1;
};

template <int N>
__device__ __forceinline__ double node(int i, double dv) { return double(i - N / 2) * dv; }

// rho = dv^3 sum f; u = sum v f / sum f; T = (sum |v|^2 f / sum f - |u|^2) / 3;
// l1 = dv^3 sum |f - rho (2 pi T)^(-3/2) exp(-|v - u|^2 / 2T)|.
template <int N>
__global__ __launch_bounds__(kThreads) void k_moments(MomArgs a) {
  constexpr int N3 = N * N * N;
  __shared__ double red[5 * (kWaves + 1)];
  const int c = blockIdx.x;
  if (c >= live_cells(a.ncells, a.ncells_dev)) return;
  const int t = threadIdx.x;
  const long row = a.idx ? long(a.idx[c]) : long(c);
  const size_t base = size_t(row) * N3;
  auto fval = [&](int j) -> double {
    return a.f_fp32 ? double(static_cast<const float*>(a.f)[base + j]) : static_cast<const double*>(a.f)[base + j];
  };
  double m[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  #pragma unroll 4
  for (int j = t; j < N3; j += kThreads) {
    const double v1 = node<N>(j / (N * N), a.dv), v2 = node<N>((j / N) % N, a.dv), v3 = node<N>(j % N, a.dv);
    const double fj = fval(j);
    m[0] += fj;
    m[1] += v1 * fj;
    m[2] += v2 * fj;
    m[3] += v3 * fj;
    m[4] += (v1 * v1 + v2 * v2 + v3 * v3) * fj;
  }
  block_sum<5>(m, red);
  const double w = a.dv * a.dv * a.dv;
  const double rho = w * m[0];
  const double u1 = m[1] / m[0], u2 = m[2] / m[0], u3 = m[3] / m[0];
  const double T = (m[4] / m[0] - (u1 * u1 + u2 * u2 + u3 * u3)) / 3.0;
  double l1 = 0.0;
  if (a.l1) {
    const double cm = rho / ((2.0 * M_PI * T) * sqrt(2.0 * M_PI * T));
    const double ia = 1.0 / (2.0 * T);
    double s[1] = {0.0};
    #pragma unroll 4
    for (int j = t; j < N3; j += kThreads) {
      const double d1 = node<N>(j / (N * N), a.dv) - u1, d2 = node<N>((j / N) % N, a.dv) - u2,
                   d3 = node<N>(j % N, a.dv) - u3;
      s[0] += fabs(fval(j) - cm * exp(-(d1 * d1 + d2 * d2 + d3 * d3) * ia));
    }
    block_sum<1>(s, red);
    l1 = w * s[0];
  }
  if (t == 0) {
    const long o = a.scatter ? row : long(c);
    if (a.rho) a.rho[o] = rho;
    if (a.u1) a.u1[o] = u1;
    if (a.u2) a.u2[o] = u2;
    if (a.u3) a.u3[o] = u3;
    if (a.T) a.T[o] = T;
    if (a.l1) a.l1[o] = l1;
  }
}

struct ParArgs {
  int ncells;
  const int32_t* ncells_dev;
  const int32_t* idx;
  const double* f;
  const double* tr;
  double dt, dv;
  double* par;  // [cell][kImexPar]
};

// Maxwellian parameters of f^n and of g = f^n - dt tr (whose invariants are
// U^{n+1}), and beta = 2 pi rho^{n+1}.
template <int N>
__global__ __launch_bounds__(kThreads) void k_imex_params(ParArgs a) {
  constexpr int N3 = N * N * N;
  __shared__ double red[10 * (kWaves + 1)];
  const int c = blockIdx.x;
  if (c >= live_cells(a.ncells, a.ncells_dev)) return;
  const int t = threadIdx.x;
  const long row = a.idx ? long(a.idx[c]) : long(c);
  const double* f = a.f + size_t(row) * N3;
  const double* tr = a.tr + size_t(row) * N3;
  double m[10] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  #pragma unroll 4
  for (int j = t; j < N3; j += kThreads) {
    const double v1 = node<N>(j / (N * N), a.dv), v2 = node<N>((j / N) % N, a.dv), v3 = node<N>(j % N, a.dv);
    const double e = v1 * v1 + v2 * v2 + v3 * v3;
    const double fj = f[j];
    const double gj = fj - a.dt * tr[j];
    m[0] += fj;
    m[1] += v1 * fj;
    m[2] += v2 * fj;
    m[3] += v3 * fj;
    m[4] += e * fj;
    m[5] += gj;
    m[6] += v1 * gj;
    m[7] += v2 * gj;
    m[8] += v3 * gj;
    m[9] += e * gj;
  }
  block_sum<10>(m, red);
  if (t == 0) {
    const double w = a.dv * a.dv * a.dv;
    double* p = a.par + size_t(c) * bzk::kImexPar;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const double* s = m + 5 * h;
      const double rho = w * s[0];
      const double u1 = s[1] / s[0], u2 = s[2] / s[0], u3 = s[3] / s[0];
      const double T = (s[4] / s[0] - (u1 * u1 + u2 * u2 + u3 * u3)) / 3.0;
      p[5 * h + 0] = rho / ((2.0 * M_PI * T) * sqrt(2.0 * M_PI * T));
      p[5 * h + 1] = u1;
      p[5 * h + 2] = u2;
      p[5 * h + 3] = u3;
      p[5 * h + 4] = 1.0 / (2.0 * T);
      if (h == 1) p[10] = 2.0 * M_PI * rho;
    }
    p[11] = 0.0;
  }
}

struct EsArgs {
  int ncells;
  const int32_t* ncells_dev;
  const int32_t* idx;
  int scatter;
  const double* f;          // the distribution (or stage value) whose moments define G
  const double* tr;         // IMEX: transport term (rows as f; null = none); PR stages: T_i
  const double* eps_cells;  // Knudsen number per row, or null
  double eps, dt;
  double beta, mu0, dv;
  double* out;
  const double* y;  // PR stage 2: y^n
  double* aux;      // PR: A (written by stage 2, read by the finish)
};

enum EsMode {
  ES_COLLIDE = 0,  // out = nu (G[f] - f)
  ES_IMEX = 1,     // out = c g + (1 - c) G, g = f - dt tr (stage solve when tr is null)
  ES_PR_STAGE2 = 2,  // g1 = Q_ES(Y1): out = y - dt T1 + dt a21 g1/eps, aux = y - dt/2 T1 + dt/(2 eps) g1
  ES_PR_FINISH = 3,  // g2 = Q_ES(Y2): out = aux - dt/2 T2 + dt/(2 eps) g2
};

constexpr double kPrA21 = 0.41421356237309505;  // 1 - 2 gamma = sqrt(2) - 1

// ES-BGK (Sec. 2.2), one cell per workgroup.
//   collision:  Q_ES = nu (G[f] - f), G from f's density, velocity and stress;
//   IMEX (Sec. 4.3): with g = f - dt tr and its rho, u, T (invariants of the
//     step), Sigma = a S(g) + (1 - a) rho (T I + u u), a = eps / (eps + (1 - beta)
//     nu dt), Theta = Sigma / rho - u u, and f^{n+1} = c g + (1 - c) G,
//     c = eps / (eps + nu dt).
// G = rho (2 pi)^(-3/2) det(Tau)^(-1/2) exp(-(v-u) Tau^-1 (v-u) / 2),
// Tau = (1 - beta) T I + beta Theta; nu = rho sqrt(T) / (mu0 (1 - beta)).
template <int N, int MODE>
__global__ __launch_bounds__(kThreads) void k_esbgk(EsArgs a) {
  constexpr bool IMEX = MODE == ES_IMEX;
  constexpr int N3 = N * N * N;
  __shared__ double red[10 * (kWaves + 1)];
  const int c = blockIdx.x;
  if (c >= live_cells(a.ncells, a.ncells_dev)) return;
  const int t = threadIdx.x;
  const long row = a.idx ? long(a.idx[c]) : long(c);
  const double* f = a.f + size_t(row) * N3;
  const double* tr = a.tr ? a.tr + size_t(row) * N3 : nullptr;
  auto h = [&](int j) -> double {
    if constexpr (IMEX) return tr ? f[j] - a.dt * tr[j] : f[j];
    else return f[j];
  };
  // sums of h, v h, v_a v_b h (11, 22, 33, 12, 13, 23)
  double m[10] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  #pragma unroll 4
  for (int j = t; j < N3; j += kThreads) {
    const double v1 = node<N>(j / (N * N), a.dv), v2 = node<N>((j / N) % N, a.dv), v3 = node<N>(j % N, a.dv);
    const double hj = h(j);
    m[0] += hj;
    m[1] += v1 * hj;
    m[2] += v2 * hj;
    m[3] += v3 * hj;
    m[4] += v1 * v1 * hj;
    m[5] += v2 * v2 * hj;
    m[6] += v3 * v3 * hj;
    m[7] += v1 * v2 * hj;
    m[8] += v1 * v3 * hj;
    m[9] += v2 * v3 * hj;
  }
  block_sum<10>(m, red);
  const double w = a.dv * a.dv * a.dv;
  const double rho = w * m[0];
  const double u[3] = {m[1] / m[0], m[2] / m[0], m[3] / m[0]};
  // Theta_ab = S_ab / rho - u_a u_b for the pairs (11, 22, 33, 12, 13, 23)
  constexpr int A[6] = {0, 1, 2, 0, 0, 1}, B[6] = {0, 1, 2, 1, 2, 2};
  double th[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) th[k] = m[4 + k] / m[0] - u[A[k]] * u[B[k]];
  const double T = (th[0] + th[1] + th[2]) / 3.0;
  const double nu = rho * sqrt(T) / (a.mu0 * (1.0 - a.beta));
  [[maybe_unused]] double cmix = 0.0;
  const double eps = a.eps_cells ? a.eps_cells[row] : a.eps;
  if constexpr (IMEX) {
    const double am = eps / (eps + (1.0 - a.beta) * nu * a.dt);
    // Sigma / rho - u u with Sigma = am S(g) + (1 - am) rho (T I + u u)
#pragma unroll
    for (int k = 0; k < 6; ++k) th[k] = am * th[k] + (1.0 - am) * (k < 3 ? T : 0.0);
    cmix = eps / (eps + nu * a.dt);
  }
  double tau[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) tau[k] = a.beta * th[k] + (k < 3 ? (1.0 - a.beta) * T : 0.0);
  // inverse of the symmetric Tau by cofactors
  const double t11 = tau[0], t22 = tau[1], t33 = tau[2], t12 = tau[3], t13 = tau[4], t23 = tau[5];
  const double c11 = t22 * t33 - t23 * t23, c22 = t11 * t33 - t13 * t13, c33 = t11 * t22 - t12 * t12;
  const double c12 = t13 * t23 - t12 * t33, c13 = t12 * t23 - t13 * t22, c23 = t12 * t13 - t11 * t23;
  const double det = t11 * c11 + t12 * c12 + t13 * c13;
  const double id = 1.0 / det;
  const double i11 = c11 * id, i22 = c22 * id, i33 = c33 * id, i12 = c12 * id, i13 = c13 * id, i23 = c23 * id;
  const double cg = rho / sqrt(8.0 * M_PI * M_PI * M_PI * det);
  const size_t orow = size_t(a.scatter ? row : long(c)) * N3;
  double* out = a.out + orow;
  #pragma unroll 4
  for (int j = t; j < N3; j += kThreads) {
    const double d1 = node<N>(j / (N * N), a.dv) - u[0], d2 = node<N>((j / N) % N, a.dv) - u[1],
                 d3 = node<N>(j % N, a.dv) - u[2];
    const double quad = i11 * d1 * d1 + i22 * d2 * d2 + i33 * d3 * d3 +
                        2.0 * (i12 * d1 * d2 + i13 * d1 * d3 + i23 * d2 * d3);
    const double G = cg * exp(-0.5 * quad);
    if constexpr (MODE == ES_IMEX) {
      out[j] = cmix * h(j) + (1.0 - cmix) * G;
    } else if constexpr (MODE == ES_COLLIDE) {
      out[j] = nu * (G - f[j]);
    } else if constexpr (MODE == ES_PR_STAGE2) {
      const double g1 = nu * (G - f[j]);
      const double y = a.y[orow + j], t1 = tr[j];
      out[j] = y - a.dt * t1 + (a.dt * kPrA21 / eps) * g1;
      a.aux[orow + j] = y - 0.5 * a.dt * t1 + (0.5 * a.dt / eps) * g1;
    } else {
      const double g2 = nu * (G - f[j]);
      out[j] = a.aux[orow + j] - 0.5 * a.dt * tr[j] + (0.5 * a.dt / eps) * g2;
    }
  }
}

struct PrArgs {
  int ncells;
  const int32_t* ncells_dev;
  const int32_t* idx;
  const double* eps_cells;
  double eps, dt, h, dv;
  const double* y;   // y^n
  const double* y1;  // stage 1 value
  const double* t1;  // transport of the stage value
  double* a;         // in: Q(Y1); out: y - dt/2 T1 + dt/(2 eps) Q(Y1)
  double* out;       // penalty solve: in R, out S(R); stage 2: Y2; finish: in Q(Y2), out y^{n+1}
};

// S(R, h) = (eps R + h beta M[R]) / (eps + h beta), beta = 2 pi rho(R): the
// solution of the implicit stage Y = R + (h/eps) beta (M[Y] - Y) (the penalty
// conserves the invariants, so M[Y] = M[R]).
template <int N, int MODE>  // MODE 1: stage 2 (forms R2 and A first, then solves in place); 2: solve y into out
__global__ __launch_bounds__(kThreads) void k_penalty(PrArgs a) {
  constexpr int N3 = N * N * N;
  __shared__ double red[5 * (kWaves + 1)];
  const int c = blockIdx.x;
  if (c >= live_cells(a.ncells, a.ncells_dev)) return;
  const int t = threadIdx.x;
  const long row = a.idx ? long(a.idx[c]) : long(c);
  const size_t base = size_t(row) * N3;
  const double eps = a.eps_cells ? a.eps_cells[row] : a.eps;
  double m[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  [[maybe_unused]] double p1[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // Maxwellian of Y1: cm, u, 1/2T, beta
  if constexpr (MODE == 1) {
    #pragma unroll 4
    for (int j = t; j < N3; j += kThreads) {
      const double v1 = node<N>(j / (N * N), a.dv), v2 = node<N>((j / N) % N, a.dv), v3 = node<N>(j % N, a.dv);
      const double y1 = a.y1[base + j];
      m[0] += y1;
      m[1] += v1 * y1;
      m[2] += v2 * y1;
      m[3] += v3 * y1;
      m[4] += (v1 * v1 + v2 * v2 + v3 * v3) * y1;
    }
    block_sum<5>(m, red);
    const double rho1 = a.dv * a.dv * a.dv * m[0];
    p1[1] = m[1] / m[0];
    p1[2] = m[2] / m[0];
    p1[3] = m[3] / m[0];
    const double T1 = (m[4] / m[0] - (p1[1] * p1[1] + p1[2] * p1[2] + p1[3] * p1[3])) / 3.0;
    p1[0] = rho1 / ((2.0 * M_PI * T1) * sqrt(2.0 * M_PI * T1));
    p1[4] = 1.0 / (2.0 * T1);
    p1[5] = 2.0 * M_PI * rho1;
#pragma unroll
    for (int k = 0; k < 5; ++k) m[k] = 0.0;
  }
  #pragma unroll 4
  for (int j = t; j < N3; j += kThreads) {
    const double v1 = node<N>(j / (N * N), a.dv), v2 = node<N>((j / N) % N, a.dv), v3 = node<N>(j % N, a.dv);
    double r;
    if constexpr (MODE == 1) {
      // P(Y1) = beta1 (M[Y1] - Y1) from Y1's own moments;
      // R2 = y - dt T1 + (dt/eps) Q(Y1) - (2 gamma dt/eps) P(Y1)   (the tableau's stage 2)
      // A  = y - dt/2 T1 + dt/(2 eps) Q(Y1)                         (P cancels in the weights)
      const double y = a.y[base + j], y1 = a.y1[base + j], t1 = a.t1[base + j], q1 = a.a[base + j];
      const double d1 = v1 - p1[1], d2 = v2 - p1[2], d3 = v3 - p1[3];
      const double g1 = p1[5] * (p1[0] * exp(-(d1 * d1 + d2 * d2 + d3 * d3) * p1[4]) - y1);
      r = y - a.dt * t1 + (a.dt / eps) * q1 - (2.0 * a.h / eps) * g1;
      a.a[base + j] = y - 0.5 * a.dt * t1 + (0.5 * a.dt / eps) * q1;
      a.out[base + j] = r;
    } else {
      r = MODE == 2 ? a.y[base + j] : a.out[base + j];
    }
    m[0] += r;
    m[1] += v1 * r;
    m[2] += v2 * r;
    m[3] += v3 * r;
    m[4] += (v1 * v1 + v2 * v2 + v3 * v3) * r;
  }
  block_sum<5>(m, red);  // also orders pass 1's writes before pass 2's reads
  const double w = a.dv * a.dv * a.dv;
  const double rho = w * m[0];
  const double u1 = m[1] / m[0], u2 = m[2] / m[0], u3 = m[3] / m[0];
  const double T = (m[4] / m[0] - (u1 * u1 + u2 * u2 + u3 * u3)) / 3.0;
  const double cm = rho / ((2.0 * M_PI * T) * sqrt(2.0 * M_PI * T));
  const double ia = 1.0 / (2.0 * T);
  const double hb = a.h * 2.0 * M_PI * rho;
  const double den = 1.0 / (eps + hb);
  #pragma unroll 4
  for (int j = t; j < N3; j += kThreads) {
    const double d1 = node<N>(j / (N * N), a.dv) - u1, d2 = node<N>((j / N) % N, a.dv) - u2,
                 d3 = node<N>(j % N, a.dv) - u3;
    const double r = MODE == 2 ? a.y[base + j] : a.out[base + j];
    a.out[base + j] = (eps * r + hb * cm * exp(-(d1 * d1 + d2 * d2 + d3 * d3) * ia)) * den;
  }
}

// y^{n+1} = A - dt/2 T2 + dt/(2 eps) Q(Y2), Q(Y2) in `out` on entry.
template <int N>
__global__ __launch_bounds__(kThreads) void k_pr_finish(PrArgs a) {
  constexpr int N3 = N * N * N;
  const int c = blockIdx.x;
  if (c >= live_cells(a.ncells, a.ncells_dev)) return;
  const long row = a.idx ? long(a.idx[c]) : long(c);
  const size_t base = size_t(row) * N3;
  const double eps = a.eps_cells ? a.eps_cells[row] : a.eps;
  for (int j = threadIdx.x; j < N3; j += kThreads)
    a.out[base + j] = a.a[base + j] - 0.5 * a.dt * a.t1[base + j] + (0.5 * a.dt / eps) * a.out[base + j];
}

// PR(2,2,2) kernels: 1 = stage-2 combination and solve, 2 = penalty solve of
// `y` into `out`, 3 = finish.
bz_status launch_pr(int kind, int n, int ncells, const PrArgs& a, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>(ncells)), block(kThreads);
#define BZ_PR_CASE(NN)                                                                \
  case NN:                                                                            \
    if (kind == 1) hipLaunchKernelGGL((k_penalty<NN, 1>), grid, block, 0, s, a);      \
    else if (kind == 2) hipLaunchKernelGGL((k_penalty<NN, 2>), grid, block, 0, s, a); \
    else hipLaunchKernelGGL((k_pr_finish<NN>), grid, block, 0, s, a);                 \
    break;
  switch (n) {
    BZ_PR_CASE(16)
    BZ_PR_CASE(24)
    BZ_PR_CASE(32)
    BZ_PR_CASE(48)
    default: return bz::fail(BZ_ERR_UNSUPPORTED, "pr222: n=%d", n);
  }
#undef BZ_PR_CASE
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return bz::fail(BZ_ERR_DEVICE, "pr222: launch failed: %s", hipGetErrorString(e));
  return BZ_OK;
}

}  // namespace

namespace bz {

bool kinetic_n_supported(int n) { return n == 16 || n == 24 || n == 32 || n == 48; }


bz_status launch_imex_params(int n, double dv, const int32_t* idx, int ncells, const int32_t* ncells_dev,
                             const double* f, const double* tr, double dt, double* par, hipStream_t s) {
  ParArgs a{ncells, ncells_dev, idx, f, tr, dt, dv, par};
  const dim3 grid(static_cast<unsigned>(ncells)), block(kThreads);
  switch (n) {
    case 16: hipLaunchKernelGGL(k_imex_params<16>, grid, block, 0, s, a); break;
    case 24: hipLaunchKernelGGL(k_imex_params<24>, grid, block, 0, s, a); break;
    case 32: hipLaunchKernelGGL(k_imex_params<32>, grid, block, 0, s, a); break;
    case 48: hipLaunchKernelGGL(k_imex_params<48>, grid, block, 0, s, a); break;
    default: return fail(BZ_ERR_UNSUPPORTED, "imex: n=%d", n);
  }
  return BZ_OK;
}

}  // namespace bz

extern "C" bz_status bz_cell_moments(int32_t n, double L, const void* f, int32_t f_dtype, const int32_t* idx,
                                     int32_t ncells, const int32_t* ncells_dev, const bz_moments_out* out,
                                     int32_t flags, void* stream) {
  bz::clear_error();
  if (!bz::kinetic_n_supported(n)) return bz::fail(BZ_ERR_UNSUPPORTED, "bz_cell_moments: n=%d", n);
  if (!(L > 0.0)) return bz::fail(BZ_ERR_ARG, "bz_cell_moments: L must be > 0");
  if (ncells < 0) return bz::fail(BZ_ERR_ARG, "bz_cell_moments: ncells < 0");
  if (!out) return bz::fail(BZ_ERR_ARG, "bz_cell_moments: null output descriptor");
  if (flags & ~int32_t(BZ_SCATTER)) return bz::fail(BZ_ERR_ARG, "bz_cell_moments: unknown flags");
  if ((flags & BZ_SCATTER) && !idx) return bz::fail(BZ_ERR_ARG, "bz_cell_moments: BZ_SCATTER needs idx");
  if (f_dtype != BZ_FP32 && f_dtype != BZ_FP64) return bz::fail(BZ_ERR_ARG, "bz_cell_moments: bad f_dtype");
  if (ncells == 0) return BZ_OK;
  if (!f) return bz::fail(BZ_ERR_ARG, "bz_cell_moments: null f");
  MomArgs a{};
  a.ncells = ncells;
  a.ncells_dev = ncells_dev;
  a.f = f;
  a.f_fp32 = f_dtype == BZ_FP32;
  a.idx = idx;
  a.scatter = (flags & BZ_SCATTER) != 0;
  a.dv = 2.0 * L / n;
  a.rho = out->rho;
  a.u1 = out->u1;
  a.u2 = out->u2;
  a.u3 = out->u3;
  a.T = out->T;
  a.l1 = out->l1;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const dim3 grid(static_cast<unsigned>(ncells)), block(kThreads);
  switch (n) {
    case 16: hipLaunchKernelGGL(k_moments<16>, grid, block, 0, s, a); break;
    case 24: hipLaunchKernelGGL(k_moments<24>, grid, block, 0, s, a); break;
    case 32: hipLaunchKernelGGL(k_moments<32>, grid, block, 0, s, a); break;
    default: hipLaunchKernelGGL(k_moments<48>, grid, block, 0, s, a); break;
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return bz::fail(BZ_ERR_DEVICE, "bz_cell_moments: launch failed: %s", hipGetErrorString(e));
  return BZ_OK;
}

namespace {

bz_status esbgk_check(const char* who, const bz_esbgk_desc* d, int32_t ncells, int32_t flags, const int32_t* idx) {
  if (!d) return bz::fail(BZ_ERR_ARG, "%s: null descriptor", who);
  if (!bz::kinetic_n_supported(d->n)) return bz::fail(BZ_ERR_UNSUPPORTED, "%s: n=%d", who, d->n);
  if (!(d->L > 0.0)) return bz::fail(BZ_ERR_ARG, "%s: L must be > 0", who);
  if (!(d->beta < 1.0) || !std::isfinite(d->beta)) return bz::fail(BZ_ERR_ARG, "%s: beta must be < 1", who);
  if (!(d->mu0 > 0.0)) return bz::fail(BZ_ERR_ARG, "%s: mu0 must be > 0", who);
  if (ncells < 0) return bz::fail(BZ_ERR_ARG, "%s: ncells < 0", who);
  if (flags & ~int32_t(BZ_SCATTER)) return bz::fail(BZ_ERR_ARG, "%s: unknown flags", who);
  if ((flags & BZ_SCATTER) && !idx) return bz::fail(BZ_ERR_ARG, "%s: BZ_SCATTER needs idx", who);
  return BZ_OK;
}

template <int MODE>
bz_status esbgk_launch(const bz_esbgk_desc* d, const EsArgs& a, int ncells, void* stream, const char* who) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  const dim3 grid(static_cast<unsigned>(ncells)), block(kThreads);
  switch (d->n) {
    case 16: hipLaunchKernelGGL((k_esbgk<16, MODE>), grid, block, 0, s, a); break;
    case 24: hipLaunchKernelGGL((k_esbgk<24, MODE>), grid, block, 0, s, a); break;
    case 32: hipLaunchKernelGGL((k_esbgk<32, MODE>), grid, block, 0, s, a); break;
    default: hipLaunchKernelGGL((k_esbgk<48, MODE>), grid, block, 0, s, a); break;
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return bz::fail(BZ_ERR_DEVICE, "%s: launch failed: %s", who, hipGetErrorString(e));
  return BZ_OK;
}

}  // namespace

extern "C" bz_status bz_esbgk_collide(const bz_esbgk_desc* d, const double* f, const int32_t* idx, int32_t ncells,
                                      const int32_t* ncells_dev, double* q, int32_t flags, void* stream) {
  bz::clear_error();
  bz_status st = esbgk_check("bz_esbgk_collide", d, ncells, flags, idx);
  if (st != BZ_OK) return st;
  if (ncells == 0) return BZ_OK;
  if (!f || !q) return bz::fail(BZ_ERR_ARG, "bz_esbgk_collide: null f or q");
  if (q == f) return bz::fail(BZ_ERR_ARG, "bz_esbgk_collide: q must not alias f");
  EsArgs a{};
  a.ncells = ncells;
  a.ncells_dev = ncells_dev;
  a.idx = idx;
  a.scatter = (flags & BZ_SCATTER) != 0;
  a.f = f;
  a.beta = d->beta;
  a.mu0 = d->mu0;
  a.dv = 2.0 * d->L / d->n;
  a.out = q;
  return esbgk_launch<ES_COLLIDE>(d, a, ncells, stream, "bz_esbgk_collide");
}

extern "C" bz_status bz_esbgk_imex_euler(const bz_esbgk_desc* d, const bz_imex_desc* im, const double* f,
                                         const double* tr, const int32_t* idx, int32_t ncells,
                                         const int32_t* ncells_dev, double* f_out, int32_t flags, void* stream) {
  bz::clear_error();
  bz_status st = esbgk_check("bz_esbgk_imex_euler", d, ncells, flags, idx);
  if (st != BZ_OK) return st;
  if (!im) return bz::fail(BZ_ERR_ARG, "bz_esbgk_imex_euler: null IMEX descriptor");
  if (!(im->dt > 0.0) || !std::isfinite(im->dt)) return bz::fail(BZ_ERR_ARG, "bz_esbgk_imex_euler: dt must be > 0");
  if (!im->eps_cells && !(im->eps > 0.0)) return bz::fail(BZ_ERR_ARG, "bz_esbgk_imex_euler: eps must be > 0");
  if (ncells == 0) return BZ_OK;
  if (!f || !tr || !f_out) return bz::fail(BZ_ERR_ARG, "bz_esbgk_imex_euler: null f, tr or f_out");
  if (f_out == f && idx && !(flags & BZ_SCATTER))
    return bz::fail(BZ_ERR_ARG, "bz_esbgk_imex_euler: in place with idx needs BZ_SCATTER");
  EsArgs a{};
  a.ncells = ncells;
  a.ncells_dev = ncells_dev;
  a.idx = idx;
  a.scatter = (flags & BZ_SCATTER) != 0;
  a.f = f;
  a.tr = tr;
  a.eps_cells = im->eps_cells;
  a.eps = im->eps;
  a.dt = im->dt;
  a.beta = d->beta;
  a.mu0 = d->mu0;
  a.dv = 2.0 * d->L / d->n;
  a.out = f_out;
  return esbgk_launch<ES_IMEX>(d, a, ncells, stream, "bz_esbgk_imex_euler");
}

// ---------------------------------------------------------------- PR(2,2,2) entry points
namespace {

constexpr double kPrGamma = 0.29289321881345248;  // 1 - 1/sqrt(2), the implicit diagonal

bz_status pr_check(const char* who, const bz_plan* p, const bz_imex_desc* d, int32_t ncells) {
  if (!p) return bz::fail(BZ_ERR_ARG, "%s: null plan", who);
  if (p->dim == 2) return bz::fail(BZ_ERR_UNSUPPORTED, "%s: three velocity dimensions only", who);
  if (!d) return bz::fail(BZ_ERR_ARG, "%s: null descriptor", who);
  if (!p->ws_dev) return bz::fail(BZ_ERR_STATE, "%s: plan not bound", who);
  if (!(d->dt > 0.0) || !std::isfinite(d->dt)) return bz::fail(BZ_ERR_ARG, "%s: dt must be > 0", who);
  if (!d->eps_cells && !(d->eps > 0.0)) return bz::fail(BZ_ERR_ARG, "%s: eps must be > 0", who);
  if (ncells < 0) return bz::fail(BZ_ERR_ARG, "%s: ncells < 0", who);
  if (!p->project && p->fp32) return bz::fail(BZ_ERR_UNSUPPORTED, "%s: an FP32 plan must project (FP64 output)", who);
  if (ncells > p->capacity)
    return bz::fail(BZ_ERR_NOMEM, "%s: %d cells exceed the bound capacity %d", who, ncells, p->capacity);
  return BZ_OK;
}

PrArgs pr_args(const bz_plan* p, const bz_imex_desc* d, const int32_t* idx, int ncells, const int32_t* ncells_dev) {
  PrArgs a{};
  a.ncells = ncells;
  a.ncells_dev = ncells_dev;
  a.idx = idx;
  a.eps_cells = d->eps_cells;
  a.eps = d->eps;
  a.dt = d->dt;
  a.h = kPrGamma * d->dt;
  a.dv = p->dv;
  return a;
}

bz_status pr_collide(const bz_plan* p, const double* f, const int32_t* idx, int ncells, const int32_t* ncells_dev,
                     double* q, hipStream_t s) {
  bz::Binding b;
  b.tables = p->tables_dev;
  b.ws = p->ws_dev;
  b.capacity = p->capacity;
  b.lay = p->ws;
  return bz::launch_collide(p, b, f, 0, idx, ncells, ncells_dev, q, 1, s, p->timing);
}

}  // namespace

extern "C" bz_status bz_pr222_stage1(const bz_plan* p, const bz_imex_desc* d, const double* y, const int32_t* idx,
                                     int32_t ncells, const int32_t* ncells_dev, double* y1, void* stream) {
  bz::clear_error();
  bz_status st = pr_check("bz_pr222_stage1", p, d, ncells);
  if (st != BZ_OK || ncells == 0) return st;
  if (!y || !y1) return bz::fail(BZ_ERR_ARG, "bz_pr222_stage1: null y or y1");
  if (y1 == y) return bz::fail(BZ_ERR_ARG, "bz_pr222_stage1: y1 must not alias y");
  PrArgs a = pr_args(p, d, idx, ncells, ncells_dev);
  a.y = y;
  a.out = y1;
  return launch_pr(2, p->n, ncells, a, static_cast<hipStream_t>(stream));
}

extern "C" bz_status bz_pr222_stage2(const bz_plan* p, const bz_imex_desc* d, const double* y, const double* y1,
                                     const double* t1, const int32_t* idx, int32_t ncells, const int32_t* ncells_dev,
                                     double* y2, double* a_out, void* stream) {
  bz::clear_error();
  bz_status st = pr_check("bz_pr222_stage2", p, d, ncells);
  if (st != BZ_OK || ncells == 0) return st;
  if (!y || !y1 || !t1 || !y2 || !a_out) return bz::fail(BZ_ERR_ARG, "bz_pr222_stage2: null array");
  const void* in[3] = {y, y1, t1};
  for (const void* q : in)
    if (q == y2 || q == a_out) return bz::fail(BZ_ERR_ARG, "bz_pr222_stage2: outputs must not alias inputs");
  if (y2 == a_out) return bz::fail(BZ_ERR_ARG, "bz_pr222_stage2: y2 and a must differ");
  hipStream_t s = static_cast<hipStream_t>(stream);
  st = pr_collide(p, y1, idx, ncells, ncells_dev, a_out, s);  // Q(Y1) into A's rows
  if (st != BZ_OK) return st;
  PrArgs a = pr_args(p, d, idx, ncells, ncells_dev);
  a.y = y;
  a.y1 = y1;
  a.t1 = t1;
  a.a = a_out;
  a.out = y2;
  return launch_pr(1, p->n, ncells, a, s);
}

extern "C" bz_status bz_pr222_finish(const bz_plan* p, const bz_imex_desc* d, const double* a_in, const double* y2,
                                     const double* t2, const int32_t* idx, int32_t ncells, const int32_t* ncells_dev,
                                     double* y_out, void* stream) {
  bz::clear_error();
  bz_status st = pr_check("bz_pr222_finish", p, d, ncells);
  if (st != BZ_OK || ncells == 0) return st;
  if (!a_in || !y2 || !t2 || !y_out) return bz::fail(BZ_ERR_ARG, "bz_pr222_finish: null array");
  if (y_out == a_in || y_out == y2 || y_out == t2) return bz::fail(BZ_ERR_ARG, "bz_pr222_finish: y_out must not alias inputs");
  hipStream_t s = static_cast<hipStream_t>(stream);
  st = pr_collide(p, y2, idx, ncells, ncells_dev, y_out, s);  // Q(Y2) into y_out's rows
  if (st != BZ_OK) return st;
  PrArgs a = pr_args(p, d, idx, ncells, ncells_dev);
  a.a = const_cast<double*>(a_in);
  a.t1 = t2;
  a.out = y_out;
  return launch_pr(3, p->n, ncells, a, s);
}

// ---------------------------------------------------------------- ES-BGK PR(2,2,2)
namespace {

bz_status es_pr_check(const char* who, const bz_esbgk_desc* d, const bz_imex_desc* im, int32_t ncells) {
  bz_status st = esbgk_check(who, d, ncells, 0, nullptr);
  if (st != BZ_OK) return st;
  if (!im) return bz::fail(BZ_ERR_ARG, "%s: null IMEX descriptor", who);
  if (!(im->dt > 0.0) || !std::isfinite(im->dt)) return bz::fail(BZ_ERR_ARG, "%s: dt must be > 0", who);
  if (!im->eps_cells && !(im->eps > 0.0)) return bz::fail(BZ_ERR_ARG, "%s: eps must be > 0", who);
  return BZ_OK;
}

EsArgs es_pr_args(const bz_esbgk_desc* d, const bz_imex_desc* im, const int32_t* idx, int ncells,
                  const int32_t* ncells_dev) {
  EsArgs a{};
  a.ncells = ncells;
  a.ncells_dev = ncells_dev;
  a.idx = idx;
  a.scatter = 1;  // every array is indexed by the cell's row
  a.eps_cells = im->eps_cells;
  a.eps = im->eps;
  a.beta = d->beta;
  a.mu0 = d->mu0;
  a.dv = 2.0 * d->L / d->n;
  return a;
}

}  // namespace

extern "C" bz_status bz_esbgk_pr222_stage1(const bz_esbgk_desc* d, const bz_imex_desc* im, const double* y,
                                           const int32_t* idx, int32_t ncells, const int32_t* ncells_dev, double* y1,
                                           void* stream) {
  bz::clear_error();
  bz_status st = es_pr_check("bz_esbgk_pr222_stage1", d, im, ncells);
  if (st != BZ_OK || ncells == 0) return st;
  if (!y || !y1) return bz::fail(BZ_ERR_ARG, "bz_esbgk_pr222_stage1: null y or y1");
  if (y1 == y) return bz::fail(BZ_ERR_ARG, "bz_esbgk_pr222_stage1: y1 must not alias y");
  EsArgs a = es_pr_args(d, im, idx, ncells, ncells_dev);
  a.f = y;
  a.tr = nullptr;
  a.dt = kPrGamma * im->dt;  // the implicit stage: Y1 = y + gamma dt Q_ES(Y1)/eps
  a.out = y1;
  return esbgk_launch<ES_IMEX>(d, a, ncells, stream, "bz_esbgk_pr222_stage1");
}

extern "C" bz_status bz_esbgk_pr222_stage2(const bz_esbgk_desc* d, const bz_imex_desc* im, const double* y,
                                           const double* y1, const double* t1, const int32_t* idx, int32_t ncells,
                                           const int32_t* ncells_dev, double* y2, double* a_out, void* stream) {
  bz::clear_error();
  bz_status st = es_pr_check("bz_esbgk_pr222_stage2", d, im, ncells);
  if (st != BZ_OK || ncells == 0) return st;
  if (!y || !y1 || !t1 || !y2 || !a_out) return bz::fail(BZ_ERR_ARG, "bz_esbgk_pr222_stage2: null array");
  const void* in[3] = {y, y1, t1};
  for (const void* q : in)
    if (q == y2 || q == a_out) return bz::fail(BZ_ERR_ARG, "bz_esbgk_pr222_stage2: outputs must not alias inputs");
  if (y2 == a_out) return bz::fail(BZ_ERR_ARG, "bz_esbgk_pr222_stage2: y2 and a must differ");
  EsArgs a = es_pr_args(d, im, idx, ncells, ncells_dev);
  a.f = y1;
  a.tr = t1;
  a.y = y;
  a.dt = im->dt;
  a.out = y2;  // R2
  a.aux = a_out;
  st = esbgk_launch<ES_PR_STAGE2>(d, a, ncells, stream, "bz_esbgk_pr222_stage2");
  if (st != BZ_OK) return st;
  EsArgs b = es_pr_args(d, im, idx, ncells, ncells_dev);
  b.f = y2;  // in place: Y2 = S(R2, gamma dt)
  b.tr = nullptr;
  b.dt = kPrGamma * im->dt;
  b.out = y2;
  return esbgk_launch<ES_IMEX>(d, b, ncells, stream, "bz_esbgk_pr222_stage2");
}

extern "C" bz_status bz_esbgk_pr222_finish(const bz_esbgk_desc* d, const bz_imex_desc* im, const double* a_in,
                                           const double* y2, const double* t2, const int32_t* idx, int32_t ncells,
                                           const int32_t* ncells_dev, double* y_out, void* stream) {
  bz::clear_error();
  bz_status st = es_pr_check("bz_esbgk_pr222_finish", d, im, ncells);
  if (st != BZ_OK || ncells == 0) return st;
  if (!a_in || !y2 || !t2 || !y_out) return bz::fail(BZ_ERR_ARG, "bz_esbgk_pr222_finish: null array");
  if (y_out == y2 || y_out == t2) return bz::fail(BZ_ERR_ARG, "bz_esbgk_pr222_finish: y_out must not alias y2 or t2");
  EsArgs a = es_pr_args(d, im, idx, ncells, ncells_dev);
  a.f = y2;
  a.tr = t2;
  a.dt = im->dt;
  a.aux = const_cast<double*>(a_in);
  a.out = y_out;  // may equal a_in (same element, same thread)
  return esbgk_launch<ES_PR_FINISH>(d, a, ncells, stream, "bz_esbgk_pr222_finish");
}
