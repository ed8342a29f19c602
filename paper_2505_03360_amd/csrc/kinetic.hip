// Per-cell reductions over the velocity grid on gfx950, FP64: macroscopic
// fields and the L1 distance of the kinetic-to-fluid criterion (Sec. 2 and
// 3.3), and the parameters of the penalised IMEX update of the Boltzmann layer
// (Sec. 4.4, eq. 1002).
//
// One workgroup of 256 threads per cell.  Each thread accumulates a strided
// subset of the nodes, then the partial sums are combined across the wave
// (butterfly) and across the four waves in a fixed order, so the result of a
// cell does not depend on the batch it is in.
#include "bz_internal.hpp"
#include "kinetic.hpp"

namespace {

constexpr int kThreads = 256;

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
template <int K>
__device__ __forceinline__ void block_sum(double (&m)[K], double* red) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m[k] += __shfl_xor(m[k], o);
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) red[k * 4 + wv] = m[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) m[k] = ((red[k * 4 + 0] + red[k * 4 + 1]) + red[k * 4 + 2]) + red[k * 4 + 3];
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
  __shared__ double red[5 * 4];
  const int c = blockIdx.x;
  if (c >= live_cells(a.ncells, a.ncells_dev)) return;
  const int t = threadIdx.x;
  const long row = a.idx ? long(a.idx[c]) : long(c);
  const size_t base = size_t(row) * N3;
  auto fval = [&](int j) -> double {
    return a.f_fp32 ? double(static_cast<const float*>(a.f)[base + j]) : static_cast<const double*>(a.f)[base + j];
  };
  double m[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
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
  __shared__ double red[10 * 4];
  const int c = blockIdx.x;
  if (c >= live_cells(a.ncells, a.ncells_dev)) return;
  const int t = threadIdx.x;
  const long row = a.idx ? long(a.idx[c]) : long(c);
  const double* f = a.f + size_t(row) * N3;
  const double* tr = a.tr + size_t(row) * N3;
  double m[10] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
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
