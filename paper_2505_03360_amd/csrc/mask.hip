// Moment-realizability regime mask (Sec. 3.2-3.3 and 4.5, Algorithm 1) on
// gfx950, FP64, and the ordered list of the cells it assigns to the
// Boltzmann layer.
//
// This file is compiled with -ffp-contract=off: every operation below is one
// IEEE FP64 operation, rounded once, evaluated in the order written (division
// and square root correctly rounded), so that the decision of each cell is a
// deterministic function of its inputs.
#include "bz_internal.hpp"

namespace {

struct MaskArgs {
  int nx, ny;
  double dx, dy, mu0, kappa0, eta0, eta1, delta0;
  int lap_mode;
  const double *rho, *ux, *uy, *T, *eps, *l1;
  const uint8_t* rin;
  const uint8_t* flags;
  uint8_t* rout;
  int32_t* counts;
  double* diag;
};

__global__ void k_mask_init(int32_t* counts) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    counts[0] = 0;
    counts[1] = 0;
  }
}

__device__ __forceinline__ bool finite(double x) { return x - x == 0.0; }

// Cell (ix, iy): stencil clamped at the border (ghost cells copy the nearest
// physical cell), central differences, 5-point Laplacians over dx*dy.
__global__ __launch_bounds__(256) void k_mask(MaskArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.nx * a.ny) return;
  const int iy = i / a.nx, ix = i % a.nx;
  const int iL = ix > 0 ? ix - 1 : 0, iR = ix < a.nx - 1 ? ix + 1 : a.nx - 1;
  const int jL = iy > 0 ? iy - 1 : 0, jR = iy < a.ny - 1 ? iy + 1 : a.ny - 1;
  const int cW = iy * a.nx + iL, cE = iy * a.nx + iR, cS = jL * a.nx + ix, cN = jR * a.nx + ix;
  const double two_dx = 2.0 * a.dx, two_dy = 2.0 * a.dy, dxdy = a.dx * a.dy;
  const double rho = a.rho[i], T = a.T[i], eps = a.eps[i];

  const double uxx = (a.ux[cE] - a.ux[cW]) / two_dx;
  const double uxy = (a.ux[cN] - a.ux[cS]) / two_dy;
  const double uyx = (a.uy[cE] - a.uy[cW]) / two_dx;
  const double uyy = (a.uy[cN] - a.uy[cS]) / two_dy;
  const double Tx = (a.T[cE] - a.T[cW]) / two_dx;
  const double Ty = (a.T[cN] - a.T[cS]) / two_dy;
  const double sqT = sqrt(T);
  const double mu = a.mu0 * sqT;
  const double kap = a.kappa0 * sqT;
  const double xi1 = (eps * mu) / (rho * T);
  const double xi2 = ((eps * eps) * (2.0 * (kap * kap))) / (((((3.0 * rho) * rho) * T) * T) * T);
  const double c43 = 4.0 / 3.0, c23 = 2.0 / 3.0;
  const double a1 = c43 * uxx - c23 * uyy;
  const double a2 = Tx * Tx;
  const double b1 = uxy + uyx;
  const double b2 = Tx * Ty;
  const double c1 = c43 * uyy - c23 * uxx;
  const double c2 = Ty * Ty;
  const double h1 = (-c23) * (uxx + uyy);
  const double dd = xi1 * b1 + xi2 * b2;
  const double pp = xi1 * (a1 - c1) + xi2 * (a2 - c2);
  const double sq = sqrt(pp * pp + 4.0 * (dd * dd));
  const double ss = (((a1 * xi1) + (a2 * xi2)) + (c1 * xi1)) + (c2 * xi2);
  const double lam_a = 0.5 * ((sq - ss) + 2.0);
  const double lam_b = 0.5 * (((-sq) - ss) + 2.0);
  const double lam_c = 1.0 - xi1 * h1;
  const double gT2 = Tx * Tx + Ty * Ty;
  const double gu2 = ((uxx * uxx + uxy * uxy) + uyx * uyx) + uyy * uyy;
  const double lux = ((((a.ux[cW] + a.ux[cE]) + a.ux[cS]) + a.ux[cN]) - 4.0 * a.ux[i]) / dxdy;
  const double luy = ((((a.uy[cW] + a.uy[cE]) + a.uy[cS]) + a.uy[cN]) - 4.0 * a.uy[i]) / dxdy;
  const double lrr = ((((a.rho[cW] + a.rho[cE]) + a.rho[cS]) + a.rho[cN]) - 4.0 * rho) / dxdy;
  const double lr = lrr / rho;
  double lu2;
  if (a.lap_mode == 0) {
    const double lu = lux + luy;
    lu2 = lu * lu;
  } else {
    lu2 = lux * lux + luy * luy;
  }
  const double inner = (lu2 + lr * lr) * (1.0 + T * T);
  const double lam_B = (eps * eps) * ((gT2 / T + gu2) + sqrt(inner));

  const uint8_t r = a.rin[i];
  uint8_t out = r;
  const bool valid = rho > 0.0 && T > 0.0 && eps >= 0.0 && finite(a.ux[i]) && finite(a.uy[i]) &&
                     finite(rho) && finite(T) && finite(eps) && finite(lam_a) && finite(lam_b) &&
                     finite(lam_c) && finite(lam_B);
  if (!valid) {
    atomicAdd(&a.counts[1], 1);
  } else {
    const bool big_B = fabs(lam_B) > a.eta1;
    const bool near_one = fabs(lam_a - 1.0) <= a.eta0 && fabs(lam_b - 1.0) <= a.eta0 &&
                          fabs(lam_c - 1.0) <= a.eta0;
    const bool close = a.l1 ? (a.l1[i] <= a.delta0) : false;
    if (r == 2) out = big_B ? 2 : 1;
    else if (r == 1) out = big_B ? 2 : ((near_one && close) ? 0 : 1);
    else if (r == 0) out = near_one ? 0 : 1;
  }
  if (a.flags) {
    const uint8_t fl = a.flags[i];
    if (fl & BZ_CELL_FORCE_BOLTZMANN) out = 2;
    if (fl & BZ_CELL_SOLID) out = BZ_REGIME_SOLID;
  }
  a.rout[i] = out;
  if (a.diag) {
    a.diag[4 * size_t(i) + 0] = lam_a;
    a.diag[4 * size_t(i) + 1] = lam_b;
    a.diag[4 * size_t(i) + 2] = lam_c;
    a.diag[4 * size_t(i) + 3] = lam_B;
  }
}

// Ascending list of the regime-2 cells (kinetic = 0) or of the kinetic cells,
// regime 1 or 2 (kinetic = 1): one workgroup sweeps the grid in tiles of 1024
// cells; wave ballots give each flagged cell its rank within the tile.
__global__ __launch_bounds__(1024) void k_compact(const uint8_t* reg, int ncell, int32_t* idx,
                                                  int32_t* counts, int kinetic) {
  __shared__ int wsum[16];
  __shared__ int base_s;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  if (t == 0) base_s = 0;
  __syncthreads();
  for (int b = 0; b < ncell; b += 1024) {
    const int i = b + t;
    const bool flag = i < ncell && (reg[i] == 2 || (kinetic && reg[i] == 1));
    const unsigned long long m = __ballot(flag);
    const int pre = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wv] = __popcll(m);
    __syncthreads();
    int off = base_s;
    for (int k = 0; k < wv; ++k) off += wsum[k];
    if (flag) idx[off + pre] = i;
    __syncthreads();
    if (t == 0) {
      int tot = 0;
      for (int k = 0; k < 16; ++k) tot += wsum[k];
      base_s += tot;
    }
    __syncthreads();
  }
  if (t == 0) counts[0] = base_s;
}

__global__ void k_copy_u8(const uint8_t* src, uint8_t* dst, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

}  // namespace

namespace bz {
void launch_copy_u8(const uint8_t* src, uint8_t* dst, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_u8, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, src, dst, n);
}

void launch_compact_kinetic(const uint8_t* regime, int ncell, int32_t* idx, int32_t* count, hipStream_t s) {
  hipLaunchKernelGGL(k_compact, dim3(1), dim3(1024), 0, s, regime, ncell, idx, count, 1);
}
}  // namespace bz

extern "C" bz_status bz_realizability_mask(const bz_mask_desc* d, const double* rho, const double* ux,
                                           const double* uy, const double* T, const double* eps,
                                           const uint8_t* regime_in, const double* l1dist,
                                           const uint8_t* cell_flags, uint8_t* regime_out,
                                           int32_t* boltz_idx, int32_t* counts, double* diag,
                                           void* stream) {
  bz::clear_error();
  if (!d) return bz::fail(BZ_ERR_ARG, "bz_realizability_mask: null descriptor");
  if (d->nx < 1 || d->ny < 1 || long(d->nx) * d->ny > (1L << 30))
    return bz::fail(BZ_ERR_ARG, "bz_realizability_mask: bad grid %dx%d", d->nx, d->ny);
  if (!(d->dx > 0.0) || !(d->dy > 0.0)) return bz::fail(BZ_ERR_ARG, "bz_realizability_mask: dx, dy must be > 0");
  if (d->laplacian_u_mode != 0 && d->laplacian_u_mode != 1)
    return bz::fail(BZ_ERR_ARG, "bz_realizability_mask: laplacian_u_mode must be 0 or 1");
  if (!rho || !ux || !uy || !T || !eps || !regime_in || !regime_out || !boltz_idx || !counts)
    return bz::fail(BZ_ERR_ARG, "bz_realizability_mask: null array");
  hipStream_t s = static_cast<hipStream_t>(stream);
  MaskArgs a{};
  a.nx = d->nx;
  a.ny = d->ny;
  a.dx = d->dx;
  a.dy = d->dy;
  a.mu0 = d->mu0;
  a.kappa0 = d->kappa0;
  a.eta0 = d->eta0;
  a.eta1 = d->eta1;
  a.delta0 = d->delta0;
  a.lap_mode = d->laplacian_u_mode;
  a.rho = rho;
  a.ux = ux;
  a.uy = uy;
  a.T = T;
  a.eps = eps;
  a.l1 = l1dist;
  a.rin = regime_in;
  a.flags = cell_flags;
  a.rout = regime_out;
  a.counts = counts;
  a.diag = diag;
  const int ncell = d->nx * d->ny;
  hipLaunchKernelGGL(k_mask_init, dim3(1), dim3(64), 0, s, counts);
  hipLaunchKernelGGL(k_mask, dim3(unsigned((ncell + 255) / 256)), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_compact, dim3(1), dim3(1024), 0, s, regime_out, ncell, boltz_idx, counts, 0);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return bz::fail(BZ_ERR_DEVICE, "bz_realizability_mask: launch failed: %s", hipGetErrorString(e));
  return BZ_OK;
}

extern "C" bz_status bz_mask_sync(const int32_t* counts, void* stream) {
  bz::clear_error();
  if (!counts) return bz::fail(BZ_ERR_ARG, "bz_mask_sync: null counts");
  hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
  int32_t host[2] = {0, 0};
  if (e == hipSuccess) e = hipMemcpy(host, counts, sizeof host, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return bz::fail(BZ_ERR_DEVICE, "bz_mask_sync: %s", hipGetErrorString(e));
  if (host[1] > 0)
    return bz::fail(BZ_ERR_NUMERIC, "bz_realizability_mask: %d cells with invalid inputs (rho <= 0, T <= 0, eps < 0 "
                    "or non-finite) kept their regime", int(host[1]));
  return BZ_OK;
}
