// Fast spectral collision operator for Maxwell molecules in two velocity
// dimensions (Sec. 4.4.1, the 2d case) for gfx950.
//
// Per cell, with fhat = DFT(f)/n^2 and, for every angle p (weight w_p = pi/m):
//   X_p = (s_p alpha_p + i alpha'_p / s_p) * fhat   (real, even multipliers,
//                                                    zero on the Nyquist lines)
//   Y_p = IDFT(X_p),  acc += w_p * Re(Y_p) * Im(Y_p)
// and the loss pass X = (Bhat_M / sL + i sL [Nyquist]) fhat, whose
// -(sL f - Im Y) Re Y = -(f - fNyq) Lambda is the loss term formed with the
// exact input f, as in three dimensions.  Q = kernel_c * acc, then the FP64
// projection on (1, v1, v2, |v|^2) or the raw output.
//
// One 64-lane wave holds 64/n cells; lane r of a cell owns row k1 = r of the
// spectrum and, after the transpose, column j2 = r of the physical grid:
//   forward: column i2 = r of f along i1, LDS transpose, row k1 = r along i2;
//            from n = 32 up fhat goes to the cell's workspace slot ([k2][k1]:
//            the n lanes of a cell write and read consecutive entries, each
//            lane only its own row), which keeps the LDS to one transpose
//            buffer per cell; at n = 16 the rows stay in LDS;
//   pass:    row k1 = r: X along k2 -> j2, LDS transpose, column j2 = r along
//            k1 -> j1, products into the lane's n accumulators.
// Layouts: f, q [i1][i2] (i2 fastest), multipliers and fhat [k2][k1] (lanes on
// k1 read consecutive entries).
#include "bz_internal.hpp"
#include "fft.hpp"
#include "gptr.hpp"

namespace {

using bzk::cx;
using bzk::gptr;
using bzk::opaque_global;

struct Args2D {
  int ncells;
  const int32_t* ncells_dev;
  const void* f;
  int f_fp32;
  const int32_t* idx;
  int scatter;
  const void* mult;  // [pass][k2][k1] pairs in the plan precision
  const void* w;     // [pass] weights, the loss scale last
  void* fs;          // workspace: fhat of compact cell c at fs + c * fs_stride, [k2][k1]
  size_t fs_stride;  // elements (complex, plan precision) per cell
  int m1;
  double C, dv;
  double ginv[16];   // (C C^T)^-1 of the four invariants
  int project;       // 1: FP64 projected output; 0: raw Q in the plan precision
  void* q;
  int32_t* status;
  int zero;          // 0 at run time: keeps the status store a per-lane store
};

__device__ __forceinline__ int live_cells2d(int ncells, const int32_t* ncells_dev) {
  int c = ncells;
  if (ncells_dev) {
    const int d = *ncells_dev;
    c = d < c ? d : c;
    if (c < 0) c = 0;
  }
  return c;
}

template <typename T>
__device__ __forceinline__ T load_f2d(const Args2D& a, size_t i) {
  return a.f_fp32 ? T(static_cast<const float*>(a.f)[i]) : T(static_cast<const double*>(a.f)[i]);
}

template <typename T, int N>
__global__ __launch_bounds__(64, 2) void k_collide2d(Args2D a) {
  constexpr int G = 64 / N;  // cells per wave
  constexpr int P = N + 1;   // LDS row pitch
  constexpr bool kWs = bz::spectrum2d_in_workspace(N);  // else the spectrum rows stay in LDS
  __shared__ cx<T> tr[G][N][P];
  __shared__ cx<T> fsl[kWs ? 1 : G][kWs ? 1 : N][kWs ? 1 : P];
  const int lane = threadIdx.x, g = lane / N, r = lane % N;
  const int cell = blockIdx.x * G + g;
  const bool live = cell < live_cells2d(a.ncells, a.ncells_dev);
  const long row = live ? (a.idx ? long(a.idx[cell]) : long(cell)) : 0;
  const size_t fbase = size_t(row) * N * N;
  // the cell's spectrum slot: the workspace holds the launched cells, not the
  // idle tail of the last wave, so idle lanes point at cell 0's slot (present
  // whenever a launch happens), never write it, and discard what they read
  cx<T>* const fsg = static_cast<cx<T>*>(a.fs) + (live ? size_t(cell) * a.fs_stride : 0) + r;
  cx<T> x[N];
  // forward: column i2 = r along i1, then row k1 = r along i2
#pragma unroll
  for (int i1 = 0; i1 < N; ++i1) x[i1] = cx<T>{live ? load_f2d<T>(a, fbase + size_t(i1) * N + r) : T(0), T(0)};
  bzk::fft<N, -1>(x);
#pragma unroll
  for (int k1 = 0; k1 < N; ++k1) tr[g][k1][r] = x[k1];
  __syncthreads();
#pragma unroll
  for (int t = 0; t < N; ++t) {
    const int i2 = bzk::first_stage_order<N>(t);
    x[i2] = tr[g][r][i2];
  }
  bzk::fft<N, -1>(x);
  const T scale = T(1) / T(N * N);
#pragma unroll
  for (int k2 = 0; k2 < N; ++k2) {
    const cx<T> v{x[k2].x * scale, x[k2].y * scale};
    if constexpr (kWs) {
      if (live) fsg[size_t(k2) * N] = v;
    } else {
      fsl[g][r][k2] = v;
    }
  }
  T acc[N];
#pragma unroll
  for (int j1 = 0; j1 < N; ++j1) acc[j1] = T(0);
  const cx<T>* mult = static_cast<const cx<T>*>(a.mult);
  const T* wt = static_cast<const T*>(a.w);
  for (int p = 0; p < a.m1; ++p) {
    __syncthreads();  // the previous pass (or the forward) has read tr
    // opaque per-pass bases: the n addresses of each row are formed here,
    // not hoisted out of the pass loop (2 registers each)
    const gptr<cx<T>> M = opaque_global(mult + size_t(p) * N * N + r);
    const gptr<cx<T>> F0 = opaque_global(fsg);
    // in groups of 16 (bounded loads in flight)
#pragma unroll
    for (int h = 0; h < N; h += 16) {
#pragma unroll
      for (int k2 = h; k2 < h + 16; ++k2) {
        const cx<T> m = M[size_t(k2) * N];
        cx<T> F;
        if constexpr (kWs) {
          const cx<T> Fl = F0[size_t(k2) * N];  // idle lanes read the slot of cell 0
          F = live ? Fl : cx<T>{T(0), T(0)};
        } else {
          F = fsl[g][r][k2];
        }
        x[k2] = cx<T>{m.x * F.x - m.y * F.y, m.x * F.y + m.y * F.x};
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    bzk::fft<N, 1>(x);  // along k2 -> j2, row k1 = r
#pragma unroll
    for (int j2 = 0; j2 < N; ++j2) tr[g][r][j2] = x[j2];
    __syncthreads();
#pragma unroll
    for (int t = 0; t < N; ++t) {
      const int k1 = bzk::first_stage_order<N>(t);
      x[k1] = tr[g][k1][r];
    }
    bzk::fft<N, 1>(x);  // along k1 -> j1, column j2 = r
    const T wp = wt[p];
    if (p == a.m1 - 1) {
      // loss pass with the input f (opaque base: the n row addresses are not
      // held across the pass loop; idle lanes read row 0 and discard it)
      auto loss = [&](auto fp) {
#pragma unroll
        for (int j1 = 0; j1 < N; ++j1) {
          const T fl = T(fp[size_t(j1) * N]);
          const T fj = live ? fl : T(0);
          acc[j1] -= (wp * fj - x[j1].y) * x[j1].x;
        }
      };
      if (a.f_fp32) loss(opaque_global(static_cast<const float*>(a.f) + fbase + r));
      else loss(opaque_global(static_cast<const double*>(a.f) + fbase + r));
    } else {
      // the angle's weight is in its multipliers (sqrt|w| on each part)
#pragma unroll
      for (int j1 = 0; j1 < N; ++j1) acc[j1] += x[j1].x * x[j1].y;
    }
  }
  const long orow = a.scatter ? row : long(cell);
  const size_t obase = size_t(orow) * N * N;
  bool bad = false;
  if (a.project) {
    // moments of Q = C acc over the cell (per lane, then across its n lanes,
    // a fixed order), lambda = G^-1 m, q = Q - (l0 + l1 v1 + l2 v2 + l3 |v|^2)
    const double v2 = (r - N / 2) * a.dv;
    double m[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int j1 = 0; j1 < N; ++j1) {
      const double v1 = (j1 - N / 2) * a.dv;
      const double qv = a.C * double(acc[j1]);
      m[0] += qv;
      m[1] += v1 * qv;
      m[2] += v2 * qv;
      m[3] += (v1 * v1 + v2 * v2) * qv;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int o = N / 2; o > 0; o >>= 1) m[k] += __shfl_xor(m[k], o);
    double lam[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < 4; ++k) s += a.ginv[4 * i + k] * m[k];
      lam[i] = s;
    }
    double* q = static_cast<double*>(a.q) + obase;
#pragma unroll
    for (int j1 = 0; j1 < N; ++j1) {
      const double v1 = (j1 - N / 2) * a.dv;
      const double ov = a.C * double(acc[j1]) - (lam[0] + lam[1] * v1 + lam[2] * v2 + lam[3] * (v1 * v1 + v2 * v2));
      if (live) q[size_t(j1) * N + r] = ov;
      bad |= live && !isfinite(ov);
    }
  } else {
    T* q = static_cast<T*>(a.q) + obase;
#pragma unroll
    for (int j1 = 0; j1 < N; ++j1) {
      const T ov = T(a.C) * acc[j1];
      if (live) q[size_t(j1) * N + r] = ov;
      bad |= live && !isfinite(ov);
    }
  }
  if (bad && a.status) a.status[threadIdx.x * a.zero] = 1;
}

template <typename T, int N>
void launch2d(const Args2D& a, int ncells, hipStream_t s) {
  constexpr int G = 64 / N;
  hipLaunchKernelGGL((k_collide2d<T, N>), dim3(static_cast<unsigned>((ncells + G - 1) / G)), dim3(64), 0, s, a);
}

}  // namespace

namespace bz {

bz_status launch_collide2d(const bz_plan* p, const Binding& b, const void* f, int f_fp32, const int32_t* idx,
                           int ncells, const int32_t* ncells_dev, void* q, int scatter, hipStream_t s, bool timed) {
  bz_plan* pm = const_cast<bz_plan*>(p);
  Args2D a{};
  a.ncells = ncells;
  a.ncells_dev = ncells_dev;
  a.f = f;
  a.f_fp32 = f_fp32;
  a.idx = idx;
  a.scatter = scatter;
  a.mult = b.tables;
  a.w = static_cast<const char*>(b.tables) + p->table_w_off;
  a.fs = static_cast<char*>(b.ws) + b.lay.fh_off;
  a.fs_stride = b.lay.fh_cell / (p->fp32 ? 8 : 16);
  a.m1 = p->m1;
  a.C = p->C;
  a.dv = p->dv;
  for (int i = 0; i < 16; ++i) a.ginv[i] = p->ginv[i];
  a.project = p->project;
  a.q = q;
  a.status = reinterpret_cast<int32_t*>(static_cast<char*>(b.ws) + b.lay.status_off);
  a.zero = 0;
  if (timed) {
    // one fused kernel: the forward share is reported as zero
    pm->ev = &pm->evs[4 * (pm->timed_calls % bz_plan::kTimingSlots)];
    (void)hipEventRecord(pm->ev[0], s);
    (void)hipEventRecord(pm->ev[1], s);
  }
  switch (p->n * 2 + (p->fp32 ? 1 : 0)) {
    case 16 * 2 + 1: launch2d<float, 16>(a, ncells, s); break;
    case 32 * 2 + 1: launch2d<float, 32>(a, ncells, s); break;
    case 64 * 2 + 1: launch2d<float, 64>(a, ncells, s); break;
    case 16 * 2: launch2d<double, 16>(a, ncells, s); break;
    case 32 * 2: launch2d<double, 32>(a, ncells, s); break;
    default: return fail(BZ_ERR_UNSUPPORTED, "two-dimensional plan: n=%d precision=%s", p->n, p->fp32 ? "fp32" : "fp64");
  }
  if (timed) {
    (void)hipEventRecord(pm->ev[2], s);
    (void)hipEventRecord(pm->ev[3], s);
    pm->timed_calls += 1;
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(BZ_ERR_DEVICE, "bz_collide_batch: launch failed: %s", hipGetErrorString(e));
  return BZ_OK;
}

}  // namespace bz
