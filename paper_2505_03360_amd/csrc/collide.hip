// Kernels of the fast spectral collision operator (Sec. 4.4.1) for gfx950.
//
// Per cell, with fhat = DFT(f)/n^3 and, for every direction p:
//   X_p = (s_p alpha_p + i alpha'_p / s_p) * fhat   (real, even multipliers,
//                                                    zero on the Nyquist planes)
//   Y_p = IDFT(X_p) = s_p IDFT(alpha_p fhat) + i IDFT(alpha'_p fhat) / s_p
//   acc += w_p * Re(Y_p) * Im(Y_p)
// Both inverse transforms of a direction are real, so one complex transform
// carries the pair; the balance factor s_p leaves the product unchanged and
// equalises the rounding of the two parts.  The loss pass carries
// X = (Bhat_M / sL + i sL [Nyquist]) fhat, i.e. Y = Lambda/sL + i sL fNyq with
// fNyq the Nyquist-mode part of f, and adds -(sL f - Im Y) Re Y =
// -(f - fNyq) Lambda = -fN Lambda, the loss term of the truncated series,
// formed with the exact input f.  The result kernel_c * acc is Q(f,f); the
// FP64 projection kernel removes its component along the five collision
// invariants.
//
// Layouts (per cell, n^3 entries): f and q [i1][i2][i3]; fhat, multipliers
// [k2][k3][k1] (k1 fastest, so that stage-A pencils along k3 are read with
// consecutive lanes on consecutive k1); acc [j1][j2][j3].
//
// Evaluation strategies (all share the multiplier tables and the projection):
//   fused (FP32, n = 16 and 32): one forward kernel, then one workgroup per
//          (cell, direction chunk) runs every direction of its chunk on chip:
//          stage-A pencils along k3 in registers, a transpose through LDS in
//          j3 slices, stage-B pencils along k2, a wave-local transpose,
//          stage-C pencils along k1, products accumulated in registers; the
//          projection or an IMEX update can run in the same kernel;
//   chunked plain (FP32 plans that use no fused kernel, and every FP64
//          plan): the stage-A pass writes K directions' intermediates at
//          once, a second kernel runs stages B and C with the B->C transpose
//          in LDS and accumulates over the chunk;
//   dealiased (either precision): f is resampled spectrally onto a 3n/2 grid,
//          the plain or chunked passes run there, and the result is
//          resampled back onto the n grid.
#include "bz_internal.hpp"
#include "fft.hpp"
#include "gptr.hpp"
#include "kinetic.hpp"

using bzk::cx;
using bzk::gptr;
using bzk::opaque_global;

namespace {

__device__ __forceinline__ int live_count(int ncells, const int32_t* ncells_dev) {
  int c = ncells;
  if (ncells_dev) {
    const int d = *ncells_dev;
    c = d < c ? d : c;
    if (c < 0) c = 0;
  }
  return c;
}

// Records a non-finite output in the status word.  The address depends on the
// lane through a run-time zero, so the store is a vector store.
__device__ __forceinline__ void flag_nonfinite(int32_t* status, int zero, bool bad) {
  if (bad && status) status[threadIdx.x * zero] = 1;
}

__global__ void k_clear_status(int32_t* status, int zero) {
  if (threadIdx.x == 0) status[threadIdx.x * zero] = 0;
}

template <typename T>
struct PlainArgs {
  const void* f;
  int f_fp32;
  const int32_t* idx;
  int ncells;
  const int32_t* ncells_dev;
  cx<T>* fh;  // [cell][k2][k3][k1]
  cx<T>* y;   // [cell][...]
  T* acc;     // [cell][...]: plane-major [j3][j1][j2] (chunked passes) or [j1][j2][j3] (resampling)
  size_t fh_stride, y_stride, acc_stride;  // elements per cell
  const cx<T>* mult;  // [pass][k2][k3][k1]
  const T* w;         // [pass]
  int pass;
  int first;  // the chunk starting at pass 0 (initialises the accumulator)
  int chunk;  // directions per chunk (stage-A volumes per cell in y)
  int m1;     // passes (directions + the loss pass)
  const float* dft;  // DFT-as-GEMM plans: matrix-core operand fragments of the inverse DFT
};

// ------------------------------------------------------------------ forward
// pass 1: pencils along i1, thread (cell, i2, i3); f -> y[cell][k1][i2][i3]
template <typename T, int N>
__global__ __launch_bounds__(256) void k_fwd1(PlainArgs<T> a) {
  const long g = long(blockIdx.x) * blockDim.x + threadIdx.x;
  const int c = int(g / (N * N));
  const int rem = int(g % (N * N));
  if (c >= live_count(a.ncells, a.ncells_dev)) return;
  const int i2 = rem / N, i3 = rem % N;
  const long row = a.idx ? long(a.idx[c]) : long(c);
  const size_t base = size_t(row) * N * N * N + size_t(i2) * N + i3;
  cx<T> x[N];
  if (a.f_fp32) {
    const float* f = static_cast<const float*>(a.f) + base;
#pragma unroll
    for (int i1 = 0; i1 < N; ++i1) x[i1] = {T(f[size_t(i1) * N * N]), T(0)};
  } else {
    const double* f = static_cast<const double*>(a.f) + base;
#pragma unroll
    for (int i1 = 0; i1 < N; ++i1) x[i1] = {T(f[size_t(i1) * N * N]), T(0)};
  }
  bzk::fft<N, -1>(x);
  cx<T>* y = a.y + c * a.y_stride + size_t(i2) * N + i3;
#pragma unroll
  for (int k1 = 0; k1 < N; ++k1) y[size_t(k1) * N * N] = x[k1];
}

// pass 2: pencils along i2, thread (cell, k1, i3), in place in y
template <typename T, int N>
__global__ __launch_bounds__(256) void k_fwd2(PlainArgs<T> a) {
  const long g = long(blockIdx.x) * blockDim.x + threadIdx.x;
  const int c = int(g / (N * N));
  const int rem = int(g % (N * N));
  if (c >= live_count(a.ncells, a.ncells_dev)) return;
  const int k1 = rem / N, i3 = rem % N;
  cx<T>* y = a.y + c * a.y_stride + size_t(k1) * N * N + i3;
  cx<T> x[N];
#pragma unroll
  for (int i2 = 0; i2 < N; ++i2) x[i2] = y[i2 * N];
  bzk::fft<N, -1>(x);
#pragma unroll
  for (int k2 = 0; k2 < N; ++k2) y[k2 * N] = x[k2];
}

// pass 3: pencils along i3, thread (cell, k2, k1); scale by n^-3 and
// write fhat[cell][k2][k3][k1] with the Nyquist modes kept (the loss pass uses them)
template <typename T, int N>
__global__ __launch_bounds__(256) void k_fwd3(PlainArgs<T> a) {
  const long g = long(blockIdx.x) * blockDim.x + threadIdx.x;
  const int c = int(g / (N * N));
  const int rem = int(g % (N * N));
  if (c >= live_count(a.ncells, a.ncells_dev)) return;
  const int k2 = rem / N, k1 = rem % N;
  const cx<T>* y = a.y + c * a.y_stride + size_t(k1) * N * N + size_t(k2) * N;
  cx<T> x[N];
#pragma unroll
  for (int i3 = 0; i3 < N; ++i3) x[i3] = y[i3];
  bzk::fft<N, -1>(x);
  const T scale = T(1.0 / (double(N) * N * N));
  cx<T>* fh = a.fh + c * a.fh_stride + size_t(k2) * N * N + k1;
#pragma unroll
  for (int k3 = 0; k3 < N; ++k3) fh[size_t(k3) * N] = cx<T>{x[k3].x * scale, x[k3].y * scale};
}

// Streaming (non-temporal) access to a complex value: for data touched once
// per launch, so that it does not evict what the launch re-reads from L2.
template <typename T>
__device__ __forceinline__ void nt_store(cx<T>* p, cx<T> v) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  v2 w;
  w.x = v.x;
  w.y = v.y;
  __builtin_nontemporal_store(w, reinterpret_cast<v2*>(p));
}
template <typename T>
__device__ __forceinline__ cx<T> nt_load(const cx<T>* p) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  const v2 w = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
  return cx<T>{w.x, w.y};
}

// ------------------------------------------------------------------ pencil pass along k2
// inverse along k2 in place (the middle pass of the spectral resampling);
// y[cell][k2][j3][k1] -> y[cell][j2][j3][k1]; thread (cell, j3, k1)
template <typename T, int N>
__global__ __launch_bounds__(256) void k_dirB(PlainArgs<T> a) {
  const long g = long(blockIdx.x) * blockDim.x + threadIdx.x;
  const int c = int(g / (N * N));
  const int rem = int(g % (N * N));
  if (c >= live_count(a.ncells, a.ncells_dev)) return;
  const int j3 = rem / N, k1 = rem % N;
  cx<T>* y = a.y + c * a.y_stride + size_t(j3) * N + k1;
  cx<T> x[N];
#pragma unroll
  for (int k2 = 0; k2 < N; ++k2) x[k2] = y[size_t(k2) * N * N];
  bzk::fft<N, 1>(x);
#pragma unroll
  for (int j2 = 0; j2 < N; ++j2) y[size_t(j2) * N * N] = x[j2];
}

// ------------------------------------------------------------------ spectral resampling
// Inverse transform on an NO-point grid of a spectrum given on NI points
// (fhat layout [k2][k3][k1]), keeping the modes |ktilde| < min(NI, NO)/2 and
// zero elsewhere: the truncated series re-sampled on the other grid (the 3/2
// rule of the dealiased plans).  Three pencil passes like the plain path:
// k_rsA (along k3, with the mode map), k_dirB (along k2), k_rsC (along k1,
// real part to a[cell][j1][j2][j3]).
template <int NI, int NO>
__device__ __forceinline__ int rs_map(int k) {  // NO-axis index -> NI-axis index, or -1 outside the band
  constexpr int B = (NI < NO ? NI : NO) / 2;
  const int kt = k < NO / 2 ? k : k - NO;
  if (kt >= B || kt <= -B) return -1;
  return kt >= 0 ? kt : kt + NI;
}

template <typename T, int NI, int NO>
__global__ __launch_bounds__(256) void k_rsA(PlainArgs<T> a) {
  const long g = long(blockIdx.x) * blockDim.x + threadIdx.x;
  const int c = int(g / (NO * NO));
  const int rem = int(g % (NO * NO));
  if (c >= live_count(a.ncells, a.ncells_dev)) return;
  const int k2 = rem / NO, k1 = rem % NO;
  const int m2 = rs_map<NI, NO>(k2), m1 = rs_map<NI, NO>(k1);
  cx<T> x[NO];
  if (m1 >= 0 && m2 >= 0) {
    const cx<T>* gin = a.fh + c * a.fh_stride + size_t(m2) * NI * NI + m1;
#pragma unroll
    for (int k3 = 0; k3 < NO; ++k3) {
      const int m3 = rs_map<NI, NO>(k3);
      x[k3] = m3 >= 0 ? gin[size_t(m3) * NI] : cx<T>{T(0), T(0)};
    }
    bzk::fft<NO, 1>(x);
  } else {
#pragma unroll
    for (int j3 = 0; j3 < NO; ++j3) x[j3] = cx<T>{T(0), T(0)};
  }
  cx<T>* y = a.y + c * a.y_stride + size_t(k2) * NO * NO + k1;
#pragma unroll
  for (int j3 = 0; j3 < NO; ++j3) y[size_t(j3) * NO] = x[j3];
}

template <typename T, int NO>
__global__ __launch_bounds__(256) void k_rsC(PlainArgs<T> a) {
  const long g = long(blockIdx.x) * blockDim.x + threadIdx.x;
  const int c = int(g / (NO * NO));
  const int rem = int(g % (NO * NO));
  if (c >= live_count(a.ncells, a.ncells_dev)) return;
  const int j2 = rem / NO, j3 = rem % NO;
  const cx<T>* y = a.y + c * a.y_stride + size_t(j2) * NO * NO + size_t(j3) * NO;
  cx<T> x[NO];
#pragma unroll
  for (int k1 = 0; k1 < NO; ++k1) x[k1] = y[k1];
  bzk::fft<NO, 1>(x);
  T* out = a.acc + c * a.acc_stride + size_t(j2) * NO + j3;
#pragma unroll
  for (int j1 = 0; j1 < NO; ++j1) out[size_t(j1) * NO * NO] = x[j1].x;
}

// ------------------------------------------------------------------ chunked plain passes
// Two kernels per chunk of directions, for the sizes and strategies without a
// fused kernel:
//   k_pA:  thread (cell, k2, k1) loads its fhat pencil along k3 once and, for
//          each direction d of the chunk, writes the inverse along k3 of
//          M_p fhat to y[cell][d][j3][k2][k1] (planes of fixed j3 contiguous);
//   k_pBC: one wave per 64/N planes of fixed j3: pencils along k2 read from
//          y, inverse, transpose through LDS inside the workgroup, inverse along
//          k1, products accumulated in registers over the chunk, accumulator
//          kept plane-major acc[cell][j3][j1][j2].
// Per cell and direction this moves fhat/K + y twice + acc twice/K (K the
// chunk, the plan's pchunk) instead of fhat + y four times + acc twice.  k_pA
// streams fhat in and y out past the L2 (non-temporal), which keeps the
// chunk's multiplier tables, shared by every cell, resident there.

// k_pA's XCD-aware block order (the share is the items per XCD).  It needs a
// cell's pencils to fill whole 256-thread blocks and is taken where it was
// measured faster: FP64 at N = 48, whose four-direction chunk of tables
// (7 MB) otherwise streams from the Infinity Cache for every cell (1024
// cells, M = 32: 44.7 -> 36.6 ms).  FP32 at N = 48 lost 2 % with it and FP64
// at N = 32 10 %; FP32 at N = 32 gained 2 %.
template <typename T, int N>
constexpr bool pa_xcd_order() { return (N * N) % 256 == 0 && sizeof(T) == 8 && N == 48; }
__host__ __device__ inline long pa_xcd_share(long total) { return (total + 7) / 8; }

template <typename T, int N>
__global__ __launch_bounds__(256) void k_pA(PlainArgs<T> a) {
  int c, rem;
  if constexpr (pa_xcd_order<T, N>()) {
    // work items (range of 256 pencils, cell) in range-major order, each of
    // the 8 XCDs (blocks are dealt round-robin over them) taking one
    // contiguous share: an XCD works on one or two pencil ranges at a time, so
    // the multiplier tables of those ranges stay in its L2 for every cell
    constexpr int RB = N * N / 256;
    const long total = long(a.ncells) * RB;
    const long item = long(blockIdx.x % 8) * pa_xcd_share(total) + blockIdx.x / 8;
    if (item >= total) return;
    c = int(item % a.ncells);
    rem = int(item / a.ncells) * 256 + int(threadIdx.x);
  } else {
    const long g = long(blockIdx.x) * blockDim.x + threadIdx.x;
    c = int(g / (N * N));
    rem = int(g % (N * N));
  }
  if (c >= live_count(a.ncells, a.ncells_dev)) return;
  const int k2 = rem / N, k1 = rem % N;
  const size_t off = size_t(k2) * N * N + k1;
  const cx<T>* fh = a.fh + c * a.fh_stride + off;
  cx<T> F[N];
#pragma unroll
  for (int k3 = 0; k3 < N; ++k3) F[k3] = nt_load(fh + size_t(k3) * N);
  for (int d = 0; d < a.chunk; ++d) {
    const int p = a.pass + d;
    if (p >= a.m1) break;
    const cx<T>* mu = a.mult + size_t(p) * N * N * N + off;
    cx<T> x[N];
#pragma unroll
    for (int k3 = 0; k3 < N; ++k3) {
      const cx<T> M = mu[size_t(k3) * N];
      x[k3] = {M.x * F[k3].x - M.y * F[k3].y, M.x * F[k3].y + M.y * F[k3].x};
    }
    bzk::fft<N, 1>(x);
    cx<T>* y = a.y + c * a.y_stride + size_t(d) * N * N * N + size_t(k2) * N + k1;
#pragma unroll
    for (int j3 = 0; j3 < N; ++j3) nt_store(y + size_t(j3) * N * N, x[j3]);
  }
}

// Planes of fixed j3 per k_pBC workgroup, one thread per pencil: the largest
// divisor of N whose planes fit 256 threads (N = 16: 16 planes, 24: 8 on 192
// threads, 32: 8, 48: 4 on 192 threads), so every lane of the workgroup is busy.
template <int N>
constexpr int plain_planes_per_group() {
  int pw = 1;
  for (int d = 1; d * N <= 256; ++d)
    if (N % d == 0) pw = d;
  return pw;
}

template <typename T, int N>
__global__ __launch_bounds__(256, 2) void k_pBC(PlainArgs<T> a) {
  constexpr int PW = plain_planes_per_group<N>();  // planes per workgroup
  constexpr int NG = N / PW;                       // workgroups per cell
  static_assert(N % PW == 0 && PW * N <= 256, "planes must tile the cell");
  __shared__ cx<T> tr[PW][N][N + 1];  // [plane][j2][k1], odd pitch
  const int c = blockIdx.x / NG, grp = blockIdx.x % NG;
  if (c >= live_count(a.ncells, a.ncells_dev)) return;
  const int t = threadIdx.x;
  const int pl = t / N;  // the block holds exactly PW * N threads
  const int k = t % N;   // stage B: k1; stage C: j2
  const int j3 = grp * PW + pl;
  T* acc = a.acc + c * a.acc_stride + size_t(j3) * N * N;  // [j1][j2] of plane j3
  T accr[N];
#pragma unroll
  for (int j1 = 0; j1 < N; ++j1) accr[j1] = !a.first ? acc[size_t(j1) * N + k] : T(0);
  const long row = a.idx ? long(a.idx[c]) : long(c);
#pragma unroll 1
  for (int d = 0; d < a.chunk; ++d) {
    const int p = a.pass + d;
    if (p >= a.m1) break;
    const T wp = a.w[p];
    {
      const gptr<cx<T>> y = opaque_global(a.y + c * a.y_stride + size_t(d) * N * N * N + size_t(j3) * N * N + k);
      cx<T> x[N];
#pragma unroll
      for (int k2 = 0; k2 < N; ++k2) x[k2] = y[k2 * N];
      bzk::fft<N, 1>(x);
#pragma unroll
      for (int j2 = 0; j2 < N; ++j2) tr[pl][j2][k] = x[j2];
    }
    __syncthreads();
    {
      cx<T> x[N];
#pragma unroll
      for (int r = 0; r < N; ++r) {
        const int k1 = bzk::first_stage_order<N>(r);
        x[k1] = tr[pl][k][k1];
      }
      bzk::fft<N, 1>(x);
      if (p == a.m1 - 1) {
        // loss pass: acc -= (sL f - Im) Re with the exact input f at (j1, j2 = k, j3)
        const size_t fb = size_t(row) * N * N * N + size_t(k) * N + j3;
        if (a.f_fp32) {
          const gptr<float> fp = opaque_global(static_cast<const float*>(a.f) + fb);
#pragma unroll
          for (int j1 = 0; j1 < N; ++j1) accr[j1] -= (wp * T(fp[j1 * N * N]) - x[j1].y) * x[j1].x;
        } else {
          const gptr<double> fp = opaque_global(static_cast<const double*>(a.f) + fb);
#pragma unroll
          for (int j1 = 0; j1 < N; ++j1) accr[j1] -= (wp * T(fp[j1 * N * N]) - x[j1].y) * x[j1].x;
        }
      } else {
#pragma unroll
        for (int j1 = 0; j1 < N; ++j1) accr[j1] += wp * x[j1].x * x[j1].y;
      }
    }
    __syncthreads();  // tr is rewritten by the next direction
  }
#pragma unroll
  for (int j1 = 0; j1 < N; ++j1) acc[size_t(j1) * N + k] = accr[j1];
}

// DFT as a matrix product on the matrix cores (BZ_XF_DFT_GEMM plans, FP32):
// k_pBC with stage C (the length-N inverse transforms along k1 of every j3
// plane) evaluated as Y = W X by v_mfma_f32_16x16x4_f32, W[j1][k1] =
// exp(+2 pi i j1 k1 / N).  Complex arithmetic in real form: K = 2N rows
// [Re X; Im X], Re Y = [Re W | -Im W] [Re X; Im X] and Im Y = [Im W | Re W] [Re
// X; Im X].  Operand layouts of the 16x16x4 instruction (64 lanes, l): A[i][k]
// with i = l % 16, k = l / 16; B[k][j] with j = l % 16, k = l / 16; D[i][j]
// with j = l % 16, i = 4 (l / 16) + r in result register r.  The A operands
// come from a fragment table in the plan's tables, [Re/Im part][row tile mt]
// [k step ks][lane], so each is one coalesced load; the B operands are the
// stage-B outputs in LDS.  A wave owns (plane, column tile) tasks and keeps
// their products accumulated in registers in D layout: (j1, j2) = (16 mt +
// 4 (l / 16) + r, 16 nt + l % 16).  The matrix product executes 8N flop per
// point against the FFT's 5 log2 N.
template <int N>
__global__ __launch_bounds__(256, 2) void k_pBC_mm(PlainArgs<float> a) {
  constexpr int PW = plain_planes_per_group<N>();
  constexpr int NG = N / PW;
  constexpr int NT = N / 16, MT = N / 16, KS = N / 2;
  constexpr int NW = PW * N / 64;              // waves per workgroup
  constexpr int TPW = PW * NT / NW;            // (plane, column tile) tasks per wave
  static_assert(N % 16 == 0 && (PW * N) % 64 == 0 && (PW * NT) % NW == 0, "whole tiles and waves");
  typedef float f4 __attribute__((ext_vector_type(4)));
  __shared__ cx<float> tr[PW][N][N + 1];  // [plane][j2][k1], odd pitch
  const int c = blockIdx.x / NG, grp = blockIdx.x % NG;
  if (c >= live_count(a.ncells, a.ncells_dev)) return;
  const int t = threadIdx.x;
  const int pl = t / N, k = t % N;  // stage B: plane, k1
  const int w = t / 64, l = t % 64;
  float* acc = a.acc + c * a.acc_stride;
  float accr[TPW][MT][4];
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    const int tk = w + i * NW, q = tk / NT, nt = tk % NT;
    const int j3 = grp * PW + q, j2 = 16 * nt + l % 16;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        accr[i][mt][r] = !a.first ? acc[size_t(j3) * N * N + size_t(16 * mt + 4 * (l / 16) + r) * N + j2] : 0.0f;
  }
  const long row = a.idx ? long(a.idx[c]) : long(c);
#pragma unroll 1
  for (int d = 0; d < a.chunk; ++d) {
    const int p = a.pass + d;
    if (p >= a.m1) break;
    const float wp = a.w[p];
    {
      const int j3 = grp * PW + pl;
      const gptr<cx<float>> y = opaque_global(a.y + c * a.y_stride + size_t(d) * N * N * N + size_t(j3) * N * N + k);
      cx<float> x[N];
#pragma unroll
      for (int k2 = 0; k2 < N; ++k2) x[k2] = y[k2 * N];
      bzk::fft<N, 1>(x);
#pragma unroll
      for (int j2 = 0; j2 < N; ++j2) tr[pl][j2][k] = x[j2];
    }
    __syncthreads();
    const gptr<float> fr = opaque_global(a.dft + l);
#pragma unroll 1
    for (int i = 0; i < TPW; ++i) {
      const int tk = w + i * NW, q = tk / NT, nt = tk % NT;
      const int j3 = grp * PW + q, j2 = 16 * nt + l % 16;
      float b[KS];  // rows 4 ks + l / 16 of [Re X; Im X] in column j2
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int kk = 4 * ks + l / 16;
        b[ks] = (4 * ks < N) ? tr[q][j2][kk].x : tr[q][j2][kk - N].y;
      }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        f4 dr = {0.0f, 0.0f, 0.0f, 0.0f}, di = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          const float ar = fr[((0 * MT + mt) * KS + ks) * 64];
          const float ai = fr[((1 * MT + mt) * KS + ks) * 64];
          dr = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, b[ks], dr, 0, 0, 0);
          di = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, b[ks], di, 0, 0, 0);
        }
        if (p == a.m1 - 1) {
          // loss pass: acc -= (sL f - Im) Re with the exact input f at (j1, j2, j3)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const size_t e = size_t(row) * N * N * N + size_t(16 * mt + 4 * (l / 16) + r) * N * N + size_t(j2) * N + j3;
            const float fv = a.f_fp32 ? static_cast<const float*>(a.f)[e] : float(static_cast<const double*>(a.f)[e]);
            accr[i][mt][r] -= (wp * fv - di[r]) * dr[r];
          }
        } else {
#pragma unroll
          for (int r = 0; r < 4; ++r) accr[i][mt][r] += wp * dr[r] * di[r];
        }
      }
    }
    __syncthreads();  // tr is rewritten by the next direction
  }
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    const int tk = w + i * NW, q = tk / NT, nt = tk % NT;
    const int j3 = grp * PW + q, j2 = 16 * nt + l % 16;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[size_t(j3) * N * N + size_t(16 * mt + 4 * (l / 16) + r) * N + j2] = accr[i][mt][r];
  }
}

// ------------------------------------------------------------------ fused FP32

// Workgroup barrier that orders LDS traffic only: global loads issued before
// it stay in flight (a full __syncthreads would wait for them).
// Orders one wave's LDS accesses across its lanes (the wave runs in lockstep;
// this only keeps the compiler from moving LDS accesses across it and waits
// for the wave's outstanding LDS operations).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

struct FusedArgs {
  int ncells;
  const int32_t* ncells_dev;
  const float* fc;    // [cell][slice][j1][thread]: FP32 copy of f in stage-C order (loss pass)
  size_t fc_stride;
  const int32_t* idx;
  const cx<float>* fh;
  size_t fh_stride;
  float* acc;
  size_t acc_stride;  // per cell (all chunks)
  const cx<float>* mult;
  const float* w;
  int m1, chunks;
  // epilogue with the conservative projection (single-chunk plans)
  int fuse_project;
  int scatter;
  double C, dv;
  double ginv[25];
  double* q;
  int32_t* status;   // set to 1 when a non-finite value is written
  int zero;           // 0 at run time: keeps the status store a per-lane (vector) store
  int imex;           // write the IMEX update of eq. (4.24) instead of Q (projection epilogue only;
                      // selects the IMEX instantiation of the kernel)
  bzk::ImexDev im;
};

// ------------------------------------------------------------------ fused forward
struct FwdArgs {
  int ncells;
  const int32_t* ncells_dev;
  const void* f;
  int f_fp32;
  const int32_t* idx;
  cx<float>* fh;  // [cell][k2][k3][k1]
  size_t fh_stride;
  int mirror;  // also write rows k2 in (N/2, N) (consumers that read every row)
  float* fc;   // [cell][slice][j1][t]: FP32 f in the collision kernel's stage-C order
  size_t fc_stride;
};

// Forward transform fhat = DFT(f) / N^3 of one cell per workgroup, FP32,
// N^2/2 threads, everything between the load of f and the write of fhat on
// chip.
//   stage 0: f is read once, coalesced, into LDS as FP32 ([i1][i2][i3], row
//            pitch N + 1), and written back out as fc in the order in which
//            the collision kernel's threads consume it in the loss pass:
//            fc[s][j1][t] = f[j1][t % N][s W + t / N] (W = N / S, S the
//            slices of that kernel), so that those reads are coalesced;
//   stage 1: thread (i1 < N/2, i3) transforms z(i2) = f[i1][i2][i3] +
//            i f[i1 + N/2][i2][i3] along i2; f is real, so the two transforms
//            follow from Z(k2) and conj Z(-k2).  Only k2 in [0, N/2] is kept:
//            fhat(-k) = conj fhat(k) gives the other rows.
//   stage 2: pencils along i1 at (k2, i3), in place in LDS.
//   stage 3: pencils along i3 at (k2, k1); scaled, written to fhat[k2][k3][k1]
//            (lanes on k1); with `mirror`, rows N - k2 (0 < k2 < N/2) are
//            written as conj fhat(-k1, k2, -k3).
// LDS [k2 in 0..N/2][i1, then k1][i3] with row pitch N + 1 (stage 3 reads with
// lanes on k1 and lands on distinct banks).
template <int N, int S>
__global__ __launch_bounds__(N * N / 2) void k_fwd_fused(FwdArgs a) {
  constexpr int T = N * N / 2, H = N / 2, P = N + 1;
  __shared__ cx<float> lds[(H + 1) * N * P];
  const int cell = blockIdx.x;
  if (cell >= live_count(a.ncells, a.ncells_dev)) return;
  const int t = threadIdx.x;
  const long row = a.idx ? long(a.idx[cell]) : long(cell);
  constexpr int N3 = N * N * N;
  static_assert(N * N * P <= 2 * (H + 1) * N * P, "f fits the LDS as FP32");
  float* lf = reinterpret_cast<float*>(lds);  // [i1][i2][i3], row pitch P
  if (a.f_fp32) {
    const float* f = static_cast<const float*>(a.f) + size_t(row) * N3;
#pragma unroll 8
    for (int e = t; e < N3; e += T) lf[(e / N) * P + e % N] = f[e];
  } else {
    const double* f = static_cast<const double*>(a.f) + size_t(row) * N3;
#pragma unroll 8
    for (int e = t; e < N3; e += T) lf[(e / N) * P + e % N] = float(f[e]);
  }
  lds_barrier();
  {
    constexpr int W = N / S, TC = N * W;
    float* fc = a.fc + cell * a.fc_stride;
#pragma unroll 8
    for (int o = t; o < N3; o += T) {
      const int tc = o % TC, j1 = (o / TC) % N, sl = o / (N * TC);
      const int j2 = tc % N, j3 = sl * W + tc / N;
      fc[o] = lf[(j1 * N + j2) * P + j3];
    }
  }
  {
    const int i3 = t % N, i1 = t / N;
    cx<float> z[N];
#pragma unroll
    for (int i2 = 0; i2 < N; ++i2) z[i2] = {lf[(i1 * N + i2) * P + i3], lf[((i1 + H) * N + i2) * P + i3]};
    lds_barrier();  // every thread has its rows: the LDS is reused below
    bzk::fft<N, -1>(z);
#pragma unroll
    for (int k2 = 0; k2 <= H; ++k2) {
      const cx<float> zp = z[k2], zm = z[(N - k2) % N];
      // transform of row i1: (Z(k) + conj Z(-k)) / 2; of row i1 + N/2: (Z(k) - conj Z(-k)) / 2i
      lds[(k2 * N + i1) * P + i3] = cx<float>{0.5f * (zp.x + zm.x), 0.5f * (zp.y - zm.y)};
      lds[(k2 * N + i1 + H) * P + i3] = cx<float>{0.5f * (zp.y + zm.y), 0.5f * (zm.x - zp.x)};
    }
  }
  lds_barrier();
  for (int q = t; q < (H + 1) * N; q += T) {
    const int k2 = q / N, i3 = q % N;
    cx<float> x[N];
#pragma unroll
    for (int r = 0; r < N; ++r) {
      const int i1 = bzk::first_stage_order<N>(r);
      x[i1] = lds[(k2 * N + i1) * P + i3];
    }
    bzk::fft<N, -1>(x);
#pragma unroll
    for (int k1 = 0; k1 < N; ++k1) lds[(k2 * N + k1) * P + i3] = x[k1];
  }
  lds_barrier();
  const float scale = 1.0f / float(N * N * N);
  cx<float>* fh = a.fh + cell * a.fh_stride;
  for (int q = t; q < (H + 1) * N; q += T) {
    const int k2 = q / N, k1 = q % N;
    cx<float> x[N];
#pragma unroll
    for (int r = 0; r < N; ++r) {
      const int i3 = bzk::first_stage_order<N>(r);
      x[i3] = lds[(k2 * N + k1) * P + i3];
    }
    bzk::fft<N, -1>(x);
#pragma unroll
    for (int k3 = 0; k3 < N; ++k3)
      fh[(size_t(k2) * N + k3) * N + k1] = cx<float>{x[k3].x * scale, x[k3].y * scale};
    if (a.mirror && k2 > 0 && k2 < H) {
      const int mk1 = (N - k1) % N;
#pragma unroll
      for (int k3 = 0; k3 < N; ++k3)
        fh[(size_t(N - k2) * N + (N - k3) % N) * N + mk1] = cx<float>{x[k3].x * scale, -x[k3].y * scale};
    }
  }
}

// N^2/S threads; S j3-slices of width W = N/S.
//   stage A: thread t owns pencils P = a*T + t (a < S) along k3 at
//            (k1, k2) = (P % N, P / N);
//   stage B: thread t owns, in every slice, the pencil along k2 at
//            (k1, j3) = (t % N, s*W + t / N);
//   stage C: thread t owns, in every slice, the pencil along k1 at
//            (j2, j3) = (t % N, s*W + t / N) and keeps its n products.
// LDS A->B: [k2][k1][j3 % W] padded to W+1 (odd stride: the stage-A writers
// and the stage-B readers step k1 on lanes).  B->C reuses the slots of the
// wave's own planes, (j2, k1) at row (N+1) j2 + k1 (N-1 rows beyond the A->B
// data): a wave synchronises only with itself between stages B and C.
template <int N, int S, bool LOSS>
__device__ __forceinline__ void fused_pass(const FusedArgs& a, cx<float>* lds, const cx<float>* fhc,
                                           const float* fcc, int p, int t, float (&acc)[S][N]) {
  constexpr int T = N * N / S;
  constexpr int W = N / S;
  constexpr int AB = W + 1;
  // stage B: lane (k1, j3 % W) = (t % N, t / N); stage C: lane (j2, j3 % W) = (t % N, t / N).
  // When N divides 64, a wave's 64 lanes cover 64/N whole j3 planes and B -> C
  // stays inside the wave; otherwise (N = 24) planes straddle waves and the
  // transpose synchronises the workgroup.
  constexpr bool wave_planes = (64 % N == 0) && (W % (64 / N) == 0);
  static_assert(wave_planes || (T % 64 == 0 && S == 1), "planes that straddle waves need whole waves, one slice");
  const int tk = t % N, tj = t / N;
  const cx<float>* mp = a.mult + size_t(p) * N * N * N;
  [[maybe_unused]] const float wp = LOSS ? a.w[p] : 0.0f;
  // stage A: each pencil is loaded (the paired gain pencils in one batch of
  // loads, whose products start as the first loads land; the unpaired ones in
  // two halves, which measured faster there), transformed, and its slice-0
  // outputs go to LDS at once; the other slices stay in registers until their turn.
  // The loads and transforms of stage A touch registers only: a wave runs
  // them while other waves are still in the previous pass's stage C, and
  // waits (LDS free) only before its first LDS write.
  cx<float> rest[S > 1 ? S : 1][S > 1 ? N - W : 1];
  if constexpr (S == 2 && !LOSS) {
    // Mirror pairing (gain passes).  With M = a + ib (a, b real and even in k) and F of a
    // real f (Hermitian), thread (k1, k2), k2 < N/2, transforms U = a F and
    // V = b F along k3 once; then pencil (k1, k2) is IDFT(X) = U^ + i V^ and
    // its mirror (-k1, -k2), whose X(k3) = M(-k3) conj(F(-k3)), is
    // conj(U^) + i conj(V^).  One set of loads and two transforms give both.
    // Row k2 = 0 mirrors onto itself: its threads take row N/2 instead, which
    // is zero (the gain multipliers vanish on the Nyquist planes).  The loss
    // pass, whose multiplier is not zero there, takes the unpaired path.
    const int k1 = t % N, k2 = t / N;
    const bool row0 = k2 == 0;
    const int k1b = row0 ? k1 : (N - k1) % N;
    const int k2b = row0 ? N / 2 : N - k2;
    const size_t off = size_t(k2) * N * N + k1;
    cx<float> u[N], v[N];
    {
      const gptr<cx<float>> fb = opaque_global(fhc + off);
      const gptr<cx<float>> mb = opaque_global(mp + off);
#pragma unroll
      for (int k3 = 0; k3 < N; ++k3) {
        if (k3 == N / 2) {  // the gain multipliers vanish on the Nyquist plane: nothing to load
          u[k3] = v[k3] = cx<float>{0.0f, 0.0f};
          continue;
        }
        const cx<float> F = fb[k3 * N], Mu = mb[k3 * N];
        u[k3] = {Mu.x * F.x, Mu.x * F.y};
        v[k3] = {Mu.y * F.x, Mu.y * F.y};
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    bzk::fft<N, 1>(u);
    bzk::fft<N, 1>(v);
    // row 0's threads write their mirror values into row N/2 (where the gain
    // multipliers vanish), which stage B then reads as zeros
    auto out_b = [&](int j) -> cx<float> { return cx<float>{u[j].x + v[j].y, v[j].x - u[j].y}; };
    lds_barrier();  // LDS free: every wave's previous stage C has read it
#pragma unroll
    for (int j = 0; j < W; ++j) {
      lds[(k2 * N + k1) * AB + j] = cx<float>{u[j].x - v[j].y, u[j].y + v[j].x};
      lds[(k2b * N + k1b) * AB + j] = out_b(j);
    }
#pragma unroll
    for (int j = W; j < N; ++j) {
      rest[0][j - W] = cx<float>{u[j].x - v[j].y, u[j].y + v[j].x};
      rest[1][j - W] = out_b(j);
    }
  } else {
#pragma unroll
  for (int q = 0; q < S; ++q) {
    const int P = q * T + t;
    const int k1 = P % N, k2 = P / N;
    const size_t off = size_t(k2) * N * N + k1;
    // Opaque per-pass bases: keeps the compiler from hoisting the n
    // per-element addresses out of the pass loop (they would occupy 2n
    // registers); loads then use base + immediate offsets.
    const gptr<cx<float>> mb = opaque_global(mp + off);
    cx<float> x[N];
    if constexpr (S == 2) {
      // loss pass of the paired kernels: fhat holds rows k2 <= N/2 only; a row
      // above is read as its Hermitian mirror, fhat(k) = conj fhat(-k)
      const bool mir = k2 > N / 2;
      const size_t moff = size_t(mir ? N - k2 : k2) * N * N + (mir ? (N - k1) % N : k1);
      const gptr<cx<float>> fb = opaque_global(fhc + moff);
      const float sg = mir ? -1.0f : 1.0f;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int k3 = h * (N / 2); k3 < (h + 1) * (N / 2); ++k3) {
          const cx<float> Fr = fb[(mir ? (N - k3) % N : k3) * N];
          const cx<float> F = {Fr.x, sg * Fr.y};
          const cx<float> M = mb[k3 * N];
          x[k3] = {M.x * F.x - M.y * F.y, M.x * F.y + M.y * F.x};
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    } else {
      const gptr<cx<float>> fb = opaque_global(fhc + off);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int k3 = h * (N / 2); k3 < (h + 1) * (N / 2); ++k3) {
          if (!LOSS && k3 == N / 2) {  // the gain multipliers vanish on the Nyquist plane
            x[k3] = cx<float>{0.0f, 0.0f};
            continue;
          }
          const cx<float> F = fb[k3 * N];
          const cx<float> M = mb[k3 * N];
          x[k3] = {M.x * F.x - M.y * F.y, M.x * F.y + M.y * F.x};
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    bzk::fft<N, 1>(x);
    if (q == 0) lds_barrier();  // LDS free: every wave's previous stage C has read it
#pragma unroll
    for (int j = 0; j < W; ++j) lds[(k2 * N + k1) * AB + j] = x[j];
    if constexpr (S > 1) {
#pragma unroll
      for (int j = W; j < N; ++j) rest[q][j - W] = x[j];
    }
  }
  }
#pragma unroll
  for (int s = 0; s < S; ++s) {
    if (s > 0) {
      lds_barrier();  // stage C of the previous slice has read the LDS
#pragma unroll
      for (int q = 0; q < S; ++q) {
        int k1, k2;
        if constexpr (S == 2 && !LOSS) {
          const int ka = t % N, kb = t / N;
          k1 = q == 0 ? ka : (kb == 0 ? ka : (N - ka) % N);
          k2 = q == 0 ? kb : (kb == 0 ? N / 2 : N - kb);
        } else {
          const int P = q * T + t;
          k1 = P % N;
          k2 = P / N;
        }
#pragma unroll
        for (int j = 0; j < W; ++j) lds[(k2 * N + k1) * AB + j] = rest[q][(s - 1) * W + j];
      }
    }
    lds_barrier();
    cx<float> rb[N];
    // read in the order the transform consumes its inputs (first sub-transform first)
#pragma unroll
    for (int r = 0; r < N; ++r) {
      const int k2 = bzk::first_stage_order<N>(r);
      if (S == 2 && !LOSS && k2 == N / 2) rb[k2] = cx<float>{0.0f, 0.0f};  // see stage A
      else rb[k2] = lds[(k2 * N + tk) * AB + tj];
    }
    bzk::fft<N, 1>(rb);
    // B -> C inside the wave: the wave has read every slot of its planes, and
    // writes (j2, k1) to row (N+1) j2 + k1 of the same planes (an injective
    // map; the row's residue j2 + k1 mod 32 keeps the writes, lanes on k1,
    // and the reads below, lanes on j2, on distinct banks)
    if constexpr (wave_planes) wave_lds_sync();
    else lds_barrier();
#pragma unroll
    for (int j2 = 0; j2 < N; ++j2) lds[((N + 1) * j2 + tk) * AB + tj] = rb[j2];
    if constexpr (wave_planes) wave_lds_sync();
    else lds_barrier();
    cx<float> rc[N];
#pragma unroll
    for (int r = 0; r < N; ++r) {
      const int k1 = bzk::first_stage_order<N>(r);
      rc[k1] = lds[((N + 1) * tk + k1) * AB + tj];
    }
    bzk::fft<N, 1>(rc);
    if constexpr (LOSS) {
      // acc -= (sL f - Im) Re with the input f, read from the FP32 copy the
      // forward kernel wrote in this thread's order ([slice][j1][thread])
      const gptr<float> fp = opaque_global(fcc + size_t(s) * N * T + t);
#pragma unroll
      for (int j1 = 0; j1 < N; ++j1) acc[s][j1] -= (wp * fp[j1 * T] - rc[j1].y) * rc[j1].x;
    } else {
      // the direction's weight is in its multipliers (sqrt|w| on each part)
#pragma unroll
      for (int j1 = 0; j1 < N; ++j1) acc[s][j1] += rc[j1].x * rc[j1].y;
    }
  }
}

// N^2/S threads; S j3-slices of width W = N/S.
//   stage A: thread t owns pencils P = a*T + t (a < S) along k3 at
//            (k1, k2) = (P % N, P / N);
//   stage B: thread t owns, in every slice, the pencil along k2 at
//            (k1, j3) = (t % N, s*W + t / N);
//   stage C: thread t owns, in every slice, the pencil along k1 at
//            (j2, j3) = (t % N, s*W + t / N) and keeps its n products.
// LDS A->B: [k2][k1][j3 % W] padded to W+1 (odd stride: the stage-A writers
// and the stage-B readers step k1 on lanes).  B->C reuses the slots of the
// wave's own planes, (j2, k1) at row (N+1) j2 + k1 (N-1 rows beyond the A->B
// data): a wave synchronises only with itself between stages B and C.
// Register budget: the paired (S = 2) kernels need up to 256 VGPRs (2 waves
// per SIMD); N = 16 with one slice fits 4 waves per SIMD (128 VGPRs); N = 24
// (one slice, 576 threads, 120 KB of LDS) runs 9 waves per CU, 3 on one SIMD.
template <int N, int S>
constexpr int fused_min_waves() { return (N <= 16 && S == 1) ? 4 : (N == 24 ? 3 : 2); }

template <int N, int S, bool IMEX>
__global__ __launch_bounds__(N * N / S, (fused_min_waves<N, S>())) void k_collide_fused(FusedArgs a) {
  constexpr int W = N / S;
  constexpr int AB = W + 1;
  __shared__ cx<float> lds[(N * N + N - 1) * AB];
  // Workgroups are dealt round-robin over the 8 XCDs: blocks b and b + 8k
  // share an XCD, so the chunks of a cell are placed 8 blocks apart and read
  // its fhat through one L2.
  const int grp = blockIdx.x / (8 * a.chunks), rr = blockIdx.x % (8 * a.chunks);
  const int cell = grp * 8 + rr % 8;
  const int chunk = rr / 8;
  if (cell >= live_count(a.ncells, a.ncells_dev)) return;
  const int p0 = int((long(chunk) * a.m1) / a.chunks);
  const int p1 = int((long(chunk + 1) * a.m1) / a.chunks);
  const int t = threadIdx.x;
  const long row = a.idx ? long(a.idx[cell]) : long(cell);
  const cx<float>* fhc = a.fh + cell * a.fh_stride;
  float acc[S][N];
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int j = 0; j < N; ++j) acc[s][j] = 0.0f;
  const int gain_end = p1 < a.m1 - 1 ? p1 : a.m1 - 1;
  const float* fcc = a.fc + cell * a.fc_stride;
  for (int p = p0; p < gain_end; ++p) fused_pass<N, S, false>(a, lds, fhc, fcc, p, t, acc);
  if (p1 == a.m1) fused_pass<N, S, true>(a, lds, fhc, fcc, a.m1 - 1, t, acc);
  const int j2 = t % N, tl = t / N;  // this thread's stage-C (j2, j3 % W)
  if (a.fuse_project) {
    // Q = C acc; moments m = sum_j (1, v1, v2, v3, |v|^2) Q_j in FP64 with a
    // fixed reduction order (per thread, then across the wave, then across
    // the waves); lambda = (C C^T)^-1 m; q = Q - (l0 + l1 v1 + ... + l4 |v|^2).
    const double v2 = (j2 - N / 2) * a.dv;
    double m[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const double v3 = (s * W + tl - N / 2) * a.dv;
#pragma unroll
      for (int j1 = 0; j1 < N; ++j1) {
        const double v1 = (j1 - N / 2) * a.dv;
        const double qv = a.C * double(acc[s][j1]);
        m[0] += qv;
        m[1] += v1 * qv;
        m[2] += v2 * qv;
        m[3] += v3 * qv;
        m[4] += (v1 * v1 + v2 * v2 + v3 * v3) * qv;
      }
    }
#pragma unroll
    for (int k = 0; k < 5; ++k)
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) m[k] += __shfl_xor(m[k], o);
    constexpr int NW = (N * N / S) / 64;
    double* red = reinterpret_cast<double*>(lds);  // [k][wave] partials, then the 5 totals
    lds_barrier();  // the last pass's stage C has read the LDS
    if ((t & 63) == 0)
#pragma unroll
      for (int k = 0; k < 5; ++k) red[k * NW + t / 64] = m[k];
    lds_barrier();
    if (t < 5) {
      double x = 0.0;
      for (int wv = 0; wv < NW; ++wv) x += red[t * NW + wv];
      red[5 * NW + t] = x;
    }
    lds_barrier();
    double lam[5];
    {
      double tot[5];
#pragma unroll
      for (int k = 0; k < 5; ++k) tot[k] = red[5 * NW + k];
#pragma unroll
      for (int i = 0; i < 5; ++i) {
        double x = 0.0;
#pragma unroll
        for (int k = 0; k < 5; ++k) x += a.ginv[5 * i + k] * tot[k];
        lam[i] = x;
      }
    }
    const long orow = a.scatter ? row : long(cell);
    double* q = a.q + size_t(orow) * N * N * N;
    [[maybe_unused]] const double eps_c = IMEX ? (a.im.eps_cells ? a.im.eps_cells[row] : a.im.eps) : 0.0;
    // Each slice of projected Q goes through LDS ([j1][j2][j3 % W], pitch W + 1
    // doubles), then the workgroup sweeps it in memory order: the stores (and
    // the IMEX update's loads of f and v.grad f) cover whole rows of W
    // consecutive j3 instead of the 16-byte pieces of the stage-C ownership.
    constexpr int T = N * N / S;
    constexpr int SP = W + 1;
    static_assert(sizeof(double) * N * N * SP <= sizeof(cx<float>) * (N * N + N - 1) * AB, "a slice fits the LDS");
    double* st = reinterpret_cast<double*>(lds);
    bool bad = false;
    // IMEX: the two Maxwellians as per-axis Gaussian tables after the staging
    // area ([mw][axis][j], 6 N doubles; written before the first slice's
    // barrier, read after it)
    [[maybe_unused]] double* gt = st + N * N * SP;
    if constexpr (IMEX) {
      static_assert(sizeof(double) * (N * N * SP + 6 * N) <= sizeof(cx<float>) * (N * N + N - 1) * AB,
                    "the Gaussian tables fit beside a slice");
      const double* par = a.im.par + size_t(cell) * bzk::kImexPar;
      if (t < 6 * N) gt[t] = bzk::axis_gaussian(par, t / (3 * N), (t / N) % 3, t % N, N, a.dv);
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const double v3 = (s * W + tl - N / 2) * a.dv;
      lds_barrier();  // the LDS is free (reduction read, or the previous slice swept)
#pragma unroll
      for (int j1 = 0; j1 < N; ++j1) {
        const double v1 = (j1 - N / 2) * a.dv;
        const double corr = lam[0] + lam[1] * v1 + lam[2] * v2 + lam[3] * v3 + lam[4] * (v1 * v1 + v2 * v2 + v3 * v3);
        st[(j1 * N + j2) * SP + tl] = a.C * double(acc[s][j1]) - corr;
      }
      lds_barrier();
#pragma unroll 4
      for (int o = t; o < N * N * W; o += T) {
        const int jw = o % W, jj = o / W;  // jj = j1 * N + j2
        const size_t e = size_t(jj) * N + s * W + jw;
        double ov = st[jj * SP + jw];
        if constexpr (IMEX) {
          const size_t fe = size_t(row) * N * N * N + e;
          const double* par = a.im.par + size_t(cell) * bzk::kImexPar;
          const int j1 = jj / N, j2 = jj % N, j3 = s * W + jw;
          const double m0 = par[0] * gt[j1] * gt[N + j2] * gt[2 * N + j3];
          const double m1 = par[5] * gt[3 * N + j1] * gt[4 * N + j2] * gt[5 * N + j3];
          ov = bzk::imex_combine(par[10], ov, a.im.f[fe], a.im.tr[fe], eps_c, a.im.dt, m0, m1);
        }
        q[e] = ov;
        bad |= !isfinite(ov);
      }
    }
    flag_nonfinite(a.status, a.zero, bad);
    return;
  }
  float* out = a.acc + cell * a.acc_stride + size_t(chunk) * N * N * N;
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int j1 = 0; j1 < N; ++j1) out[size_t(j1) * N * N + size_t(j2) * N + s * W + tl] = acc[s][j1];
}

// ------------------------------------------------------------------ projection
struct ProjArgs {
  int ncells;
  const int32_t* ncells_dev;
  const int32_t* idx;
  int scatter;
  const void* acc;  // [cell][chunks][n^3] of float or double
  int acc_fp32;
  size_t acc_stride;  // elements per cell
  int chunks;
  double C, dv;
  double ginv[25];
  int project;  // 1: FP64 projection, FP64 output
  void* q;
  int q_fp32;   // output type when project == 0
  int imex;     // write the IMEX update of eq. (4.24) (FP64) instead of Q
  bzk::ImexDev im;
  int32_t* status;  // set to 1 when a non-finite value is written
  int zero;         // 0 at run time (per-lane store address)
};

__device__ __forceinline__ double load_acc(const ProjArgs& a, size_t i) {
  return a.acc_fp32 ? double(static_cast<const float*>(a.acc)[i]) : static_cast<const double*>(a.acc)[i];
}

constexpr int kProjThreads = 1024;
constexpr int kProjWaves = kProjThreads / 64;

// Sum of five per-thread FP64 values over the workgroup in a fixed order
// (across each wave, then wave by wave); every thread gets the totals.
// red holds 5 * (kProjWaves + 1) doubles.
__device__ __forceinline__ void proj_sum5(double (&m)[5], double* red) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
#pragma unroll
  for (int k = 0; k < 5; ++k)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m[k] += __shfl_xor(m[k], o);
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < 5; ++k) red[k * kProjWaves + wv] = m[k];
  __syncthreads();
  if (t < 5) {
    double x = red[t * kProjWaves];
    for (int w = 1; w < kProjWaves; ++w) x += red[t * kProjWaves + w];
    red[5 * kProjWaves + t] = x;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 5; ++k) m[k] = red[5 * kProjWaves + k];
}

__device__ __forceinline__ void proj_lambda(const ProjArgs& a, const double (&tot)[5], double (&lam)[5]) {
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    double x = 0.0;
#pragma unroll
    for (int k = 0; k < 5; ++k) x += a.ginv[5 * i + k] * tot[k];
    lam[i] = x;
  }
}

// One workgroup per cell.  qr_j = C * sum_chunks acc; moments m = C qr
// (1, v1, v2, v3, |v|^2) reduced in a fixed order; lambda = G^-1 m;
// q_j = qr_j - (l0 + l1 v1 + l2 v2 + l3 v3 + l4 |v|^2).
template <int N>
__global__ __launch_bounds__(kProjThreads) void k_project(ProjArgs a) {
  constexpr int N3 = N * N * N;
  const int c = blockIdx.x;
  if (c >= live_count(a.ncells, a.ncells_dev)) return;
  const size_t base = size_t(c) * a.acc_stride;
  const size_t row = a.scatter ? size_t(a.idx[c]) : size_t(c);
  const size_t frow = a.idx ? size_t(a.idx[c]) : size_t(c);  // row of the input f
  const int t = threadIdx.x;
  auto qraw = [&](int j) {
    double s = 0.0;
    for (int ch = 0; ch < a.chunks; ++ch) s += load_acc(a, base + size_t(ch) * N3 + j);
    return a.C * s;
  };
  const double eps_c = a.imex ? (a.im.eps_cells ? a.im.eps_cells[frow] : a.im.eps) : 0.0;
  // IMEX: the two Maxwellians as per-axis Gaussian tables [mw][axis][j]
  __shared__ double gt[6 * N];
  const double* par = a.im.par + size_t(c) * bzk::kImexPar;
  if (a.imex) {
    if (t < 6 * N) gt[t] = bzk::axis_gaussian(par, t / (3 * N), (t / N) % 3, t % N, N, a.dv);
    __syncthreads();
  }
  double lam[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (a.project) {
    __shared__ double red[5 * (kProjWaves + 1)];
    double m[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int j = t; j < N3; j += kProjThreads) {
      const double v1 = (j / (N * N) - N / 2) * a.dv, v2 = ((j / N) % N - N / 2) * a.dv, v3 = (j % N - N / 2) * a.dv;
      const double qv = qraw(j);
      m[0] += qv;
      m[1] += v1 * qv;
      m[2] += v2 * qv;
      m[3] += v3 * qv;
      m[4] += (v1 * v1 + v2 * v2 + v3 * v3) * qv;
    }
    proj_sum5(m, red);
    proj_lambda(a, m, lam);
  }
  bool bad = false;
#pragma unroll 4
  for (int j = t; j < N3; j += kProjThreads) {
    const double v1 = (j / (N * N) - N / 2) * a.dv, v2 = ((j / N) % N - N / 2) * a.dv, v3 = (j % N - N / 2) * a.dv;
    double v = qraw(j);
    if (a.project) v -= lam[0] + lam[1] * v1 + lam[2] * v2 + lam[3] * v3 + lam[4] * (v1 * v1 + v2 * v2 + v3 * v3);
    if (a.imex) {
      const size_t fe = frow * N3 + j;
      const int j1 = j / (N * N), j2 = (j / N) % N, j3 = j % N;
      const double m0 = par[0] * gt[j1] * gt[N + j2] * gt[2 * N + j3];
      const double m1 = par[5] * gt[3 * N + j1] * gt[4 * N + j2] * gt[5 * N + j3];
      v = bzk::imex_combine(par[10], v, a.im.f[fe], a.im.tr[fe], eps_c, a.im.dt, m0, m1);
    }
    if (a.imex || a.project || !a.q_fp32) static_cast<double*>(a.q)[row * N3 + j] = v;
    else static_cast<float*>(a.q)[row * N3 + j] = float(v);
    bad |= !isfinite(v);
  }
  flag_nonfinite(a.status, a.zero, bad);
}

// Projection of a plane-major accumulator acc[cell][j3][j1][j2] (one chunk,
// in the plan precision A, from the chunked plain passes).  Moments are summed in the
// accumulator's own order (fixed); the output [j1][j2][j3] is written through
// LDS tiles of 64 (j1, j2) columns so that both the reads and the writes are
// coalesced.
template <int N, typename A>
__global__ __launch_bounds__(kProjThreads) void k_project_pm(ProjArgs a) {
  constexpr int N2 = N * N, N3 = N2 * N, TC = 64;
  static_assert(N2 % TC == 0, "column tiles cover the plane");
  const int c = blockIdx.x;
  if (c >= live_count(a.ncells, a.ncells_dev)) return;
  const A* acc = static_cast<const A*>(a.acc) + size_t(c) * a.acc_stride;
  const size_t row = a.scatter ? size_t(a.idx[c]) : size_t(c);
  const size_t frow = a.idx ? size_t(a.idx[c]) : size_t(c);
  const int t = threadIdx.x;
  __shared__ double red[5 * (kProjWaves + 1)];
  __shared__ double tile[N][TC + 1];  // [j3][column]
  double lam[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (a.project) {
    double m[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int e = t; e < N3; e += kProjThreads) {
      const int j3 = e / N2, j1 = (e / N) % N, j2 = e % N;
      const double v1 = (j1 - N / 2) * a.dv, v2 = (j2 - N / 2) * a.dv, v3 = (j3 - N / 2) * a.dv;
      const double qv = a.C * double(acc[e]);
      m[0] += qv;
      m[1] += v1 * qv;
      m[2] += v2 * qv;
      m[3] += v3 * qv;
      m[4] += (v1 * v1 + v2 * v2 + v3 * v3) * qv;
    }
    proj_sum5(m, red);
    proj_lambda(a, m, lam);
  }
  const double eps_c = a.imex ? (a.im.eps_cells ? a.im.eps_cells[frow] : a.im.eps) : 0.0;
  // IMEX: the two Maxwellians as per-axis Gaussian tables [mw][axis][j]
  // (read after the first tile's barrier)
  __shared__ double gt[6 * N];
  const double* par = a.im.par + size_t(c) * bzk::kImexPar;
  if (a.imex && t < 6 * N) gt[t] = bzk::axis_gaussian(par, t / (3 * N), (t / N) % 3, t % N, N, a.dv);
  bool bad = false;
  for (int J0 = 0; J0 < N2; J0 += TC) {
    __syncthreads();  // the previous tile has been written out
    for (int i = t; i < N * TC; i += kProjThreads) {
      const int j3 = i / TC, jj = i % TC;
      tile[j3][jj] = a.C * double(acc[j3 * N2 + J0 + jj]);
    }
    __syncthreads();
    for (int i = t; i < TC * N; i += kProjThreads) {
      const int jj = i / N, j3 = i % N;
      const int J = J0 + jj;
      const int j1 = J / N, j2 = J % N;
      const size_t j = size_t(J) * N + j3;  // [j1][j2][j3]
      const double v1 = (j1 - N / 2) * a.dv, v2 = (j2 - N / 2) * a.dv, v3 = (j3 - N / 2) * a.dv;
      double qv = tile[j3][jj];
      if (a.project) qv -= lam[0] + lam[1] * v1 + lam[2] * v2 + lam[3] * v3 + lam[4] * (v1 * v1 + v2 * v2 + v3 * v3);
      if (a.imex) {
        const size_t fe = frow * N3 + j;
        const double m0 = par[0] * gt[j1] * gt[N + j2] * gt[2 * N + j3];
        const double m1 = par[5] * gt[3 * N + j1] * gt[4 * N + j2] * gt[5 * N + j3];
        qv = bzk::imex_combine(par[10], qv, a.im.f[fe], a.im.tr[fe], eps_c, a.im.dt, m0, m1);
      }
      if (a.imex || a.project || !a.q_fp32) static_cast<double*>(a.q)[row * N3 + j] = qv;
      else static_cast<float*>(a.q)[row * N3 + j] = float(qv);
      bad |= !isfinite(qv);
    }
  }
  flag_nonfinite(a.status, a.zero, bad);
}

// Launch the projection of a plan's accumulator (plane-major for the chunked
// plain passes); false for a grid size without an instantiation.
bool launch_project(int n, bool plane_major, const ProjArgs& pa, int ncells, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>(ncells)), block(kProjThreads);
  switch (n) {
    case 16:
      if (plane_major && pa.acc_fp32) hipLaunchKernelGGL((k_project_pm<16, float>), grid, block, 0, s, pa);
      else if (plane_major) hipLaunchKernelGGL((k_project_pm<16, double>), grid, block, 0, s, pa);
      else hipLaunchKernelGGL(k_project<16>, grid, block, 0, s, pa);
      return true;
    case 24:
      if (plane_major && pa.acc_fp32) hipLaunchKernelGGL((k_project_pm<24, float>), grid, block, 0, s, pa);
      else if (plane_major) hipLaunchKernelGGL((k_project_pm<24, double>), grid, block, 0, s, pa);
      else hipLaunchKernelGGL(k_project<24>, grid, block, 0, s, pa);
      return true;
    case 32:
      if (plane_major && pa.acc_fp32) hipLaunchKernelGGL((k_project_pm<32, float>), grid, block, 0, s, pa);
      else if (plane_major) hipLaunchKernelGGL((k_project_pm<32, double>), grid, block, 0, s, pa);
      else hipLaunchKernelGGL(k_project<32>, grid, block, 0, s, pa);
      return true;
    case 48:
      if (plane_major && pa.acc_fp32) hipLaunchKernelGGL((k_project_pm<48, float>), grid, block, 0, s, pa);
      else if (plane_major) hipLaunchKernelGGL((k_project_pm<48, double>), grid, block, 0, s, pa);
      else hipLaunchKernelGGL(k_project<48>, grid, block, 0, s, pa);
      return true;
    default:
      return false;
  }
}

// ------------------------------------------------------------------ launchers
template <typename T, int N>
void launch_plain_forward(const PlainArgs<T>& a, int ncells, hipStream_t s) {
  const long threads = long(ncells) * N * N;
  const dim3 grid(unsigned((threads + 255) / 256)), block(256);
  hipLaunchKernelGGL((k_fwd1<T, N>), grid, block, 0, s, a);
  hipLaunchKernelGGL((k_fwd2<T, N>), grid, block, 0, s, a);
  hipLaunchKernelGGL((k_fwd3<T, N>), grid, block, 0, s, a);
}

template <typename T, int N>
void launch_plain_dirs(PlainArgs<T> a, int ncells, int m1, hipStream_t s) {
  const long threads = long(ncells) * N * N;
  const dim3 grid(pa_xcd_order<T, N>() ? unsigned(8 * pa_xcd_share(threads / 256)) : unsigned((threads + 255) / 256)),
      block(256);
  constexpr int PW = plain_planes_per_group<N>();
  const dim3 grid_bc(unsigned(long(ncells) * (N / PW))), block_bc(unsigned(PW * N));
  a.m1 = m1;
  for (int p0 = 0; p0 < m1; p0 += a.chunk) {
    a.pass = p0;
    a.first = p0 == 0;
    hipLaunchKernelGGL((k_pA<T, N>), grid, block, 0, s, a);
    if constexpr (sizeof(T) == 4 && N % 16 == 0) {
      if (a.dft) {
        hipLaunchKernelGGL((k_pBC_mm<N>), grid_bc, block_bc, 0, s, a);
        continue;
      }
    }
    hipLaunchKernelGGL((k_pBC<T, N>), grid_bc, block_bc, 0, s, a);
  }
}

template <typename T>
bz_status run_plain(const bz_plan* p, const PlainArgs<T>& a, int ncells, hipStream_t s, bool fwd_only,
                    bool timed) {
  if (!fwd_only && (a.chunk < 1 || a.chunk > bz::kPlainChunkMax))
    return bz::fail(BZ_ERR_STATE, "plain path: %d directions per chunk", a.chunk);
  switch (p->n) {
    case 16:
      launch_plain_forward<T, 16>(a, ncells, s);
      if (timed) (void)hipEventRecord(const_cast<bz_plan*>(p)->ev[1], s);
      if (!fwd_only) launch_plain_dirs<T, 16>(a, ncells, p->m1, s);
      break;
    case 24:
      launch_plain_forward<T, 24>(a, ncells, s);
      if (timed) (void)hipEventRecord(const_cast<bz_plan*>(p)->ev[1], s);
      if (!fwd_only) launch_plain_dirs<T, 24>(a, ncells, p->m1, s);
      break;
    case 32:
      launch_plain_forward<T, 32>(a, ncells, s);
      if (timed) (void)hipEventRecord(const_cast<bz_plan*>(p)->ev[1], s);
      if (!fwd_only) launch_plain_dirs<T, 32>(a, ncells, p->m1, s);
      break;
    case 48:
      launch_plain_forward<T, 48>(a, ncells, s);
      if (timed) (void)hipEventRecord(const_cast<bz_plan*>(p)->ev[1], s);
      if (!fwd_only) launch_plain_dirs<T, 48>(a, ncells, p->m1, s);
      break;
    default:
      return bz::fail(BZ_ERR_UNSUPPORTED, "plain path: n=%d", p->n);
  }
  return BZ_OK;
}

template <int N, int S>
void launch_fwd_fused(const FwdArgs& a, int ncells, hipStream_t s) {
  hipLaunchKernelGGL((k_fwd_fused<N, S>), dim3(unsigned(ncells)), dim3(N * N / 2), 0, s, a);
}

template <int N, int S>
void launch_fused(const FusedArgs& a, int ncells, hipStream_t s) {
  const dim3 grid(unsigned((ncells + 7) / 8 * 8 * a.chunks)), block(N * N / S);
  if (a.imex) hipLaunchKernelGGL((k_collide_fused<N, S, true>), grid, block, 0, s, a);
  else hipLaunchKernelGGL((k_collide_fused<N, S, false>), grid, block, 0, s, a);
}

}  // namespace

template <typename T, int NI, int NO>
void launch_resample(PlainArgs<T> a, int ncells, hipStream_t s) {
  const long threads = long(ncells) * NO * NO;
  const dim3 grid(unsigned((threads + 255) / 256)), block(256);
  hipLaunchKernelGGL((k_rsA<T, NI, NO>), grid, block, 0, s, a);
  hipLaunchKernelGGL((k_dirB<T, NO>), grid, block, 0, s, a);
  hipLaunchKernelGGL((k_rsC<T, NO>), grid, block, 0, s, a);
}

// Dealiased plan: fhat at n; the truncated series on the padded grid; the
// padded operator's raw Q; its spectrum; back to the n modes; projection.
template <typename T, int N, int NP>
bz_status launch_dealiased(const bz_plan* p, const bz::Binding& b, const void* f, int f_fp32, const int32_t* idx,
                           int ncells, const int32_t* ncells_dev, void* q, int scatter, hipStream_t s, bool timed,
                           const bzk::ImexDev* imex) {
  bz_plan* pm = const_cast<bz_plan*>(p);
  char* ws = static_cast<char*>(b.ws);
  const bz::WsLayout& lay = b.lay;
  constexpr bool F32 = sizeof(T) == 4;
  if (timed) {
    pm->ev = &pm->evs[4 * (pm->timed_calls % bz_plan::kTimingSlots)];
    (void)hipEventRecord(pm->ev[0], s);
  }
  PlainArgs<T> a{};
  a.ncells = ncells;
  a.ncells_dev = ncells_dev;
  // 1. fhat at n (input rows idx[c])
  a.f = f;
  a.f_fp32 = f_fp32;
  a.idx = idx;
  a.fh = reinterpret_cast<cx<T>*>(ws + lay.fh_off);
  a.fh_stride = lay.fh_cell / sizeof(cx<T>);
  a.y = reinterpret_cast<cx<T>*>(ws + lay.y_off);
  a.y_stride = lay.y_cell / sizeof(cx<T>);
  launch_plain_forward<T, N>(a, ncells, s);
  // 2. the truncated series sampled on the padded grid
  a.acc = reinterpret_cast<T*>(ws + lay.fp_off);
  a.acc_stride = lay.fp_cell / sizeof(T);
  launch_resample<T, N, NP>(a, ncells, s);
  if (timed) (void)hipEventRecord(pm->ev[1], s);
  // 3. raw Q of the padded operator (compact cells)
  const bz::Binding pb = bz::make_binding(p->pad, b.tables, ws + lay.pad_off,
                                          p->pad->ws_fixed + size_t(b.capacity) * lay.pad_cell);
  bz_status st = bz::launch_collide(p->pad, pb, ws + lay.fp_off, F32 ? 1 : 0, nullptr, ncells, ncells_dev,
                                    ws + lay.qp_off, 0, s, false);
  if (st != BZ_OK) return st;
  // 4. its spectrum on the padded grid
  PlainArgs<T> c{};
  c.ncells = ncells;
  c.ncells_dev = ncells_dev;
  c.f = ws + lay.qp_off;
  c.f_fp32 = F32 ? 1 : 0;
  c.idx = nullptr;
  c.fh = reinterpret_cast<cx<T>*>(ws + lay.gp_off);
  c.fh_stride = lay.gp_cell / sizeof(cx<T>);
  c.y = reinterpret_cast<cx<T>*>(ws + lay.y_off);
  c.y_stride = lay.y_cell / sizeof(cx<T>);
  launch_plain_forward<T, NP>(c, ncells, s);
  // 5. back to the n modes: Q at the n grid in the accumulator region
  c.acc = reinterpret_cast<T*>(ws + lay.acc_off);
  c.acc_stride = lay.acc_cell / sizeof(T);
  launch_resample<T, NP, N>(c, ncells, s);
  if (timed) (void)hipEventRecord(pm->ev[2], s);
  // 6. projection / output (the padded Q already carries the kernel constant)
  ProjArgs pa{};
  pa.ncells = ncells;
  pa.ncells_dev = ncells_dev;
  pa.idx = idx;
  pa.scatter = scatter;
  pa.acc = ws + lay.acc_off;
  pa.acc_fp32 = F32 ? 1 : 0;
  pa.chunks = 1;
  pa.acc_stride = lay.acc_cell / sizeof(T);
  pa.C = 1.0;
  pa.dv = p->dv;
  for (int i = 0; i < 25; ++i) pa.ginv[i] = p->ginv[i];
  pa.project = p->project;
  pa.q = q;
  pa.q_fp32 = p->fp32;
  pa.status = reinterpret_cast<int32_t*>(ws + lay.status_off);
  if (imex) {
    pa.imex = 1;
    pa.im = *imex;
  }
  if (!launch_project(N, false, pa, ncells, s)) return bz::fail(BZ_ERR_UNSUPPORTED, "projection: n=%d", N);
  if (timed) {
    (void)hipEventRecord(pm->ev[3], s);
    pm->timed_calls += 1;
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return bz::fail(BZ_ERR_DEVICE, "bz_collide_batch: launch failed: %s", hipGetErrorString(e));
  return BZ_OK;
}

namespace bz {

void launch_clear_status(void* ws, const WsLayout& lay, hipStream_t s) {
  hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, s,
                     reinterpret_cast<int32_t*>(static_cast<char*>(ws) + lay.status_off), 0);
}

bool fused_supported(int n, int fp32) { return fp32 && (n == 16 || n == 24 || n == 32); }

bool dft_gemm_supported(int n, int fp32) { return fp32 && (n == 16 || n == 32 || n == 48); }

bool fused_slices_supported(int n, int slices) {
  return (n == 16 && (slices == 1 || slices == 2)) || (n == 24 && slices == 1) || (n == 32 && slices == 2);
}

// Direction chunks per cell when the descriptor leaves them open.  One
// workgroup per cell at n = 32 (143 KB of LDS: one per CU) fills the 256 CUs
// only from 256 cells up; plans for smaller batches split each cell's
// directions over two or four workgroups, as long as chunks x cells stays
// within 256 (32 cells 13.8 -> 7.4 us per cell, 128 cells 3.6 -> 2.9; at 160
// cells two chunks need a second round of workgroups and lose).  The n = 16
// kernels fit several workgroups per CU and gain up to 512 cells (64 cells
// 1.87 -> 0.82 us per cell with four, 512 cells 0.27 -> 0.23 with two).
int fused_default_chunks(int n, int max_cells) {
  if (n == 32 || n == 24) return max_cells <= 64 ? 4 : (max_cells <= 128 ? 2 : 1);
  if (n == 16) return max_cells <= 256 ? 4 : (max_cells <= 512 ? 2 : 1);
  return 1;
}

bz_status launch_collide(const bz_plan* p, const Binding& b, const void* f, int f_fp32,
                         const int32_t* idx, int ncells, const int32_t* ncells_dev, void* q,
                         int scatter, hipStream_t s, bool timed, const bzk::ImexDev* imex) {
  if (p->dim == 2) {
    if (imex) return fail(BZ_ERR_UNSUPPORTED, "IMEX update: three velocity dimensions only");
    return launch_collide2d(p, b, f, f_fp32, idx, ncells, ncells_dev, q, scatter, s, timed);
  }
  if (p->pad) {
    if (p->fp32)
      return p->n == 16 ? launch_dealiased<float, 16, 24>(p, b, f, f_fp32, idx, ncells, ncells_dev, q, scatter, s, timed, imex)
                        : launch_dealiased<float, 32, 48>(p, b, f, f_fp32, idx, ncells, ncells_dev, q, scatter, s, timed, imex);
    return p->n == 16 ? launch_dealiased<double, 16, 24>(p, b, f, f_fp32, idx, ncells, ncells_dev, q, scatter, s, timed, imex)
                      : launch_dealiased<double, 32, 48>(p, b, f, f_fp32, idx, ncells, ncells_dev, q, scatter, s, timed, imex);
  }
  bz_plan* pm = const_cast<bz_plan*>(p);
  char* ws = static_cast<char*>(b.ws);
  const WsLayout& lay = b.lay;
  const size_t n3 = size_t(p->n) * p->n * p->n;
  if (timed) {
    pm->ev = &pm->evs[4 * (pm->timed_calls % bz_plan::kTimingSlots)];
    (void)hipEventRecord(pm->ev[0], s);
  }
  ProjArgs pa{};
  pa.ncells = ncells;
  pa.ncells_dev = ncells_dev;
  pa.idx = idx;
  pa.scatter = scatter;
  pa.acc = ws + lay.acc_off;
  pa.acc_fp32 = p->fp32;
  pa.chunks = p->transform == BZ_XF_FUSED ? p->chunks : 1;
  pa.acc_stride = lay.acc_cell / (p->fp32 ? 4 : 8);
  pa.C = p->C;
  pa.dv = p->dv;
  for (int i = 0; i < 25; ++i) pa.ginv[i] = p->ginv[i];
  pa.project = p->project;
  pa.q = q;
  pa.q_fp32 = p->fp32;
  pa.status = reinterpret_cast<int32_t*>(ws + lay.status_off);
  if (imex) {
    pa.imex = 1;
    pa.im = *imex;
  }
  bz_status st = BZ_OK;
  bool fused_projection = false;
  if (p->fp32) {
    PlainArgs<float> a{};
    a.f = f;
    a.f_fp32 = f_fp32;
    a.idx = idx;
    a.ncells = ncells;
    a.ncells_dev = ncells_dev;
    a.fh = reinterpret_cast<cx<float>*>(ws + lay.fh_off);
    a.y = reinterpret_cast<cx<float>*>(ws + lay.y_off);
    a.acc = reinterpret_cast<float*>(ws + lay.acc_off);
    a.fh_stride = lay.fh_cell / sizeof(cx<float>);
    a.y_stride = lay.y_cell / sizeof(cx<float>);
    a.chunk = p->pchunk;
    a.acc_stride = lay.acc_cell / sizeof(float);
    a.mult = static_cast<const cx<float>*>(b.tables);
    a.w = reinterpret_cast<const float*>(static_cast<const char*>(b.tables) + p->table_w_off);
    if (p->transform == BZ_XF_DFT_GEMM)
      a.dft = reinterpret_cast<const float*>(static_cast<const char*>(b.tables) + p->table_dft_off);
    if (p->transform == BZ_XF_FUSED) {
      FwdArgs fw{};
      fw.ncells = ncells;
      fw.ncells_dev = ncells_dev;
      fw.f = f;
      fw.f_fp32 = f_fp32;
      fw.idx = idx;
      fw.fh = a.fh;
      fw.fh_stride = a.fh_stride;
      fw.mirror = p->slices == 1 ? 1 : 0;  // the one-slice kernels read every row
      fw.fc = reinterpret_cast<float*>(ws + lay.y_off);
      fw.fc_stride = lay.y_cell / sizeof(float);
      if (p->n == 32) launch_fwd_fused<32, 2>(fw, ncells, s);
      else if (p->n == 24) launch_fwd_fused<24, 1>(fw, ncells, s);
      else if (p->n == 16 && p->slices == 1) launch_fwd_fused<16, 1>(fw, ncells, s);
      else if (p->n == 16) launch_fwd_fused<16, 2>(fw, ncells, s);
      else return fail(BZ_ERR_UNSUPPORTED, "fused path: n=%d", p->n);
      if (timed) (void)hipEventRecord(pm->ev[1], s);
      FusedArgs fa{};
      fa.ncells = ncells;
      fa.ncells_dev = ncells_dev;
      fa.fc = fw.fc;
      fa.fc_stride = fw.fc_stride;
      fa.idx = idx;
      fa.fh = a.fh;
      fa.fh_stride = a.fh_stride;
      fa.acc = a.acc;
      fa.acc_stride = a.acc_stride;
      fa.mult = a.mult;
      fa.w = a.w;
      fa.m1 = p->m1;
      fa.chunks = p->chunks;
      fa.fuse_project = (p->chunks == 1 && p->project) ? 1 : 0;
      fa.scatter = scatter;
      fa.C = p->C;
      fa.dv = p->dv;
      for (int i = 0; i < 25; ++i) fa.ginv[i] = p->ginv[i];
      fa.q = static_cast<double*>(q);
      fa.status = reinterpret_cast<int32_t*>(ws + lay.status_off);
      if (imex && fa.fuse_project) {
        fa.imex = 1;
        fa.im = *imex;
      }
      fused_projection = fa.fuse_project != 0;
      if (p->n == 32) launch_fused<32, 2>(fa, ncells, s);
      else if (p->n == 24) launch_fused<24, 1>(fa, ncells, s);
      else if (p->n == 16 && p->slices == 1) launch_fused<16, 1>(fa, ncells, s);
      else if (p->n == 16) launch_fused<16, 2>(fa, ncells, s);
      else return fail(BZ_ERR_UNSUPPORTED, "fused path: n=%d", p->n);
    } else {
      st = run_plain<float>(p, a, ncells, s, false, timed);
    }
  } else {
    PlainArgs<double> a{};
    a.f = f;
    a.f_fp32 = f_fp32;
    a.idx = idx;
    a.ncells = ncells;
    a.ncells_dev = ncells_dev;
    a.fh = reinterpret_cast<cx<double>*>(ws + lay.fh_off);
    a.y = reinterpret_cast<cx<double>*>(ws + lay.y_off);
    a.acc = reinterpret_cast<double*>(ws + lay.acc_off);
    a.fh_stride = lay.fh_cell / sizeof(cx<double>);
    a.y_stride = lay.y_cell / sizeof(cx<double>);
    a.chunk = p->pchunk;
    a.acc_stride = lay.acc_cell / sizeof(double);
    a.mult = static_cast<const cx<double>*>(b.tables);
    a.w = reinterpret_cast<const double*>(static_cast<const char*>(b.tables) + p->table_w_off);
    st = run_plain<double>(p, a, ncells, s, false, timed);
  }
  if (st != BZ_OK) return st;
  if (timed) (void)hipEventRecord(pm->ev[2], s);
  if (!fused_projection && !launch_project(p->n, p->transform != BZ_XF_FUSED, pa, ncells, s))
    return fail(BZ_ERR_UNSUPPORTED, "projection: n=%d", p->n);
  if (timed) {
    (void)hipEventRecord(pm->ev[3], s);
    pm->timed_calls += 1;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(BZ_ERR_DEVICE, "bz_collide_batch: launch failed: %s", hipGetErrorString(e));
  (void)n3;
  return BZ_OK;
}

}  // namespace bz
